"""Pins of the full-grid oracle (oracle.dense) against the paper and closed forms."""
import numpy as np
import pytest

import workloads
from oracle import dense


def _ghost_apply(g, order):
    """Central differences with ghost points taken literally from eq. compBCs'
    stated consequences: f_{-1} = -f_0, f_M = -f_{M-1} (first derivative),
    f_{-1} = f_0, f_M = f_{M-1} (second derivative)."""
    M = g.size
    h = 1.0 / M
    sign = -1.0 if order == 1 else 1.0
    p = np.concatenate([[sign * g[0]], g, [sign * g[-1]]])
    if order == 1:
        return (p[2:] - p[:-2]) / (2 * h)
    return (p[2:] - 2 * p[1:-1] + p[:-2]) / h**2


@pytest.mark.parametrize("M", [8, 64, 128])
def test_ghost_rules(M):
    g = np.random.default_rng(M).standard_normal(M)
    assert np.allclose(dense.d1_ghost(M) @ g, _ghost_apply(g, 1), rtol=0, atol=1e-12 * M)
    assert np.allclose(dense.d2_ghost(M) @ g, _ghost_apply(g, 2), rtol=0, atol=1e-12 * M * M)


@pytest.mark.parametrize("M", [8, 128])
def test_compbcs_sums_vanish(M):
    """eq. compBCs: the grid sum of every discrete composition derivative is zero."""
    g = np.random.default_rng(1).random(M)
    for D in (dense.d1_ghost(M), dense.d2_ghost(M), dense.d1_periodic(M), dense.d2_periodic(M)):
        assert abs(np.sum(D @ g)) < 1e-12 * np.abs(D).max() * M


def test_discrete_moment_identities():
    """D1g^T phi = (-1/2, -1, ..., -1, -1/2) and h D2g^T phi = e_0 - e_{M-1}
    (cell-centred nodes): the mean is moved only by boundary terms."""
    M = 128
    h = 1.0 / M
    phi = dense.phi_nodes(M)
    d1 = dense.d1_ghost(M).T @ phi
    ref = -np.ones(M)
    ref[0] = ref[-1] = -0.5
    assert np.allclose(d1, ref, atol=1e-11)
    d2 = h * dense.d2_ghost(M).T @ phi
    ref2 = np.zeros(M)
    ref2[0], ref2[-1] = 1.0, -1.0
    assert np.allclose(d2, ref2, atol=1e-9)


def test_ou_moments_2d_mixing():
    """2-D LMSE mixing + dissipation is an Ornstein-Uhlenbeck process in
    composition space: the means stay fixed, each variance relaxes as
    var(t) = nu/Omega + (var0 - nu/Omega) e^{-2 Omega t} and the covariance as
    cov0 e^{-2 Omega t}.  The CFD2 stencils reproduce these moment laws
    exactly in the interior, so with negligible boundary mass the discrete
    solution must follow them (C1 geometry, 100 RK4 steps)."""
    w = workloads.get_workload("c1_2d_M64")
    M = w.M
    f = dense.dense_from_terms(workloads.ic_terms(w), 2, M)
    P = dense.DenseProblem(2, M, w.omega, 0.0, w.nu_phi)
    h = 1.0 / M
    p1, p2 = P.phi

    def moments(f):
        m1 = h * h * np.sum(p1 * f)
        m2 = h * h * np.sum(p2 * f)
        v1 = h * h * np.sum((p1 - m1) ** 2 * f)
        v2 = h * h * np.sum((p2 - m2) ** 2 * f)
        c = h * h * np.sum((p1 - m1) * (p2 - m2) * f)
        return m1, m2, v1, v2, c

    m1, m2, v1, v2, c0 = moments(f)
    n = 100
    for _ in range(n):
        f = P.step(f, w.dt, "rk4")
    t = n * w.dt
    e = np.exp(-2 * w.omega * t)
    vinf = w.nu_phi / w.omega
    M1, M2, V1, V2, C = moments(f)
    assert abs(h * h * np.sum(f) - 1.0) < 1e-13
    assert abs(M1 - m1) < 1e-9 and abs(M2 - m2) < 1e-9
    assert abs(V1 - (vinf + (v1 - vinf) * e)) < 1e-9
    assert abs(V2 - (vinf + (v2 - vinf) * e)) < 1e-9
    assert abs(C - c0 * e) < 1e-9


def test_fourier_mode_x_rk4():
    """A Fourier mode is an eigenvector of the periodic CFD2 convection-
    diffusion operator with symbol lambda = -i U sin(k h)/h - 4 Gamma sin^2(k h/2)/h^2;
    RK4 multiplies it by R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24, z = dt lambda."""
    M = 16
    x = workloads.x_points(M)
    U0, Gam, dt, q = 0.7, 3e-3, 1e-2, 3
    kap = 2 * np.pi * q
    zero = np.zeros((M, M, M))
    U = [zero + U0, zero, zero]
    P = dense.DenseProblem(5, M, omega=0.0, k_react=0.0, nu_phi=0.0, gamma=Gam, U=U)
    phipart = np.random.default_rng(2).random((M, M))
    e0 = np.exp(1j * (kap * x + 0.3))
    f = np.einsum("ab,c->abc", phipart, e0.real)[..., None, None] * np.ones((1, 1, 1, M, M))
    h = 1.0 / M
    lam = -1j * U0 * np.sin(kap * h) / h - 4 * Gam * np.sin(kap * h / 2) ** 2 / h**2
    z = dt * lam
    R = 1 + z + z**2 / 2 + z**3 / 6 + z**4 / 24
    n = 7
    for _ in range(n):
        f = P.step(f, dt, "rk4")
    ref = np.einsum("ab,c->abc", phipart, (R**n * e0).real)[..., None, None] * np.ones((1, 1, 1, M, M))
    assert np.max(np.abs(f - ref)) < 1e-13 * np.max(np.abs(ref)) * 10


def _paper_5d(k_react):
    w = workloads.get_workload("t_5d_M8_exact", ic="paper", k_react=k_react)
    from oracle.stepper import MPSStepper  # velocity field as the MPS side builds it
    U = MPSStepper(w).velocity_dense()
    P = dense.DenseProblem(5, w.M, w.omega, w.k_react, w.nu_phi, w.gamma, U)
    f = dense.dense_from_terms(workloads.ic_terms(w), 5, w.M)
    return w, P, f


@pytest.mark.parametrize("k_react", [0.0, 10.0])
def test_paper_invariants_5d(k_react):
    """<1>(x) = 1 at every x and t; avg<Phi1> - avg<Phi2> = 0 for all t by the
    symmetry of S_a and of the initial condition; avg<Phi_a> = 1/2 at Da = 0."""
    w, P, f = _paper_5d(k_react)
    for _ in range(5):
        f = P.step(f, w.dt, "rk4")
    assert np.max(np.abs(P.norm_field(f) - 1.0)) < 1e-13
    obs = P.observables(f)
    assert abs(obs["mean1"] - obs["mean2"]) < 1e-14
    if k_react == 0.0:
        assert abs(obs["mean1"] - 0.5) < 1e-13
    else:
        assert obs["mean1"] < 0.5 - 1e-4  # consumption


def test_reaction_moment_identity():
    """With Omega = nu = 0 the reaction alone moves the mean by
    d<Phi_a>/dt = k h^2 sum_i d_{i_a} phi1 phi2 f, d = D1g^T phi = (-1/2, -1, ..., -1/2):
    both species are consumed at the rate of the bilinear source."""
    M, k = 32, 7.0
    P = dense.DenseProblem(2, M, omega=0.0, k_react=k, nu_phi=0.0)
    f = np.random.default_rng(3).random((M, M))
    r = P.rhs(f)
    h = 1.0 / M
    p1, p2 = P.phi
    d = -np.ones(M)
    d[0] = d[-1] = -0.5
    for a in (0, 1):
        dm = h * h * np.sum(P.phi[a] * r)
        da = d.reshape((M, 1)) if a == 0 else d.reshape((1, M))
        ref = k * h * h * np.sum(da * p1 * p2 * f)
        assert abs(dm - ref) < 1e-12 * abs(ref)
        assert dm < 0


def test_separability_at_zero_mixing():
    """Supplementary Text: with C_Omega = 0 (and no reaction) the equation is
    separable between the compositions and x, so a product initial PDF stays a
    product: the unfoldings phi1 | rest and (phi1 phi2) | x keep rank one."""
    w = workloads.get_workload("t_5d_M8_exact", omega=0.0, k_react=0.0)
    from oracle.stepper import MPSStepper
    U = MPSStepper(w).velocity_dense()
    M = w.M
    P = dense.DenseProblem(5, M, 0.0, 0.0, w.nu_phi, w.gamma, U)
    g = workloads.ic_terms(w)[0][1]
    f = dense.dense_from_terms([(1.0, g)], 5, M)
    for _ in range(5):
        f = P.step(f, w.dt, "rk4")
    for cut in (M, M * M):
        s = np.linalg.svd(f.reshape(cut, -1), compute_uv=False)
        assert s[1] < 1e-12 * s[0]


def _dense_case(name):
    from oracle import stepper
    w = workloads.get_workload(name)
    P = stepper.MPSStepper(w).dense_problem()
    f0 = dense.dense_from_terms(workloads.ic_terms(w), w.ndims, w.M)
    return w, P, f0


@pytest.mark.parametrize("name", ["t_5d_M8_chi16", "t_2d_M64_serial"])
@pytest.mark.parametrize("param", ["omega", "k_react"])
def test_tangent_matches_central_differences(name, param):
    """The tangent-linear step (derivative of the discrete RK4 map with respect
    to Omega or k, mean-field dependence included) against central finite
    differences of the step itself, over three steps."""
    w, P, f0 = _dense_case(name)
    theta = getattr(P, param)
    h = 1e-4 * max(1.0, abs(theta))
    f, df = f0.copy(), np.zeros_like(f0)
    fp, fm = f0.copy(), f0.copy()
    Pp, Pm = P.with_params(**{param: theta + h}), P.with_params(**{param: theta - h})
    for _ in range(3):
        f, df = P.step_tangent(f, df, w.dt, param, w.integrator)
        fp, fm = Pp.step(fp, w.dt, w.integrator), Pm.step(fm, w.dt, w.integrator)
    fd = (fp - fm) / (2 * h)
    assert np.linalg.norm(df - fd) <= 1e-6 * np.linalg.norm(fd), np.linalg.norm(df - fd) / np.linalg.norm(fd)
    # the derivative of the (linear) product statistic is that statistic of df
    jp, jm = P.observables(fp)["product"], P.observables(fm)["product"]
    assert abs(P.observables(df)["product"] - (jp - jm) / (2 * h)) <= 1e-6 * max(1e-12, abs(jp - jm) / (2 * h)) + 1e-12


def test_tangent_state_direction():
    """Along a state direction v (no parameter), the tangent step is the
    derivative d/ds step(f + s v); the mean field's own dependence on f (the
    term m_a(v) f) is essential here."""
    w, P, f0 = _dense_case("t_5d_M8_chi16")
    v = np.random.default_rng(11).standard_normal(f0.shape) * np.abs(f0).max()
    _, dv = P.step_tangent(f0, v, w.dt, None, w.integrator)
    s = 1e-4
    fd = (P.step(f0 + s * v, w.dt) - P.step(f0 - s * v, w.dt)) / (2 * s)
    assert np.linalg.norm(dv - fd) <= 1e-8 * np.linalg.norm(fd)
