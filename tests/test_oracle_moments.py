"""Pins of the moment-equation oracle (oracle.moments) against closed forms,
analytic derivatives and the dense Fokker-Planck oracle."""
import numpy as np
import pytest

from oracle import dense, moments


def _grid(M):
    x = np.arange(M) / M
    return np.meshgrid(x, x, x, indexing="ij")


@pytest.mark.parametrize("M,k,gam,c", [(16, (1, 2, 3), 1e-2, (0.0, 0.0, 0.0)),
                                        (32, (3, 0, 5), 0.0, (0.7, -0.4, 1.3)),
                                        (32, (2, 7, 1), 5e-3, (-1.1, 0.2, 0.5))])
def test_fourier_mode_rk2(M, k, gam, c):
    """A Fourier mode of the periodic CFD2 operator with constant Gamma and
    constant velocity is an eigenvector: D1 -> i sin(theta)/h, D2 ->
    -4 sin^2(theta/2)/h^2, and one Heun step multiplies it by 1 + z + z^2/2."""
    h = 1.0 / M
    j = np.meshgrid(*(np.arange(M),) * 3, indexing="ij")
    th = [2 * np.pi * ki / M for ki in k]
    ph = sum(t * ji for t, ji in zip(th, j))
    m0 = np.cos(ph)
    U = [np.full((M, M, M), ci) for ci in c]
    G = np.full((M, M, M), gam)
    dt = 0.2 * h * h / max(gam, 1e-3) if gam > 0 else 0.2 * h
    z = dt * (gam * sum(-4 * np.sin(t / 2) ** 2 / h**2 for t in th)
              - 1j * sum(ci * np.sin(t) / h for ci, t in zip(c, th)))
    want = np.real((1 + z + z * z / 2) * np.exp(1j * ph))
    got = moments.step(m0, U, G, dt)
    assert np.max(np.abs(got - want)) < 1e-12


def _var_coeff_case(M):
    X1, X2, X3 = _grid(M)
    tp = 2 * np.pi
    G = 1.0 + 0.5 * np.sin(tp * X1) * np.cos(tp * X3)
    dG = [0.5 * tp * np.cos(tp * X1) * np.cos(tp * X3), 0.0 * X1,
          -0.5 * tp * np.sin(tp * X1) * np.sin(tp * X3)]
    m = np.sin(2 * tp * X1 + 0.2) * np.cos(tp * X2) + 0.3 * np.cos(tp * X3)
    dm = [2 * tp * np.cos(2 * tp * X1 + 0.2) * np.cos(tp * X2),
          -tp * np.sin(2 * tp * X1 + 0.2) * np.sin(tp * X2),
          -0.3 * tp * np.sin(tp * X3)]
    d2m = [-(2 * tp) ** 2 * np.sin(2 * tp * X1 + 0.2) * np.cos(tp * X2),
           -tp**2 * np.sin(2 * tp * X1 + 0.2) * np.cos(tp * X2),
           -0.3 * tp**2 * np.cos(tp * X3)]
    exact = sum(G * d2m[i] + dG[i] * dm[i] for i in range(3))  # d_i (G d_i m)
    return m, G, exact


def test_variable_diffusion_second_order():
    """div(G grad m) against its analytic value: the error falls by about 4
    per halving of h (a dropped grad G . grad m term would leave an O(1)
    error)."""
    errs = []
    for M in (16, 32, 64):
        m, G, exact = _var_coeff_case(M)
        zero = [np.zeros_like(m)] * 3
        errs.append(np.max(np.abs(moments.rhs(m, zero, G) - exact)) / np.max(np.abs(exact)))
    assert errs[0] < 0.2
    for a, b in zip(errs, errs[1:]):
        assert 3.5 < a / b < 4.5, errs


def _velocity_case(M):
    """A periodic divergence-free field: the Taylor-Green family of eq.
    velField (k = 4 pi, amplitudes 1, 1, -2) plus a shear that depends on x2,
    x3 only, with analytic gradients grad[i][j] = dU_i/dx_j."""
    X1, X2, X3 = _grid(M)
    k = 4 * np.pi
    S = [np.sin(k * X) for X in (X1, X2, X3)]
    C = [np.cos(k * X) for X in (X1, X2, X3)]
    tp = 2 * np.pi
    b = 0.6
    sh = b * np.sin(tp * X2 + 0.3) * np.cos(tp * X3)
    U = [C[0] * S[1] * S[2] + sh, S[0] * C[1] * S[2], -2 * S[0] * S[1] * C[2]]
    g = [[-k * S[0] * S[1] * S[2],
          k * C[0] * C[1] * S[2] + b * tp * np.cos(tp * X2 + 0.3) * np.cos(tp * X3),
          k * C[0] * S[1] * C[2] - b * tp * np.sin(tp * X2 + 0.3) * np.sin(tp * X3)],
         [k * C[0] * C[1] * S[2], -k * S[0] * S[1] * S[2], k * S[0] * C[1] * C[2]],
         [-2 * k * C[0] * S[1] * C[2], -2 * k * S[0] * C[1] * C[2], 2 * k * S[0] * S[1] * S[2]]]
    return U, g


def test_velocity_case_divergence_free():
    U, g = _velocity_case(8)
    assert np.max(np.abs(g[0][0] + g[1][1] + g[2][2])) < 1e-12


def test_smagorinsky_second_order():
    """gamma_SGS = C_s Delta^2 / 2 |S| against the analytic strain norm; the
    error falls by about 4 per halving of h."""
    c_s, gamma = 0.11, 1e-3
    errs = []
    for M in (32, 64, 128):
        U, g = _velocity_case(M)
        delta = 3.0 / M
        s = np.sqrt(sum((g[i][j] + g[j][i]) ** 2 for i in range(3) for j in range(3)))
        exact = gamma + c_s * delta**2 / 2 * s
        got = moments.gamma_total(U, gamma, c_s, delta)
        errs.append(np.max(np.abs(got - exact)) / np.max(exact - gamma))
    assert errs[0] < 0.1
    for a, b in zip(errs, errs[1:]):
        assert 3.3 < a / b < 4.5, errs


def test_omega_field_paper_range():
    """C_Omega = 1 at M = 128 with Delta = 3/M gives Omega_mix of order one to
    ten for eq. velField (the LMSE rate is gamma + gamma_SGS over Delta^2)."""
    M = 128
    x = np.arange(M) / M
    k = 4 * np.pi
    X1, X2, X3 = np.meshgrid(x, x, x, indexing="ij")
    jet = np.exp(-((X2 - 0.5) ** 2 + (X3 - 0.5) ** 2) / (2 * (1 / 6) ** 2))
    U = [np.cos(k * X1) * np.sin(k * X2) * np.sin(k * X3) - jet,
         np.sin(k * X1) * np.cos(k * X2) * np.sin(k * X3),
         -2 * np.sin(k * X1) * np.sin(k * X2) * np.cos(k * X3)]
    delta = 3.0 / M
    G = moments.gamma_total(U, 1e-3, 0.11, delta)
    om = moments.omega_field(G, 1.0, delta)
    assert np.min(om) >= 1e-3 / delta**2 * (1 - 1e-12)
    assert 1.0 < np.min(om) < np.max(om) < 10.0


def test_matches_dense_fokker_planck_moment():
    """With the composition-space terms switched off (Omega = nu = k = 0) the
    first composition moment of the dense Fokker-Planck solution obeys the
    moment equation exactly: the x operators act on every composition slice
    alike, so taking the moment commutes with them."""
    M = 8
    U, _ = _velocity_case(M)
    gam = 2e-3
    prob = dense.DenseProblem(5, M, 0.0, 0.0, 0.0, gam, U)
    rng = np.random.default_rng(7)
    f = rng.random((M,) * 5)
    dt = 1e-3
    G = np.full((M, M, M), gam)
    for a in (0, 1):
        m = prob.mean_field(f, a)[0, 0]
        g = f.copy()
        mm = m.copy()
        for _ in range(3):
            g = prob.step(g, dt, integrator="rk2")
            mm = moments.step(mm, U, G, dt)
        got = prob.mean_field(g, a)[0, 0]
        assert np.max(np.abs(got - mm)) < 1e-13 * np.max(np.abs(mm))


def test_error_measures_closed_forms():
    T = 17
    shape = (4, 4, 4)
    rng = np.random.default_rng(3)
    ex = rng.random((2, T) + shape)
    e = 0.03
    mean_x = ex + e
    c = 0.01
    mean_bar = np.stack([np.full(T, 0.5 + c), np.full(T, 0.5 - c)])
    norm_x = np.full((T,) + shape, 1.0 - 2e-4)
    up, dn, cu, cd = moments.error_measures(mean_bar, mean_x, ex, norm_x)
    assert abs(up - c) < 1e-15
    assert abs(dn - e) < 1e-14
    assert abs(cu - 2 * c) < 1e-15
    assert abs(cd - 2e-4) < 1e-15
    # a linear ramp over the 17 samples t = 0, T0/8, ..., 2 T0: the mean of
    # (k / 16)^2 over k = 0..16 is 1496 / (17 * 256) = 0.34375
    ramp = np.arange(T) / 16.0
    bar = np.stack([0.5 + ramp, 0.5 + 0 * ramp])
    _, _, cu, _ = moments.error_measures(bar, mean_x, None, norm_x)
    assert abs(cu * cu - 0.34375) < 1e-15


def test_matches_dense_fokker_planck_moment_variable_diffusivity():
    """The same commutation with a variable diffusivity field G(x) in the
    expanded form used by both solvers."""
    M = 8
    U, _ = _velocity_case(M)
    X1, X2, X3 = _grid(M)
    G = 2e-3 * (1.0 + 0.5 * np.sin(2 * np.pi * X1) * np.cos(2 * np.pi * X3 + 0.4))
    prob = dense.DenseProblem(5, M, 0.0, 0.0, 0.0, 0.0, U, G=G)
    f = np.random.default_rng(8).random((M,) * 5)
    dt = 1e-3
    for a in (0, 1):
        mm = prob.mean_field(f, a)[0, 0]
        g = f.copy()
        for _ in range(3):
            g = prob.step(g, dt, integrator="rk2")
            mm = moments.step(mm, U, G, dt)
        got = prob.mean_field(g, a)[0, 0]
        assert np.max(np.abs(got - mm)) < 1e-13 * np.max(np.abs(mm))


def test_step_at_points_equals_step():
    """The point-by-point Heun step reproduces the whole-grid step."""
    M = 16
    U, _ = _velocity_case(M)
    X1, X2, X3 = _grid(M)
    G = 1e-2 * (1.0 + 0.5 * np.sin(2 * np.pi * X1) * np.cos(2 * np.pi * X3))
    m = np.random.default_rng(2).random((M, M, M))
    dt = 1e-4
    pts = np.random.default_rng(3).integers(0, M, size=(40, 3))
    pts[0] = (0, 0, 0)
    pts[1] = (M - 1, M - 1, M - 1)
    want = moments.step(m, U, G, dt)[tuple(pts.T)]
    got = moments.step_at(m, U, G, dt, pts)
    assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(want))
