"""Flow-case kernels and protocol (HIP library through the C ABI) against the
oracle: the Smagorinsky field, the moment equation, dense evaluation of
MPSs, composition moments as x-fields, squared-difference sums and the
error measures of eq. RMSE0, and a short end-to-end run of the protocol.

Tolerances: the dense stencil kernels and reductions are the oracle's
arithmetic in another summation order, so they agree to 1e-12 relative;
the end-to-end run inherits the truncated-rounding agreement of the MPS
steps (about 1e-9 relative on these sizes, see test_gpu_parity), which
bounds the error measures' difference by about 1e-8 absolute.
"""
import numpy as np
import pytest

import workloads
from oracle import dense as odense, moments, stepper, tt
from oracle.dense import dense_from_terms
from tests import cases
from tests.helpers import TRUNC_TOL_F64, random_tt

q = pytest.importorskip("paper_2407_09169_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = q.Context(0)
    yield c
    c.close()


def _cuda(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _paper_velocity(M):
    """eq. velField on the M^3 grid (x1, x2, x3), from the seeded-input module."""
    w = workloads.get_workload("t_5d_M8_chi16", bits=int(np.log2(M)), ic="paper")
    U = []
    for comp in workloads.velocity_terms(w):
        u = np.zeros((M, M, M))
        for c, (v1, v2, v3) in comp:
            ones = np.ones(M)
            v1 = ones if v1 is None else v1
            v2 = ones if v2 is None else v2
            v3 = ones if v3 is None else v3
            u += c * np.einsum("i,j,k->ijk", v1, v2, v3)
        U.append(u)
    return U


def _close(got, want, rtol):
    scale = max(np.max(np.abs(want)), 1e-300)
    assert np.max(np.abs(got - want)) <= rtol * scale, np.max(np.abs(got - want)) / scale


@pytest.mark.parametrize("bits", [3, 5, 6])
def test_smagorinsky_matches_oracle(ctx, bits):
    M = 1 << bits
    U = _paper_velocity(M)
    delta = 3.0 / M
    want = moments.gamma_total(U, 1e-3, 0.11, delta)
    import torch
    Ud = _cuda(np.concatenate([u.ravel() for u in U]))
    G = torch.empty(M ** 3, dtype=torch.float64, device="cuda")
    q.smagorinsky(ctx, bits, Ud, G, 0.11, delta, 1e-3)
    _close(G.cpu().numpy().reshape(M, M, M), want, 1e-12)


@pytest.mark.parametrize("bits,count,steps", [(3, 1, 3), (4, 2, 5), (5, 2, 8), (6, 2, 3), (7, 1, 2)])
def test_moment_steps_match_oracle(ctx, bits, count, steps):
    """Smagorinsky diffusivity (strengthened so that the variable-coefficient
    term matters), eq. velField, seeded random initial means."""
    import torch
    M = 1 << bits
    U = _paper_velocity(M)
    delta = 3.0 / M
    c_s = 2.0
    G = moments.gamma_total(U, 1e-3, c_s, delta)
    assert np.max(G) > 3 * np.min(G)
    rng = np.random.default_rng([bits, count])
    m0 = rng.random((count, M, M, M))
    dt = 0.2 / (M * M * np.max(G) * 6 + M * 4)
    want = m0.copy()
    for k in range(steps):
        want = np.stack([moments.step(want[a], U, G, dt) for a in range(count)])
    Ud = _cuda(np.concatenate([u.ravel() for u in U]))
    Gd = torch.empty(M ** 3, dtype=torch.float64, device="cuda")
    q.smagorinsky(ctx, bits, Ud, Gd, c_s, delta, 1e-3)
    m = _cuda(m0.ravel())
    work = torch.empty_like(m)
    q.moment_steps(ctx, bits, Ud, Gd, m, work, dt, steps)
    _close(m.cpu().numpy().reshape(count, M, M, M), want, 1e-12)
    # the solution moved away from the start
    assert np.max(np.abs(want - m0)) > 1e-3


@pytest.mark.parametrize("ranks", [[1, 2, 1], [1, 2, 4, 8, 5, 3, 2, 1],
                                   [1] + [2, 4, 8] + [8] * 9 + [8, 4, 2] + [1],
                                   [1] + [2, 4, 8, 16] + [16] * 12 + [16, 8, 4, 2] + [1]])
def test_to_dense_matches_oracle(ctx, ranks):
    import torch
    cores = random_tt(ranks, seed=len(ranks))
    want = tt.tt_full(cores).ravel()
    x = q.TT.from_cores(ctx, cores)
    out = torch.empty(want.size, dtype=torch.float64, device="cuda")
    q.to_dense(ctx, x, out)
    _close(out.cpu().numpy(), want, 1e-12)


def test_moment_field_matches_oracle(ctx):
    w = workloads.get_workload("t_5d_M8_chi16")
    st = stepper.MPSStepper(w)
    f_or = st.initial_state()
    F = st.to_dense(f_or)  # (phi1, phi2, x1, x2, x3)
    M = w.M
    h = 1.0 / M
    phi = odense.phi_nodes(M)
    prob, f = q.setup_workload(ctx, w)
    import torch
    out = torch.empty(M ** 3, dtype=torch.float64, device="cuda")
    for w1, w2 in ((phi, None), (None, phi), (None, None), (phi, phi)):
        a1 = np.ones(M) if w1 is None else w1
        a2 = np.ones(M) if w2 is None else w2
        want = h * h * np.einsum("i,j,ijabc->abc", a1, a2, F)
        x = prob.moment_field(f, w1, w2)
        q.to_dense(ctx, x, out)
        x.free()
        # the two sides build the truncated initial state independently
        _close(out.cpu().numpy().reshape(M, M, M), want, 1e-8)
    f.free()
    prob.close()


@pytest.mark.parametrize("n,with_b,c", [(1, False, 0.0), (255, True, 0.0), (12345, True, 0.5),
                                        (1 << 21, False, 1.0), ((1 << 22) + 77, True, -0.25)])
def test_sq_diff_sum(ctx, n, with_b, c):
    rng = np.random.default_rng(n)
    a = rng.standard_normal(n)
    b = rng.standard_normal(n) if with_b else None
    want = float(np.sum((a - (b if with_b else 0.0) - c) ** 2))
    got = q.sq_diff_sum(ctx, _cuda(a), None if b is None else _cuda(b), c)
    assert abs(got - want) <= 1e-12 * want


def test_error_measures_match_oracle():
    T = 17
    rng = np.random.default_rng(11)
    shape = (4, 4, 4)
    mean_bar = 0.5 + 0.01 * rng.standard_normal((2, T))
    ex = rng.random((2, T) + shape)
    mx = ex + 0.001 * rng.standard_normal((2, T) + shape)
    nx = 1.0 + 1e-3 * rng.standard_normal((T,) + shape)
    want = moments.error_measures(mean_bar, mx, ex, nx)
    sq_mean = np.mean((mx - ex) ** 2, axis=(2, 3, 4))
    sq_norm = np.mean((nx - 1.0) ** 2, axis=(1, 2, 3))
    got = q.error_measures(mean_bar, sq_mean, sq_norm)
    assert np.allclose(got, want, rtol=1e-13, atol=0)
    got = q.error_measures(mean_bar, None, sq_norm)
    assert np.isnan(got[1]) and np.allclose([got[0], got[2], got[3]],
                                            [want[0], want[2], want[3]], rtol=1e-13)


def _oracle_fields(w, fields, chi_field, c_omega=1.0):
    """The oracle stepper and the dense diffusivity of the moment equation for
    the protocol's three settings: constant coefficients (fields None), the
    seeded x-fields G(x), Omega(x) (fields True), or the paper's closure
    (fields "smagorinsky": gamma + gamma_SGS from the velocity on the grid,
    Delta = 3 / M, cut to chi_field by the oracle's TT-SVD, and Omega_mix =
    c_omega G / Delta^2 of the cut field)."""
    M = w.M
    if not fields:
        return stepper.MPSStepper(w), np.full((M, M, M), w.gamma)
    if fields is True:
        st = _field_stepper(w)
        return st, st.dense_problem().G
    assert fields == "smagorinsky"
    st0 = stepper.MPSStepper(w)
    xo = st0._x_order()
    delta = 3.0 / M
    Gd = moments.gamma_total(st0.velocity_dense(), w.gamma, 0.11, delta)
    g = tt.tt_svd(tt.dense_to_sites(Gd, xo, w.bits), rel_tol=0.0, chi=chi_field)
    om = [G.copy() for G in g]
    om[0] = om[0] * (c_omega / (delta * delta))
    st = stepper.MPSStepper(w, {"G": g, "Omega": om})
    return st, tt.sites_to_dense(tt.tt_full(g), xo, w.bits, 3)


def _oracle_flow(w, T, k, fields=None, chi_field=None):
    st, G = _oracle_fields(w, fields, chi_field)
    f = st.initial_state()
    M, h = w.M, 1.0 / w.M
    phi = odense.phi_nodes(M)
    U = st.velocity_dense()
    F = st.to_dense(f)
    m = [h * h * np.einsum("i,iabc->abc", phi, F.sum(axis=1)),
         h * h * np.einsum("j,jabc->abc", phi, F.sum(axis=0))]
    bar, mx, ex, nx = np.zeros((2, T)), [[], []], [[], []], []
    for t in range(T):
        if t > 0:
            for _ in range(k):
                f, _ = st.step(f)
                m = [moments.step(m[a], U, G, w.dt) for a in range(2)]
        F = st.to_dense(f)
        obs = st.observables(f)
        bar[0, t], bar[1, t] = obs["mean1"], obs["mean2"]
        nx.append(h * h * F.sum(axis=(0, 1)))
        mx[0].append(h * h * np.einsum("i,iabc->abc", phi, F.sum(axis=1)))
        mx[1].append(h * h * np.einsum("j,jabc->abc", phi, F.sum(axis=0)))
        ex[0].append(m[0])
        ex[1].append(m[1])
    return moments.error_measures(bar, np.array(mx), np.array(ex), np.array(nx))


def test_flow_protocol_matches_oracle(ctx):
    """A short run of the protocol at Da = 0 (RK2, 5 samples, 2 steps apart)."""
    from paper_2407_09169_amd import flow
    w = workloads.get_workload("t_5d_M8_chi16", k_react=0.0, integrator="rk2")
    T, k = 5, 2
    want = _oracle_flow(w, T, k)
    got = flow.run(ctx, w, n_samples=T, steps_per_sample=k)
    vals = [got["E2b_up"], got["E2b_down"], got["E2c_up"], got["E2c_down"]]
    assert all(np.isfinite(vals))
    assert vals[1] > 0.0
    assert np.allclose(vals, want, rtol=1e-6, atol=1e-8), (vals, want)


def _field_stepper(w):
    st0 = stepper.MPSStepper(w)
    xo = st0._x_order()
    fields = {k: st0._separable(terms, xo, 3) for k, terms in workloads.flow_field_terms(w).items()}
    return stepper.MPSStepper(w, fields)


@pytest.mark.parametrize("integrator", ["rk2", "rk4"])
def test_field_step_untruncated_equals_dense(ctx, integrator):
    """Variable G(x) and Omega(x) at exact ranks: the GPU step reproduces the
    full-grid solver with the same fields."""
    w = workloads.get_workload("t_5d_M8_exact", integrator=integrator)
    st = _field_stepper(w)
    P = st.dense_problem()
    prob, f = q.setup_workload(ctx, w, "f64", fields=True)
    fd = dense_from_terms(workloads.ic_terms(w), w.ndims, w.M)
    for _ in range(3):
        prob.step(f, 1)
        fd = P.step(fd, w.dt, integrator)
        err = np.linalg.norm(st.to_dense(f.cores()) - fd) / np.linalg.norm(fd)
        assert err < 1e-11, err
    prob.close()


@pytest.mark.parametrize("name,integrator,steps", [(n, i, k) for n, i, k, fl in cases.STEP_CASES if fl])
def test_field_step_truncated_matches_oracle(ctx, name, integrator, steps):
    """Truncated FP64 steps with the x-fields, to the same bound as the
    constant-coefficient steps (TRUNC_TOL_F64)."""
    w = workloads.get_workload(name, integrator=integrator)
    st = _field_stepper(w)
    prob, f = q.setup_workload(ctx, w, "f64", fields=True)
    fo = st.initial_state()
    tol = TRUNC_TOL_F64
    for i in range(steps):
        prob.step(f, 1)
        fo, _ = st.step(fo)
        err = np.linalg.norm(st.to_dense(f.cores()) - st.to_dense(fo)) / np.linalg.norm(st.to_dense(fo))
        assert err < tol, (name, i, err, tol)
    with pytest.raises(q.QttError):
        prob.step_tangent(f, {"omega": prob.state()}, 1)
    prob.close()


@pytest.mark.parametrize("fields,chi_field", [(True, None), ("smagorinsky", 8)])
def test_flow_protocol_with_fields_matches_oracle(ctx, fields, chi_field):
    """The protocol with G(x) and Omega(x), the seeded fields or the paper's
    closure (Smagorinsky field cut to a bond cap of 8, Omega = G / Delta^2),
    against the oracle's run of the same protocol (field stepper and the
    moment equation with the same dense G), to the tolerance of the
    constant-coefficient run."""
    from paper_2407_09169_amd import flow
    w = workloads.get_workload("t_5d_M8_chi16", k_react=0.0, integrator="rk2", ic="paper")
    T, k = 5, 2
    want = _oracle_flow(w, T, k, fields, chi_field)
    got = flow.run(ctx, w, n_samples=T, steps_per_sample=k, fields=fields,
                   chi_field=chi_field if chi_field else 16)
    vals = [got["E2b_up"], got["E2b_down"], got["E2c_up"], got["E2c_down"]]
    assert all(np.isfinite(vals)), vals
    assert vals[1] > 0.0
    if fields == "smagorinsky":
        assert got["field_discarded"] > 0.0  # the cap truncates the closure field
    assert np.allclose(vals, want, rtol=1e-6, atol=1e-8), (vals, want)


def test_flow_protocol_with_fields_runs(ctx):
    """The protocol with G(x) and Omega(x) on the 16^5 grid: finite measures,
    the mass-norm error at the truncation level, and the exact-mean error
    above zero."""
    from paper_2407_09169_amd import flow
    w = workloads.get_workload("t_5d_M16_chi32", k_react=0.0, integrator="rk2")
    got = flow.run(ctx, w, n_samples=5, steps_per_sample=2, fields=True)
    vals = [got["E2b_up"], got["E2b_down"], got["E2c_up"], got["E2c_down"]]
    assert all(np.isfinite(vals)), vals
    assert 0.0 < vals[1] < 1e-2 and vals[3] < 1e-2, vals


@pytest.mark.parametrize("bits,count,closure", [(8, 1, "smagorinsky"), (8, 2, "smagorinsky"),
                                                 (9, 2, "analytic")])
def test_moment_steps_full_size_sampled(ctx, bits, count, closure):
    """M = 256 and 512, one and two fields, one step in the launch
    configuration the bench times (column kernel, 16 planes per workgroup):
    sampled points against the oracle's point-by-point
    step, including the tile, chunk and periodic edges.  At 256^3 the
    diffusivity is the Smagorinsky field (checked against the oracle's); at
    512^3 it is a given smooth field passed to both sides."""
    import torch
    M = 1 << bits
    n = M ** 3
    rng = np.random.default_rng(bits)
    dev = torch.device("cuda")
    U = _paper_velocity(M)
    delta = 3.0 / M
    Ud = _cuda(np.concatenate([u.ravel() for u in U]))
    pts = rng.integers(0, M, size=(400, 3))
    edges = np.array([[0, 0, 0], [M - 1, M - 1, M - 1], [15, 3, 63], [16, 4, 64], [M - 1, 0, 64],
                      [31, M - 1, 0], [32, 127, 191], [33, 128, 255]])
    pts = np.concatenate([pts, edges % M])
    if closure == "smagorinsky":
        Gd = torch.empty(n, dtype=torch.float64, device=dev)
        q.smagorinsky(ctx, bits, Ud, Gd, 2.0, delta, 1e-3)
        Gor = moments.gamma_total(U, 1e-3, 2.0, delta)
        want_g = Gor[tuple(pts.T)]
        got_g = Gd.cpu().numpy().reshape(M, M, M)[tuple(pts.T)]
        assert np.max(np.abs(got_g - want_g)) <= 1e-12 * np.max(np.abs(want_g))
    else:
        x = np.arange(M) / M
        Gor = 1e-3 * (1.0 + 0.5 * np.sin(2 * np.pi * x)[:, None, None]
                      * np.cos(2 * np.pi * x)[None, None, :] + 0 * x[None, :, None])
        Gd = _cuda(Gor.ravel())
    m0 = rng.random((count, M, M, M))
    dt = 0.2 / (M * M * float(Gor.max()) * 6 + M * 4)
    m = _cuda(m0.ravel())
    work = torch.empty_like(m)
    q.moment_steps(ctx, bits, Ud, Gd, m, work, dt, 1)
    got = m.cpu().numpy().reshape(count, M, M, M)
    for a in range(count):
        want = moments.step_at(m0[a], U, Gor, dt, pts)
        _close(got[a][tuple(pts.T)], want, 1e-12)


@pytest.mark.parametrize("bits,chi", [(3, 4), (4, 8), (5, 16)])
def test_from_dense_matches_oracle(ctx, bits, chi):
    """The truncated TT-SVD of a smooth non-separable 3-D field: same
    reconstruction as the oracle's TT-SVD at the same cap, and the discarded
    weight equals the squared approximation error."""
    import torch
    M = 1 << bits
    X1, X2, X3 = np.meshgrid(*(np.arange(M) / M,) * 3, indexing="ij")
    F = np.exp(np.sin(2 * np.pi * X1) * np.cos(2 * np.pi * X2) + 0.5 * np.sin(2 * np.pi * (X2 + X3)))
    F += 0.2 * np.cos(2 * np.pi * (X1 + 2 * X3)) * np.sin(4 * np.pi * X2)
    cores = tt.tt_svd(F.reshape((2,) * (3 * bits)), rel_tol=0.0, chi=chi)
    want = tt.tt_full(cores).ravel()
    x, disc = q.from_dense(ctx, _cuda(F.ravel()), chi)
    out = torch.empty(M ** 3, dtype=torch.float64, device="cuda")
    q.to_dense(ctx, x, out)
    got = out.cpu().numpy()
    err2 = float(np.sum((F.ravel() - want) ** 2))
    assert err2 > 1e-12 * np.sum(F ** 2)  # the cap truncates
    # Gram truncation resolves the kept subspace to about sqrt(eps) sigma_1
    assert np.max(np.abs(got - want)) <= 1e-7 * np.max(np.abs(F))
    assert abs(disc - err2) <= 1e-6 * err2 + 1e-9 * np.sum(F ** 2)


def test_flow_protocol_smagorinsky_runs(ctx):
    """The protocol with the paper's closure: the Smagorinsky field from the
    velocity, cut to a bond cap, and Omega = C_Omega G / Delta^2."""
    from paper_2407_09169_amd import flow
    w = workloads.get_workload("t_5d_M16_chi32", k_react=0.0, integrator="rk2", ic="paper")
    got = flow.run(ctx, w, n_samples=4, steps_per_sample=1, fields="smagorinsky", chi_field=8)
    vals = [got["E2b_up"], got["E2b_down"], got["E2c_up"], got["E2c_down"]]
    assert all(np.isfinite(vals)), vals
    assert got["field_discarded"] >= 0.0
    assert vals[1] < 1e-2 and vals[3] < 1e-2, vals


@pytest.mark.parametrize("bits", [9, 10])
def test_from_dense_full_size(ctx, bits):
    """512^3 and 1024^3 (8 GiB): a sum of two separable smooth terms whose QTT
    singular values fall to rounding level within the cap chi = 8: sampled
    entries equal the field's values to the resolution of a Gram-based cut
    (about sqrt(eps) sigma_1, the floor of reading R9: 3 sqrt(2^-52)), and
    what is discarded is rounding noise."""
    import torch
    M = 1 << bits
    dev = torch.device("cuda")
    x = torch.arange(M, dtype=torch.float64, device=dev) / M
    a = (torch.sin(2 * np.pi * x), torch.cos(4 * np.pi * x) + 2.0, torch.exp(torch.sin(2 * np.pi * x)))
    b = (1.0 + 0.5 * x, torch.sin(6 * np.pi * x), torch.ones_like(x))
    F = (a[0][:, None, None] * a[1][None, :, None] * a[2][None, None, :]
         + b[0][:, None, None] * b[1][None, :, None] * b[2][None, None, :]).reshape(-1)
    xt, disc = q.from_dense(ctx, F, 8)
    out = torch.empty_like(F)
    q.to_dense(ctx, xt, out)
    idx = torch.as_tensor(np.random.default_rng(bits).integers(0, M ** 3, size=4096), device=dev)
    err = (out[idx] - F[idx]).abs().max().item()
    scale = F.abs().max().item()
    assert err <= 3 * np.sqrt(2.0 ** -52) * scale, err / scale
    assert disc <= 1e-12 * float((F * F).sum())
    del F, out
    torch.cuda.empty_cache()
