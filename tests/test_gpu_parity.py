"""HIP path vs the CPU oracle, element by element on seeded inputs (needs an MI355X).

Tolerances (FP64 path): operator construction and exact arithmetic agree to
1e-12 relative (rounding only).  Results that went through truncating
roundings are held to the fixed bounds of tests/helpers.py: CUT_TOL_F64
(3 sqrt(eps)) for random chains whose cuts sit on clear spectral gaps, and
TRUNC_TOL_F64 (1e-7) for time steps, whose inputs carry weight below the
sqrt(eps) floor of the HIP path's Gram-matrix truncation; the CPU test
tests/test_tolerances.py checks both readings on these very cases.
"""
import numpy as np
import pytest

import workloads
from oracle import dense, stepper, tt
from tests import cases
from tests.helpers import CUT_TOL_F64, TRUNC_TOL_F64, full, random_tt, rel

q = pytest.importorskip("paper_2407_09169_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = q.Context(0)
    yield c
    c.close()


def _dense_of(st, cores):
    return st.to_dense([np.asarray(G) for G in cores])


# ----------------------------------------------------------------------------- a1
@pytest.mark.parametrize("bits", [3, 5])
@pytest.mark.parametrize("op", ["D1G", "D2G", "D1P", "D2P", "PHI", "D1G_PHI"])
def test_mpo_build_1d_operators(ctx, op, bits):
    M = 1 << bits
    ref = {"D1G": dense.d1_ghost(M), "D2G": dense.d2_ghost(M), "D1P": dense.d1_periodic(M),
           "D2P": dense.d2_periodic(M), "PHI": np.diag(dense.phi_nodes(M)),
           "D1G_PHI": dense.d1_ghost(M) @ np.diag(dense.phi_nodes(M))}[op]
    W, mb = q.mpo_build(ctx, 1, bits, q.TT_SERIAL, [(1.0, {0: op}, -1)])
    A = tt.mpo_full(W.cores())
    assert np.max(np.abs(A - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert mb <= {"D1G": 5, "D2G": 5, "D1P": 3, "D2P": 3, "PHI": 2, "D1G_PHI": 6}[op]


@pytest.mark.parametrize("ordering", ["serial", "interleaved"])
def test_mpo_build_two_dims(ctx, ordering):
    bits, M = 3, 8
    o = q.TT_SERIAL if ordering == "serial" else q.TT_INTERLEAVED
    W, _ = q.mpo_build(ctx, 2, bits, o, [(0.7, {0: "D1G_PHI"}, -1), (-1.3, {0: "PHI", 1: "D2G"}, -1)])
    order = ([(d, b) for d in range(2) for b in range(bits)] if o == q.TT_SERIAL
             else [(d, b) for b in range(bits) for d in range(2)])
    I = np.eye(M)
    K = 0.7 * np.kron(dense.d1_ghost(M) @ np.diag(dense.phi_nodes(M)), I) \
        - 1.3 * np.kron(np.diag(dense.phi_nodes(M)), dense.d2_ghost(M))
    perm = tt.site_perm(order, bits)
    N = 2 * bits
    Kp = K.reshape((2,) * (2 * N)).transpose(perm + [N + p for p in perm]).reshape(1 << N, 1 << N)
    assert np.max(np.abs(tt.mpo_full(W.cores()) - Kp)) <= 1e-12 * np.max(np.abs(Kp))


# ------------------------------------------------------------------- inputs
@pytest.mark.parametrize("name", ["t_5d_M8_exact"] + cases.IC_CASES)
def test_from_separable_matches_oracle(ctx, name):
    w = workloads.get_workload(name)
    st = stepper.MPSStepper(w)
    ordering = q.TT_SERIAL if w.ordering == "serial" else q.TT_INTERLEAVED
    f = q.from_separable(ctx, w.ndims, w.bits, ordering, workloads.ic_terms(w), w.chi)
    fo = st.initial_state()
    tol = TRUNC_TOL_F64 if name in cases.IC_CASES else 1e-12
    assert rel(_dense_of(st, f.cores()), st.to_dense(fo)) < tol
    if w.ndims == 5:
        xo = st._x_order()
        for comp, Uo in zip(workloads.velocity_terms(w), st.U):
            u = q.from_separable(ctx, 3, w.bits, q.TT_SERIAL, comp, w.vel_rank)
            du = tt.sites_to_dense(full(u.cores()), xo, w.bits, 3)
            assert rel(du, tt.sites_to_dense(tt.tt_full(Uo), xo, w.bits, 3)) < 1e-11


# ----------------------------------------------------------------- a3, a4
def test_apply_and_axpby(ctx):
    Wc = cases.random_mpo(8, 3, 10)
    W = q.TT.from_cores(ctx, Wc, kind=q.TT_MPO)
    xc = random_tt([1, 2, 4, 8, 8, 8, 4, 2, 1], 11)
    yc = random_tt([1, 2, 3, 5, 6, 5, 3, 2, 1], 12)
    x = q.TT.from_cores(ctx, xc)
    y = q.TT.from_cores(ctx, yc)
    Wx = q.apply_mpo(ctx, W, x)
    ref = tt.mpo_full(Wc) @ full(xc).reshape(-1)
    assert rel(full(Wx.cores()).reshape(-1), ref) < 1e-13
    s = q.axpby(ctx, [0.3, -2.0], [x, y])
    assert rel(full(s.cores()), 0.3 * full(xc) - 2.0 * full(yc)) < 1e-14
    ip = float(np.sum(full(xc) * full(yc)))
    assert abs(q.inner(ctx, x, y) - ip) < 1e-12 * np.linalg.norm(full(xc)) * np.linalg.norm(full(yc))


@pytest.mark.parametrize("bonds", [[1, 1, 1, 3, 3, 1, 1, 1], [2, 1, 3, 1, 2, 1, 4, 1], [5, 5, 1, 1, 1, 1, 1, 1]])
def test_apply_uneven_mpo_bonds(ctx, bonds):
    """MPO x MPS with bond-1 stretches and uneven bonds (as an operator acting
    on one dimension of a chain has) against the dense product."""
    N = 9
    rng = np.random.default_rng(13)
    caps = [1] + bonds + [1]
    Wc = [rng.standard_normal((caps[n], 2, 2, caps[n + 1])) for n in range(N)]
    W = q.TT.from_cores(ctx, Wc, kind=q.TT_MPO)
    xc = random_tt([1, 2, 4, 8, 8, 8, 8, 4, 2, 1], 14)
    Wx = q.apply_mpo(ctx, W, q.TT.from_cores(ctx, xc))
    ref = tt.mpo_full(Wc) @ full(xc).reshape(-1)
    assert rel(full(Wx.cores()).reshape(-1), ref) < 1e-13


@pytest.mark.parametrize("dim", [0, 1, 2, 3, 4])
def test_apply_single_dimension_operator(ctx, dim):
    """An operator built by mpo_build on one dimension of a 5-D chain, applied
    with mps_apply_mpo to a random state, against the dense finite-difference
    matrix along that axis.  (A random state: the seeded initial PDF does not
    vary along x2 and x3, where the derivative would vanish.)"""
    w = workloads.get_workload("t_5d_M8_chi16")
    st = stepper.MPSStepper(w)
    N, M = w.n_sites, w.M
    xc = random_tt([min(2 ** n, 2 ** (N - n), 12) for n in range(N + 1)], 15 + dim)
    op = "D1G" if dim < 2 else "D1P"
    D = dense.d1_ghost(M) if dim < 2 else dense.d1_periodic(M)
    F = st.to_dense(xc)
    ref = np.moveaxis(np.tensordot(D, F, axes=(1, dim)), 0, dim)
    W, _ = q.mpo_build(ctx, 5, w.bits, q.TT_SERIAL, [(1.0, {dim: op}, -1)])
    y = q.apply_mpo(ctx, W, q.TT.from_cores(ctx, xc))
    assert rel(_dense_of(st, y.cores()), ref) < 1e-13


# --------------------------------------------------------------------- a5
def test_round_det_untruncated(ctx):
    xc = random_tt([1, 2, 4, 8, 16, 16, 8, 4, 2, 1], 21, decay=0.5)
    r = q.round_det(ctx, q.TT.from_cores(ctx, xc), 64)
    assert rel(full(r.cores()), full(xc)) < 1e-13


def _run_rounding_case(ctx, kind, inp, dtype="f64"):
    if kind == "det":
        return q.round_det(ctx, q.TT.from_cores(ctx, inp["x"]), inp["chi"])
    mpos = [None if W is None else q.TT.from_cores(ctx, W, kind=q.TT_MPO) for W in inp["mpos"]]
    xs = [q.TT.from_cores(ctx, x) for x in inp["xs"]]
    left = q.TT.from_cores(ctx, inp["Zl"]) if kind == "two_sided" else None
    return q.round_sketch(ctx, inp["coeffs"], mpos, xs, q.TT.from_cores(ctx, inp["Z"]), inp["chi"],
                          dtype, sketch_left=left)


@pytest.mark.parametrize("name", sorted(cases.ROUNDING_CASES))
def test_rounding_matches_oracle(ctx, name):
    """Deterministic, one-sided and two-sided roundings of random chains
    (bond sizes up to the 5-D chi = 128 workload's: QR of 288 x 144 sketches,
    eigen-decompositions of 144 x 144 Gram matrices) against the oracle."""
    kind, inp, ref, _ = cases.ROUNDING_CASES[name]()
    out = _run_rounding_case(ctx, kind, inp)
    err = rel(full(out.cores()), full(ref))
    print(f"{name}: {err:.3e} (tol {CUT_TOL_F64:.1e})")
    assert err < CUT_TOL_F64, (name, err)


# Reduced-precision contractions against the FP64 oracle: FP32 inputs carry
# relative rounding 2^-24, accumulated over K <= 72 terms per contraction
# (sqrt(K) 2^-24 ~ 5e-7 per product); the smallest kept singular value of
# this case is 8e-3 sigma_1, so the kept subspace moves by at most about
# 5e-7 / 8e-3 ~ 6e-5: tolerance 1e-4.  BF16 splits every operand into a high
# and a low BF16 part (relative 2^-16 per product instead of 2^-24): the same
# bound scaled by 2^8, 2.5e-2.
@pytest.mark.parametrize("dtype,tol", [("f32", 1e-4), ("bf16", 2.5e-2)])
def test_round_sketch_reduced_precision(ctx, dtype, tol):
    kind, inp, ref, _ = cases.ROUNDING_CASES["sketch_N10_chi12"]()
    out = _run_rounding_case(ctx, kind, inp, dtype)
    err = rel(full(out.cores()), full(ref))
    assert err < tol, (dtype, err)


# --------------------------------------------------------------- a6 step
@pytest.mark.parametrize("name,integrator", [("t_5d_M8_exact", "rk4"), ("c1_2d_M64_exact", "rk2")])
def test_step_untruncated_equals_dense(ctx, name, integrator):
    w = workloads.get_workload(name, integrator=integrator)
    st = stepper.MPSStepper(w)
    prob, f = q.setup_workload(ctx, w, "f64")
    P = st.dense_problem()
    fd = dense.dense_from_terms(workloads.ic_terms(w), w.ndims, w.M)
    for _ in range(3):
        prob.step(f, 1)
        fd = P.step(fd, w.dt, integrator)
        err = rel(_dense_of(st, f.cores()), fd)
        assert err < 1e-11, (name, err)


@pytest.mark.parametrize("tile", [str(t) for t in range(1, 8)])
def test_step_untruncated_each_f64_tile(ctx, monkeypatch, tile):
    """The untruncated FP64 step with every FP64 contraction forced onto one
    tile of the SIMT kernel (64 and 32 wide, and the 16-wide ones the
    autotuner tries on shapes with M or N of at most 16): the dense solver's
    result to 1e-11, as with the measured choice."""
    monkeypatch.setenv("QTTPDF_F64_TILE", tile)
    w = workloads.get_workload("t_5d_M8_exact", integrator="rk4")
    st = stepper.MPSStepper(w)
    prob, f = q.setup_workload(ctx, w, "f64")
    P = st.dense_problem()
    fd = dense.dense_from_terms(workloads.ic_terms(w), w.ndims, w.M)
    for _ in range(2):
        prob.step(f, 1)
        fd = P.step(fd, w.dt, "rk4")
        err = rel(_dense_of(st, f.cores()), fd)
        assert err < 1e-11, (tile, err)


@pytest.mark.parametrize("name,integrator,steps", [(n, i, k) for n, i, k, fl in cases.STEP_CASES if not fl])
def test_step_truncated_matches_oracle(ctx, name, integrator, steps):
    """Truncated FP64 steps agree with the oracle (the same randomized schedule
    and sketches, SVD truncation) to TRUNC_TOL_F64."""
    w = workloads.get_workload(name, integrator=integrator)
    st = stepper.MPSStepper(w)
    prob, f = q.setup_workload(ctx, w, "f64")
    fo = st.initial_state()
    tol = TRUNC_TOL_F64
    for i in range(steps):
        prob.step(f, 1)
        fo, _ = st.step(fo)
        err = rel(_dense_of(st, f.cores()), st.to_dense(fo))
        print(f"{name} {integrator} step {i + 1}: {err:.3e} (tol {tol:.0e})")
        assert err < tol, (name, i, err, tol)
    obs_o = st.observables(fo)
    for k, v in obs_o.items():
        g = prob.observable(f, k)
        assert abs(g - v) <= tol * max(1.0, abs(v)), (k, g, v)


def test_step_graph_replay_is_deterministic(ctx):
    """Replays of the recorded step graph give bitwise identical results to an
    eager run of the same plan (several replays, eager work in between)."""
    import os
    w = workloads.get_workload("t_5d_M8_chi16")
    prob, f = q.setup_workload(ctx, w, "f64")
    prob2, g = q.setup_workload(ctx, w, "f64")
    for i in range(3):
        prob.step(f, 1)
        os.environ["QTTPDF_NO_GRAPH"] = "1"
        try:
            prob2.step(g, 1)
        finally:
            del os.environ["QTTPDF_NO_GRAPH"]
        assert np.array_equal(np.concatenate([c.ravel() for c in f.cores()]),
                              np.concatenate([c.ravel() for c in g.cores()]))


def test_l2_diff(ctx):
    xc = random_tt([1, 2, 4, 8, 4, 2, 1], 41)
    yc = [c.copy() for c in xc]
    yc[3] = yc[3] * (1 + 1e-9)
    x, y = q.TT.from_cores(ctx, xc), q.TT.from_cores(ctx, yc)
    ref = rel(full(xc), full(yc))
    assert abs(q.l2_diff(ctx, x, y) - ref) <= 1e-6 * ref


def test_mean_field_matches_oracle(ctx):
    w = workloads.get_workload("t_5d_M8_exact")
    st = stepper.MPSStepper(w)
    prob, f = q.setup_workload(ctx, w, "f64")
    fo = st.initial_state()
    xo = st._x_order()
    for a in (0, 1):
        m = prob.mean_field(f, a)
        md = tt.sites_to_dense(full(m.cores()), xo, w.bits, 3)
        mo = tt.sites_to_dense(tt.tt_full(st.mean_field_raw(fo, a)), xo, w.bits, 3)
        assert rel(md, mo) < 1e-13
