"""The boundary's reporting and option calls against the oracle and against
the plain calls: rounding with a relative tolerance and its outcome record,
the precision argument of the explicit MPO x MPS product, per-step records,
non-finite detection, and the caller's allocator (needs an MI355X)."""
import numpy as np
import pytest

import workloads
from oracle import tt
from tests import cases
from tests.helpers import CUT_TOL_F64, full, random_tt, rel

q = pytest.importorskip("paper_2407_09169_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = q.Context(0)
    yield c
    c.close()


def _graded(seed):
    """8-site chain whose middle bond has singular values 0.6^i (i < 16)."""
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((16, 16)))
    V, _ = np.linalg.qr(rng.standard_normal((16, 16)))
    T = (U * 0.6 ** np.arange(16)) @ V.T
    return tt.tt_svd(T.reshape((2,) * 8), rel_tol=0.0)


@pytest.mark.parametrize("chi,rel_tol", [(16, 0.0), (16, 1e-3), (6, 0.0), (16, 0.05)])
def test_round_rel_tol_and_info_match_oracle(ctx, chi, rel_tol):
    """mps_round with a relative tolerance: the kept singular values at every
    bond are those above rel_tol sigma_1 (at most chi), as in the oracle's
    SVD truncation; the outcome record's discarded weights, largest bond and
    norm agree with the oracle's."""
    xc = _graded(81)
    ref, info_o = tt.round_det(xc, chi, rel_tol)
    out, info = q.round_det(ctx, q.TT.from_cores(ctx, xc), chi, rel_tol, with_info=True)
    assert rel(full(out.cores()), full(ref)) < CUT_TOL_F64
    assert info["max_bond"] == max(info_o["ranks"])
    s1 = info_o["norm2"]
    assert abs(info["norm2"] - s1) <= 1e-12 * s1
    for a, b in zip(info["per_bond"], info_o["discarded"]):
        assert abs(a - b) <= 1e-12 * s1 + 1e-10 * b
    assert abs(info["discarded_weight"] - sum(info_o["discarded"])) <= 1e-12 * s1


@pytest.mark.parametrize("dtype,tol,pipeline", [("f64", 1e-14, None)] + [
    ("f64", 1e-14, f"f64 tile {t}") for t in range(1, 8)] + [
    (d, t, pl) for d, t in (("f32", 2e-7), ("bf16", 1e-4)) for pl in (None, "0", "1", "2", "3", "4", "5")])
def test_apply_mpo_precision(ctx, monkeypatch, dtype, tol, pipeline):
    """Explicit MPO x MPS product with FP64 products, FP32-rounded operands
    (relative 2^-24 per operand: a product errs by at most 2^-23 of its size,
    and the two products of an entry add at most that again), or BF16 high
    and low parts (2^-16 per product): entries against the FP64 dense
    product, relative to the largest entry.  pipeline: every MFMA launch
    forced onto one of the three pipelines with 64 x 64 tiles (0-2) or with
    32 x 32 tiles (3-5), every FP64 launch onto one of its seven tiles (64 or
    32 wide, and the 16-wide ones) (None: the measured choice)."""
    if pipeline is not None and pipeline.startswith("f64 tile"):
        monkeypatch.setenv("QTTPDF_F64_TILE", pipeline.split()[-1])
    elif pipeline is not None:
        monkeypatch.setenv("QTTPDF_MFMA_PIPELINE", pipeline)
    Wc = cases.random_mpo(8, 3, 91)
    xc = random_tt([1, 2, 4, 8, 8, 8, 4, 2, 1], 92)
    W = q.TT.from_cores(ctx, Wc, kind=q.TT_MPO)
    y = q.apply_mpo(ctx, W, q.TT.from_cores(ctx, xc), dtype)
    ref = tt.mpo_full(Wc) @ full(xc).reshape(-1)
    exact = q.apply_mpo(ctx, W, q.TT.from_cores(ctx, xc), "f64")
    # entry-wise: the cores of the product, against the FP64 cores
    for a, b in zip(y.cores(), exact.cores()):
        assert np.max(np.abs(a - b)) <= tol * max(np.max(np.abs(b)), 1e-300)
    assert rel(full(exact.cores()).reshape(-1), ref) < 1e-13


def test_step_records(ctx):
    """tt_step_ex records avg <1> - 1, the final rounding's discarded weight
    and the largest kept bond after every step, and advances f exactly as
    tt_step does (bitwise)."""
    w = workloads.get_workload("t_5d_M8_chi16")
    p1, f1 = q.setup_workload(ctx, w, "f64")
    p2, f2 = q.setup_workload(ctx, w, "f64")
    recs = p1.step_ex(f1, 3)
    assert len(recs) == 3
    p2.step(f2, 3)
    ctx.synchronize()
    for a, b in zip(f1.cores(), f2.cores()):
        assert np.array_equal(a, b)
    disc, _ = p1.step_info()
    r = recs[-1]
    assert abs(r["mass_dev"] - (p1.observable(f1, "mass") - 1.0)) < 1e-14
    assert abs(r["discarded_weight"] - float(np.sum(disc))) <= 1e-12 * max(1.0, float(np.sum(disc)))
    assert all(1 <= x["max_bond"] <= w.chi and x["nonfinite"] == 0 for x in recs)
    assert all(abs(x["mass_dev"]) < 1e-8 for x in recs)


def test_nonfinite_is_reported(ctx):
    """A NaN put into the state through tt_set_cores reaches the roundings of
    the next step: tt_step_ex stops with TT_ERR_NONFINITE and records it; a
    plain tt_step is reported by the next tt_step_info, which clears the
    condition."""
    w = workloads.get_workload("t_5d_M8_chi16")
    p, f = q.setup_workload(ctx, w, "f64")
    cores = f.cores()
    cores[5][0, 1, 0] = np.nan
    f.set_cores(cores)
    with pytest.raises(q.QttError) as e:
        p.step_ex(f, 2)
    assert e.value.status == 4 and e.value.records[0]["nonfinite"] == 1
    p.step(f, 1)
    with pytest.raises(q.QttError, match="NaN or Inf"):
        p.step_info()
    p.step_info()  # cleared


def test_torch_allocator(ctx):
    """With PyTorch's caching allocator registered, the library's device
    memory is torch's (its allocated-bytes counter grows by the problem's
    workspaces) and a step gives bitwise the result of the hipMalloc path."""
    import torch
    w = workloads.get_workload("t_5d_M8_chi16")
    p0, f0 = q.setup_workload(ctx, w, "f64")
    p0.step(f0, 2)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    q.use_torch_allocator()
    try:
        p1, f1 = q.setup_workload(ctx, w, "f64")
        p1.step(f1, 2)
        ctx.synchronize()
        assert torch.cuda.memory_allocated() > before
        for a, b in zip(f1.cores(), f0.cores()):
            assert np.array_equal(a, b)
        f1.free()
        p1.close()
    finally:
        q.use_torch_allocator(False)
    assert torch.cuda.memory_allocated() >= before


@pytest.mark.parametrize("N,cap,ell,chi", [(10, 24, 20, 12), (16, 160, 144, 128)])
def test_round_zero_chain(ctx, N, cap, ell, chi):
    """The degenerate input of a rounding: a chain of zero cores.  Every
    sketch, Gram matrix and eigenvalue is zero; the deterministic and the
    two-sided sketched roundings return the zero tensor with finite cores,
    and the outcome record reports zero norm and zero discarded weight."""
    from tests.helpers import gaussian_sketch
    caps = [min(2 ** n, 2 ** (N - n), cap) for n in range(N + 1)]
    zc = [np.zeros((caps[n], 2, caps[n + 1])) for n in range(N)]
    x = q.TT.from_cores(ctx, zc)
    out, info = q.round_det(ctx, x, chi, 1e-3, with_info=True)
    cores = out.cores()
    assert all(np.all(np.isfinite(c)) for c in cores)
    assert np.abs(full(cores)).max() == 0.0
    assert info["norm2"] == 0.0 and info["discarded_weight"] == 0.0
    assert all(v == 0.0 for v in info["per_bond"])
    Z, _ = gaussian_sketch(N, ell, 91)
    Zl, _ = gaussian_sketch(N, ell, 92)
    out2 = q.round_sketch(ctx, [1.0], [None], [x], q.TT.from_cores(ctx, Z), chi,
                          sketch_left=q.TT.from_cores(ctx, Zl))
    cores2 = out2.cores()
    assert all(np.all(np.isfinite(c)) for c in cores2)
    assert np.abs(full(cores2)).max() == 0.0
