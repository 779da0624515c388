"""Batched stepping (tt_batch_create / tt_step_batched): many uneven problems
advanced by one graph launch give exactly the results of stepping each
problem alone, and those results follow the oracle."""
import numpy as np
import pytest

import paper_2407_09169_amd as q
import workloads
from oracle import stepper
from tests import cases
from tests.helpers import TRUNC_TOL_F64, mps_rel, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = q.Context(0)
    yield c
    c.close()


@pytest.fixture
def request_close():
    """Closes the batches a test registers, also when it fails (a batch must
    not outlive its context)."""
    held = []
    yield held.append
    for b in held:
        b.close()


@pytest.mark.parametrize("fuse", ["1", "0"])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batched_equals_single(ctx, monkeypatch, request_close, dtype, fuse):
    """Six uneven instances, two pairs of equal structure (fused into shared
    launches unless QTTPDF_BATCH_FUSE=0): bitwise the results of stepping
    each instance alone, over two calls."""
    monkeypatch.setenv("QTTPDF_BATCH_FUSE", fuse)
    ws = cases.small_batch(6)
    batched = [q.setup_workload(ctx, w, dtype) for w in ws]
    single = [q.setup_workload(ctx, w, dtype) for w in ws]
    b = q.Batch(ctx, [p for p, _ in batched], [f for _, f in batched])
    request_close(b)
    assert b.info()["fused_classes"] == (2 if fuse == "1" else 0), b.info()
    b.step(2)
    for (p, f) in single:
        p.step(f, 2)
    b.step(1)
    for (p, f) in single:
        p.step(f, 1)
    ctx.synchronize()
    for w, (_, fb), (_, fs) in zip(ws, batched, single):
        for gb, gs in zip(fb.cores(), fs.cores()):
            assert np.array_equal(gb, gs), w.name
    b.close()


def test_batched_instances_match_oracle(ctx):
    ws = cases.small_batch(3)
    insts = [q.setup_workload(ctx, w, "f64") for w in ws]
    b = q.Batch(ctx, [p for p, _ in insts], [f for _, f in insts])
    sts = [stepper.MPSStepper(w) for w in ws]
    fos = [st.initial_state() for st in sts]
    for i in range(2):
        b.step(1)
        for j, st in enumerate(sts):
            fos[j], _ = st.step(fos[j])
        ctx.synchronize()
        for j, (w, st, (_, f)) in enumerate(zip(ws, sts, insts)):
            err = rel(st.to_dense([np.asarray(G) for G in f.cores()]), st.to_dense(fos[j]))
            assert err < TRUNC_TOL_F64, (w.name, i, err)
    b.close()


def test_ensemble_instances_at_real_shapes_match_oracle(ctx):
    """Instances of the 64-instance ensemble at their own grids and bond caps
    (64^5 with chi = 64 and 128, 128^5 with chi = 64, FP64), stepped together
    as one batch, against one oracle step each, compared as MPSs."""
    ws = cases.c4_instances()
    insts = [q.setup_workload(ctx, w, "f64") for w in ws]
    b = q.Batch(ctx, [p for p, _ in insts], [f for _, f in insts])
    b.step(1)
    ctx.synchronize()
    for w, (p, f) in zip(ws, insts):
        st = stepper.MPSStepper(w)
        fo, _ = st.step(st.initial_state())
        err = mps_rel(f.cores(), fo)
        print(f"{w.name}: {err:.3e} (tol {TRUNC_TOL_F64:.0e})", flush=True)
        assert err < TRUNC_TOL_F64, (w.name, err)
    b.close()
    for p, f in insts:
        f.free()
        p.close()


def test_fused_class_at_ensemble_shapes(ctx):
    """Four 64^5 chi = 64 instances of one structure with their own Omega, k,
    dt, velocity, initial PDF and sketches, stepped as one fused class (FP32):
    each bitwise equal to its own tt_step, and the first against the oracle
    to the FP32 step bound of the full-size parity test (3e-5)."""
    w0 = workloads.batch_workloads(count=1, seed=4, bits=(6,), chis=(64,))[0]
    ws = [w0.replace(seed=2000 + i, omega=0.5 + 0.9 * i, k_react=5.0 + 10.0 * i,
                     dt=workloads.stable_dt(5, 6, 0.5 + 0.9 * i, 5.0 + 10.0 * i)) for i in range(4)]
    batched = [q.setup_workload(ctx, w, "f32") for w in ws]
    single = [q.setup_workload(ctx, w, "f32") for w in ws]
    b = q.Batch(ctx, [p for p, _ in batched], [f for _, f in batched])
    try:
        assert b.info()["fused_classes"] == 1 and b.info()["fused_instances"] == 4, b.info()
        b.step(2)
        for p, f in single:
            p.step(f, 2)
        ctx.synchronize()
        for w, (_, fb), (_, fs) in zip(ws, batched, single):
            d = mps_rel(fb.cores(), [np.asarray(G) for G in fs.cores()])
            print(f"{w.name}: fused against alone {d:.3e}", flush=True)
        for w, (_, fb), (_, fs) in zip(ws, batched, single):
            for gb, gs in zip(fb.cores(), fs.cores()):
                assert np.array_equal(gb, gs), w.name
    finally:
        b.close()
    st = stepper.MPSStepper(ws[0])
    fo = st.initial_state()
    for _ in range(2):
        fo, _ = st.step(fo)
    err = mps_rel(batched[0][1].cores(), fo)
    print(f"fused instance 0 against the oracle: {err:.3e}", flush=True)
    assert err < 3e-5, err
    for p, f in batched + single:
        f.free()
        p.close()
