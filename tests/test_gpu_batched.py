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


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batched_equals_single(ctx, dtype):
    ws = cases.small_batch(6)
    batched = [q.setup_workload(ctx, w, dtype) for w in ws]
    single = [q.setup_workload(ctx, w, dtype) for w in ws]
    b = q.Batch(ctx, [p for p, _ in batched], [f for _, f in batched])
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
