"""Batched stepping (tt_batch_create / tt_step_batched): many uneven problems
advanced by one graph launch give exactly the results of stepping each
problem alone, and those results follow the oracle."""
import numpy as np
import pytest

import paper_2407_09169_amd as q
import workloads
from oracle import stepper
from tests.helpers import rel, truncation_sensitivity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = q.Context(0)
    yield c
    c.close()


def _small_batch(count):
    return workloads.batch_workloads(count=count, seed=7, bits=(3, 4), chis=(8, 16, 32))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batched_equals_single(ctx, dtype):
    ws = _small_batch(6)
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
    ws = _small_batch(3)
    insts = [q.setup_workload(ctx, w, "f64") for w in ws]
    b = q.Batch(ctx, [p for p, _ in insts], [f for _, f in insts])
    sts = [stepper.MPSStepper(w) for w in ws]
    fos = [st.initial_state() for st in sts]
    sens = [0.0] * len(ws)
    for i in range(2):
        b.step(1)
        for j, st in enumerate(sts):
            fos[j], infos = st.step(fos[j])
            sens[j] += truncation_sensitivity(infos)
        ctx.synchronize()
        for j, (w, st, (_, f)) in enumerate(zip(ws, sts, insts)):
            err = rel(st.to_dense([np.asarray(G) for G in f.cores()]), st.to_dense(fos[j]))
            assert err < 1e-10 + 10 * sens[j], (w.name, i, err, sens[j])
    b.close()
