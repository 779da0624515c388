"""The mean-field term of the stage operator in its two recorded forms: the
block sum A (the term's diag(<Phi_a>) embedded next to the fixed operator in
one MPO) and the Hadamard form (the fixed operator and each mean-field term
-Omega D1g^(phi_a) diag(<Phi_a>) rounded as separate terms, the diagonal
x-site cores contracted without their zeros, which keeps the cost of an
uncapped mean composition down).  Both against the oracle with the mean
compositions kept whole (chi_mean at the x chain's bond cap), and against
each other (needs an MI355X)."""
import os

import numpy as np
import pytest

from oracle import stepper
from tests import cases
from tests.helpers import TRUNC_TOL_F64, rel

q = pytest.importorskip("paper_2407_09169_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = q.Context(0)
    yield c
    c.close()


def _setup(ctx, w, dtype, form):
    os.environ["QTTPDF_MEAN_FORM"] = form
    try:
        return q.setup_workload(ctx, w, dtype)
    finally:
        del os.environ["QTTPDF_MEAN_FORM"]


@pytest.mark.parametrize("name,chi_mean,steps", cases.UNCAPPED_MEAN_CASES)
def test_hadamard_form_matches_oracle(ctx, name, chi_mean, steps):
    w = cases.uncapped(name, chi_mean)
    st = stepper.MPSStepper(w)
    fo = st.initial_state()
    runs = {form: _setup(ctx, w, "f64", form) for form in ("split", "block")}
    for i in range(steps):
        fo, _ = st.step(fo)
        ref = st.to_dense(fo)
        got = {}
        for form, (p, f) in runs.items():
            p.step(f, 1)
            got[form] = st.to_dense([np.asarray(G) for G in f.cores()])
            err = rel(got[form], ref)
            print(f"{name} chi_mean={chi_mean} {form} step {i + 1}: {err:.3e} (tol {TRUNC_TOL_F64:.0e})",
                  flush=True)
            assert err < TRUNC_TOL_F64, (form, i, err)
        # same sums in another order: the two forms agree to rounding
        assert rel(got["split"], got["block"]) < 1e-10
    for p, f in runs.values():
        f.free()
        p.close()


def test_hadamard_form_reduced_precision(ctx):
    """FP32 contractions in the Hadamard form against the FP64 block form
    after two steps (the FP32 step bound of the full-size parity test)."""
    w = cases.uncapped("t_5d_M16_chi32", 32)
    p1, f1 = _setup(ctx, w, "f32", "split")
    p2, f2 = _setup(ctx, w, "f64", "block")
    p1.step(f1, 2)
    p2.step(f2, 2)
    assert q.l2_diff(ctx, f1, f2) < 3e-5
