"""Justification, on the CPU, of the fixed FP64 tolerances TRUNC_TOL_F64 and
CUT_TOL_F64 (tests/helpers.py) for every GPU parity case held to them.

The HIP path cuts bonds from eigen-decompositions of FP64 Gram matrices; the
oracle from SVDs.  Two facts make the fixed bound sufficient:
* on the random chains, every cut sits on a clear spectral gap far above the
  Gram floor: the first-order movement of the kept subspaces under relative
  noise eps of the Gram entries is below a tenth of the tolerance;
* on the time-step workloads (whose inputs do have weight below the floor),
  the oracle's own schedule with the truncation emulated from Gram matrices
  stays within a third of the tolerance of the SVD oracle over the steps the
  GPU tests take.
"""
import contextlib

import numpy as np
import pytest

import workloads
from oracle import stepper, tt
from tests import cases
from tests.helpers import CUT_TOL_F64, TRUNC_TOL_F64, cut_sensitivity, mps_rel, rel, trunc_gram_mixed


@contextlib.contextmanager
def gram_truncation():
    """Run the oracle with the HIP path's truncation (Gram eigenvectors)."""
    saved = tt.trunc_svd_mixed, tt.trunc_svd
    tt.trunc_svd_mixed = lambda cores, c, chi, rel_tol=0.0: (trunc_gram_mixed(cores, c, chi), {})
    tt.trunc_svd = lambda X, chi, rel_tol=0.0: (trunc_gram_mixed(X, len(X) - 1, chi), {})
    try:
        yield
    finally:
        tt.trunc_svd_mixed, tt.trunc_svd = saved


@pytest.mark.parametrize("name", sorted(cases.ROUNDING_CASES))
def test_random_chain_cuts_on_clear_gaps(name):
    _, _, _, info = cases.ROUNDING_CASES[name]()
    s = cut_sensitivity([info])
    assert s < CUT_TOL_F64 / 10, (name, s)


def _run(st, steps):
    f = st.initial_state()
    out = []
    for _ in range(steps):
        f, _ = st.step(f)
        out.append(st.to_dense(f))
    return out


@pytest.mark.parametrize("name,integrator,steps,fields", cases.STEP_CASES)
def test_gram_floor_of_step_cases(name, integrator, steps, fields):
    w = workloads.get_workload(name, integrator=integrator)
    make = cases.field_stepper if fields else stepper.MPSStepper
    ref = _run(make(w), steps)
    with gram_truncation():
        emu = _run(make(w), steps)
    worst = max(rel(a, b) for a, b in zip(emu, ref))
    assert worst < TRUNC_TOL_F64 / 3, (name, worst)


def test_gram_floor_of_batch_cases():
    for w in cases.small_batch(3):
        ref = _run(stepper.MPSStepper(w), 2)
        with gram_truncation():
            emu = _run(stepper.MPSStepper(w), 2)
        worst = max(rel(a, b) for a, b in zip(emu, ref))
        assert worst < TRUNC_TOL_F64 / 3, (w.name, worst)


@pytest.mark.slow
def test_gram_floor_of_ensemble_instances():
    """One step of the ensemble instances checked at their real shapes."""
    for w in cases.c4_instances():
        st = stepper.MPSStepper(w)
        ref, _ = st.step(st.initial_state())
        with gram_truncation():
            st2 = stepper.MPSStepper(w)
            emu, _ = st2.step(st2.initial_state())
        assert mps_rel(emu, ref) < TRUNC_TOL_F64 / 3, w.name


@pytest.mark.parametrize("name", cases.IC_CASES)
def test_gram_floor_of_initial_states(name):
    w = workloads.get_workload(name)
    st = stepper.MPSStepper(w)
    ref = st.to_dense(st.initial_state())
    with gram_truncation():
        emu = st.to_dense(st.initial_state())
    assert rel(emu, ref) < TRUNC_TOL_F64 / 3


@pytest.mark.slow
@pytest.mark.parametrize("name,integrator,fields", [("c3_5d_M1024_chi128", "rk4", False),
                                                    ("c2_5d_M128_chi64", "rk2", True)])
def test_gram_floor_of_full_size_steps(name, integrator, fields):
    """One step at the full sizes the GPU parity tests take (the bench's
    1024^5 chi = 128 workload; the paper's 128^5 grid with the x-fields),
    compared as MPSs (about 45 s on the host)."""
    kw = {"integrator": integrator}
    if fields:
        kw["k_react"] = 0.0
    w = workloads.get_workload(name, **kw)
    make = cases.field_stepper if fields else stepper.MPSStepper
    st = make(w)
    ref, _ = st.step(st.initial_state())
    with gram_truncation():
        st2 = make(w)
        emu, _ = st2.step(st2.initial_state())
    assert mps_rel(emu, ref) < TRUNC_TOL_F64 / 3


@pytest.mark.parametrize("name,chi_mean,steps", cases.UNCAPPED_MEAN_CASES)
def test_gram_floor_of_uncapped_mean_cases(name, chi_mean, steps):
    w = cases.uncapped(name, chi_mean)
    ref = _run(stepper.MPSStepper(w), steps)
    with gram_truncation():
        emu = _run(stepper.MPSStepper(w), steps)
    worst = max(rel(a, b) for a, b in zip(emu, ref))
    assert worst < TRUNC_TOL_F64 / 3, (name, worst)
