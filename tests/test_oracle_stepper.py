"""Pins of the MPS stepper oracle: without truncation it must reproduce the
pinned full-grid solver (the paper: chi large makes the MPS exact)."""
import numpy as np
import pytest

import workloads
from oracle import dense, stepper, tt


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("name,integrator", [("c1_2d_M64_exact", "rk4"),
                                             ("c1_2d_M64_exact", "rk2"),
                                             ("t_5d_M8_exact", "rk4")])
def test_untruncated_mps_equals_dense(name, integrator):
    w = workloads.get_workload(name, integrator=integrator)
    st = stepper.MPSStepper(w)
    f = st.initial_state()
    P = st.dense_problem()
    fd = dense.dense_from_terms(workloads.ic_terms(w), w.ndims, w.M)
    assert _rel(st.to_dense(f), fd) < 1e-13
    for _ in range(4):
        f, _ = st.step(f)
        fd = P.step(fd, w.dt, integrator)
        assert _rel(st.to_dense(f), fd) < 1e-12
    obs_t, obs_d = st.observables(f), P.observables(fd)
    for k in obs_d:
        assert abs(obs_t[k] - obs_d[k]) < 1e-12 * max(1.0, abs(obs_d[k])), k


def test_mean_field_mps_equals_dense():
    w = workloads.get_workload("t_5d_M8_exact")
    st = stepper.MPSStepper(w)
    f = st.initial_state()
    P = st.dense_problem()
    fd = st.to_dense(f)
    xo = st._x_order()
    for a in (0, 1):
        m = st.mean_field_raw(f, a)
        md = tt.sites_to_dense(tt.tt_full(m), xo, w.bits, 3)
        assert np.allclose(md, P.mean_field(fd, a)[0, 0], atol=1e-14)


def test_truncated_step_reports_and_conserves():
    """A truncated run stays close to the full-grid solution and keeps <1> = 1
    to within the truncation level; every rounding reports its discarded weight."""
    w = workloads.get_workload("t_5d_M8_chi16")
    st = stepper.MPSStepper(w)
    f = st.initial_state()
    P = st.dense_problem()
    fd = dense.dense_from_terms(workloads.ic_terms(w), 5, w.M)
    for _ in range(3):
        f, infos = st.step(f)
        fd = P.step(fd, w.dt, w.integrator)
    assert len(infos) == 5
    assert max(tt.ranks(f)) <= w.chi
    err = _rel(st.to_dense(f), fd)
    assert err < 5e-2
    mass = P.norm_field(st.to_dense(f))
    assert np.max(np.abs(mass - 1.0)) < 10 * err + 1e-12


def _field_stepper(w):
    st0 = stepper.MPSStepper(w)
    xo = st0._x_order()
    fields = {k: st0._separable(terms, xo, 3) for k, terms in workloads.flow_field_terms(w).items()}
    return stepper.MPSStepper(w, fields)


@pytest.mark.parametrize("integrator", ["rk2", "rk4"])
def test_untruncated_mps_with_fields_equals_dense(integrator):
    """Variable diffusivity G(x) and mixing frequency Omega(x): the exact-rank
    MPS stepper reproduces the full-grid solver with the same fields."""
    w = workloads.get_workload("t_5d_M8_exact", integrator=integrator)
    st = _field_stepper(w)
    P = st.dense_problem()
    assert P.G is not None and P.Omega is not None
    assert np.ptp(P.G) > 0.3 * w.gamma and np.ptp(P.Omega) > 0.3 * w.omega
    f = st.initial_state()
    fd = st.to_dense(f)
    for _ in range(3):
        f, _ = st.step(f)
        fd = P.step(fd, w.dt, integrator)
        assert _rel(st.to_dense(f), fd) < 1e-12
    # the fields change the solution: a constant-coefficient run differs
    P0 = stepper.MPSStepper(w).dense_problem()
    f0 = st.to_dense(st.initial_state())
    for _ in range(3):
        f0 = P0.step(f0, w.dt, integrator)
    assert _rel(f0, fd) > 1e-6


def test_constant_fields_reduce_to_constants():
    w = workloads.get_workload("t_5d_M8_exact")
    st = stepper.MPSStepper(w)
    P = st.dense_problem()
    M = w.M
    Pf = dense.DenseProblem(5, M, w.omega, w.k_react, w.nu_phi, 0.0, P.U,
                            G=np.full((M, M, M), w.gamma), Omega=np.full((M, M, M), w.omega))
    f = st.to_dense(st.initial_state())
    assert _rel(Pf.rhs(f), P.rhs(f)) < 1e-14
