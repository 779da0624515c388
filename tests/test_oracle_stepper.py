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
    assert len(infos) == 4  # k1, k2, k3 and the final combination (k4 joins it unrounded)
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


@pytest.mark.parametrize("name,integrator", [("c1_2d_M64_exact", "rk4"), ("t_5d_M8_exact", "rk2")])
def test_untruncated_svd_schedule_equals_dense(name, integrator):
    """The paper's plain schedule (explicit products, QR + truncated-SVD
    rounding of every product and stage combination) is exact when chi covers
    every bond."""
    w = workloads.get_workload(name, integrator=integrator)
    st = stepper.MPSStepper(w, rounding="svd")
    f = st.initial_state()
    P = st.dense_problem()
    fd = st.to_dense(f)
    for _ in range(3):
        f, _ = st.step(f)
        fd = P.step(fd, w.dt, integrator)
        assert _rel(st.to_dense(f), fd) < 1e-12


@pytest.mark.parametrize("name,steps", [("c1_2d_M64", 5), ("t_2d_M64_serial", 5),
                                        ("t_5d_M8_chi16", 3), ("t_5d_M16_chi32", 1)])
def test_randomized_schedule_against_plain_svd_schedule(name, steps):
    """At truncated chi, the randomized two-sided schedule (the one the GPU
    path runs) and the paper's plain QR + SVD schedule approximate the same
    discrete solution about equally well: measured from the same (rounded)
    initial state against the full-grid solver, the randomized step's error
    is within 5 % of the plain one's (measured 0.79 to 1.0 of it: the
    randomized schedule truncates less often, the plain one also rounds
    every stage input and the last stage's product), and the two schedules
    differ from each other by less than the plain schedule's own error
    (measured 0.02 to 0.72 of it).  A rounding that dropped or mis-signed a
    term, or truncated the wrong subspace, fails both."""
    w = workloads.get_workload(name)
    sk = stepper.MPSStepper(w)
    sv = stepper.MPSStepper(w, rounding="svd")
    f1 = sk.initial_state()
    f2 = sv.initial_state()
    P = sk.dense_problem()
    fd = sk.to_dense(f1)
    assert _rel(sv.to_dense(f2), fd) < 1e-13
    for _ in range(steps):
        f1, _ = sk.step(f1)
        f2, _ = sv.step(f2)
        fd = P.step(fd, w.dt, w.integrator)
    d1, d2 = sk.to_dense(f1), sv.to_dense(f2)
    e_rand, e_svd = _rel(d1, fd), _rel(d2, fd)
    assert e_svd > 1e-13  # truncation is active
    assert e_rand <= 1.05 * e_svd
    assert _rel(d1, d2) <= 1.0 * e_svd
    assert max(tt.ranks(f1)) <= w.chi and max(tt.ranks(f2)) <= w.chi


def _mixture_moments(M, gA, gB):
    """Discrete first moments h sum phi g of the four normalised composition
    Gaussians (A and B, for phi1 and phi2)."""
    phi = dense.phi_nodes(M)
    h = 1.0 / M
    return [h * np.dot(phi, g) for g in (gA[0], gB[0], gA[1], gB[1])]


@pytest.mark.parametrize("window", ["constant", "x1"])
def test_covariances_closed_form(window):
    """eq. RACov and eq. SGSCov on a mixture f = w(x) G_A(phi) + (1 - w(x))
    G_B(phi) of two product Gaussians: with a, b the means of Phi_1 under
    G_A, G_B and c, d those of Phi_2, the local means are
    <Phi_1>(x) = w a + (1 - w) b and <Phi_2>(x) = w c + (1 - w) d, so
    R12 = var_x(w) (a - b)(c - d) and Y12 = avg_x(w (1 - w)) (a - b)(c - d).
    A constant w gives R12 = 0 exactly.  Checked for the MPS and the dense
    observables (the seeded 5-D initial state has this form, eq. initPDF)."""
    w = workloads.get_workload("t_5d_M8_exact")
    M = w.M
    terms = workloads.ic_terms(w)
    gA, gB = terms[0][1][:2], terms[1][1][:2]
    win = terms[0][1][2] if window == "x1" else np.full(M, 0.3)
    a, b, c, d = _mixture_moments(M, gA, gB)
    st = stepper.MPSStepper(w)
    f = st._separable([(1.0, [gA[0], gA[1], win, None, None]),
                       (1.0, [gB[0], gB[1], 1.0 - win, None, None])], st.order, 5)
    ob = st.observables(f)
    obd = st.dense_problem().observables(st.to_dense(f))
    R12 = (np.mean(win ** 2) - np.mean(win) ** 2) * (a - b) * (c - d)
    Y12 = np.mean(win * (1.0 - win)) * (a - b) * (c - d)
    assert abs(Y12) > 1e-5  # the centres differ: a non-trivial covariance
    for o in (ob, obd):
        assert abs(o["R12"] - R12) < 1e-14
        assert abs(o["Y12"] - Y12) < 1e-14
        assert abs(o["mass"] - 1.0) < 1e-14
    if window == "constant":
        assert abs(ob["R12"]) < 1e-15
