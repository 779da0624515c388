"""One step of the full 5-D workload (grid 1024^5 as 50 quantics cores,
chi = 128, sketch width 144; the configuration the bench times) on the HIP
path against the oracle's MPS stepper on the same seeded inputs (needs an
MI355X; the oracle step takes about 15 s on the host).

The tensors have 2^50 entries, so they are compared as MPSs: the difference
a - b is written exactly as a block sum (bond 256), left-orthogonalised by
QR, and its norm read off the last core. No inner products are subtracted,
so the measured difference carries no cancellation error. The observables
(integrals of section "Integrated quantities") are compared as well.

Tolerances. The oracle cuts every bond by SVD; the HIP path from the
eigen-decomposition of an FP64 Gram matrix, blind to singular directions
below sqrt(eps) sigma_1. FP64 is held to TRUNC_TOL_F64 (1e-7; the CPU
test test_gram_floor_of_full_size_steps checks that a Gram-matrix emulation
of the truncation moves these very steps by less than a third of it).
FP32-MFMA contractions (the bench's path) round their inputs to 2^-24 and
accumulate K <= 2304 products in FP32: about sqrt(K) 2^-24 = 3e-6 relative
per rounding, five roundings per RK4 step adding in quadrature to ~7e-6;
tolerance 3e-5. BF16 (split operands, 2^-16 per product) runs only the
sketches of the stage slopes, which pick the bases; the projections and the
stage combination stay FP32. It is held to the BF16 target stated for the
method before any run, 1e-2 relative L2.
"""
import numpy as np
import pytest

import workloads
from oracle import stepper, tt
from tests.helpers import TRUNC_TOL_F64, mps_diff_norm, mps_norm

q = pytest.importorskip("paper_2407_09169_amd")

pytestmark = pytest.mark.gpu

NAME = "c3_5d_M1024_chi128"


_diff_norm, _norm = mps_diff_norm, mps_norm


@pytest.fixture(scope="module")
def oracle_step():
    w = workloads.get_workload(NAME)
    st = stepper.MPSStepper(w)
    f0 = st.initial_state()
    f1, _ = st.step(f0)
    return w, f1, st.observables(f1)


@pytest.fixture(scope="module")
def ctx():
    c = q.Context(0)
    yield c
    c.close()


def _check_step(ctx, oracle_step, dtype, tol, label=""):
    w, fo, obs_o = oracle_step
    prob, f = q.setup_workload(ctx, w, dtype)
    prob.step(f, 1)
    fg = [np.asarray(G, dtype=np.float64) for G in f.cores()]
    assert len(fg) == len(fo) == w.n_sites
    err = _diff_norm(fg, fo) / _norm(fo)
    print(f"{NAME} {dtype}{label}: relative L2 difference {err:.3e} (tol {tol:.1e})", flush=True)
    assert err < tol, (dtype, err, tol)
    for k, v in obs_o.items():
        g = prob.observable(f, k)
        assert abs(g - v) <= tol * max(1.0, abs(v)), (k, g, v)
    prob.close()


@pytest.mark.parametrize("dtype,tol", [("f64", TRUNC_TOL_F64), ("f32", 3e-5), ("bf16", 1e-2)])
def test_full_size_step_matches_oracle(ctx, oracle_step, dtype, tol):
    _check_step(ctx, oracle_step, dtype, tol)


@pytest.mark.parametrize("pipeline", ["0", "1", "2", "3", "4", "5"])
@pytest.mark.parametrize("dtype,tol", [("f32", 3e-5), ("bf16", 1e-2)])
def test_full_size_step_each_mfma_pipeline(ctx, oracle_step, monkeypatch, pipeline, dtype, tol):
    """The same step with every MFMA launch forced onto one pipeline (K tile
    32 with one LDS buffer; K tile 32 or 64 with two) and one output tile
    (64 x 64 for 0-2, 32 x 32 for 3-5), at the tolerances above: the measured
    choice per shape may take any of them."""
    monkeypatch.setenv("QTTPDF_MFMA_PIPELINE", pipeline)
    _check_step(ctx, oracle_step, dtype, tol, f" pipeline {pipeline}")


@pytest.fixture(scope="module")
def oracle_step_chi256():
    """One oracle step of the chi = 256 workload (about a minute on the host)."""
    w = workloads.get_workload("c3_5d_M1024_chi256")
    st = stepper.MPSStepper(w)
    f1, _ = st.step(st.initial_state())
    return w, f1, st.observables(f1)


@pytest.mark.parametrize("dtype,tol", [("f64", TRUNC_TOL_F64), ("f32", 3e-5)])
def test_chi256_step_matches_oracle(ctx, oracle_step_chi256, dtype, tol):
    """The chi = 256 case of the same workload (sketch width 288: its QR and
    eigen problems exceed one CU's registers and run on the global-memory
    and blocked kernels) against one oracle step, compared as MPSs, with the
    same bounds as chi = 128; every core finite."""
    w, fo, obs_o = oracle_step_chi256
    prob, f = q.setup_workload(ctx, w, dtype)
    prob.step(f, 1)
    cores = [np.asarray(G, dtype=np.float64) for G in f.cores()]
    assert all(np.all(np.isfinite(G)) for G in cores), dtype
    err = _diff_norm(cores, fo) / _norm(fo)
    print(f"c3_5d_M1024_chi256 {dtype}: relative L2 difference {err:.3e} (tol {tol:.1e})", flush=True)
    assert err < tol, (dtype, err, tol)
    for k, v in obs_o.items():
        g = prob.observable(f, k)
        assert abs(g - v) <= tol * max(1.0, abs(v)), (k, g, v)
    f.free()
    prob.close()


def test_field_step_at_paper_grid_matches_oracle(ctx):
    """One RK2 step on the paper's 128^5 grid (chi = 64) with the x-fields G(x)
    and Omega(x), FP64, against the oracle's field stepper on the same seeded
    inputs; same bound as the constant-coefficient step."""
    w = workloads.get_workload("c2_5d_M128_chi64", integrator="rk2", k_react=0.0)
    st0 = stepper.MPSStepper(w)
    xo = st0._x_order()
    fields = {k: st0._separable(t, xo, 3) for k, t in workloads.flow_field_terms(w).items()}
    st = stepper.MPSStepper(w, fields)
    fo, _ = st.step(st.initial_state())
    tol = TRUNC_TOL_F64
    prob, f = q.setup_workload(ctx, w, "f64", fields=True)
    prob.step(f, 1)
    fg = f.cores()
    err = _diff_norm(fg, fo) / _norm(fo)
    print(f"field step 128^5 chi=64: rel diff {err:.3e} (tol {tol:.3e})")
    assert err < tol, (err, tol)
    f.free()
    prob.close()
