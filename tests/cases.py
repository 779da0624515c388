"""Inputs of the FP64 parity cases that are held to the truncation tolerance
(tests only).  The GPU parity tests run them on the HIP path; the CPU test
tests/test_tolerances.py checks, on the same inputs, that the tolerance is
justified for each of them."""
import numpy as np

from oracle import tt
from tests.helpers import gaussian_sketch, random_tt


def random_mpo(N, D, seed):
    rng = np.random.default_rng(seed)
    caps = [1] + [D] * (N - 1) + [1]
    return [rng.standard_normal((caps[n], 2, 2, caps[n + 1])) for n in range(N)]


# ------------------------------------------------------- random-chain roundings
# Each case: name -> function returning (kind, inputs, oracle result, oracle info).
#   kind "det":       inputs {"x"}; chi
#   kind "sketch":    inputs {"coeffs", "mpos", "xs", "Z", "chi"}
#   kind "two_sided": inputs as "sketch" plus "Zl"


def _det(chi):
    xc = random_tt([1, 2, 4, 8, 16, 16, 8, 4, 2, 1], 21, decay=0.5)
    ref, info = tt.round_det(xc, chi)
    return "det", {"x": xc, "chi": chi}, ref, info


def _sketch():
    N = 10
    Wc = random_mpo(N, 3, 30)
    xc = random_tt([1, 2, 4, 8, 16, 24, 16, 8, 4, 2, 1], 31, decay=0.7)
    yc = random_tt([1, 2, 4, 8, 12, 12, 12, 8, 4, 2, 1], 32, decay=0.7)
    Z, ell = gaussian_sketch(N, 20, 33)
    chi = 12
    inp = {"coeffs": [1.0, -0.25, 3.0], "mpos": [Wc, Wc, None], "xs": [xc, yc, xc], "Z": Z, "chi": chi}
    ref, info = tt.round_sketch(list(zip(inp["coeffs"], inp["mpos"], inp["xs"])), Z, ell, chi)
    return "sketch", inp, ref, info


def _large(ell, chi):
    """Bond sizes of the 5-D chi = 128 workload (QR of 288 x 144 sketches,
    eigen-decompositions of 144 x 144 Gram matrices) on a 16-core chain."""
    N = 16
    caps = [min(2 ** n, 2 ** (N - n), 160) for n in range(N + 1)]
    xc = random_tt(caps, 51, decay=0.99)
    Wc = random_mpo(N, 2, 52)
    Z, ellr = gaussian_sketch(N, ell, 53)
    inp = {"coeffs": [1.0, 0.5], "mpos": [Wc, None], "xs": [xc, xc], "Z": Z, "chi": chi}
    ref, info = tt.round_sketch(list(zip(inp["coeffs"], inp["mpos"], inp["xs"])), Z, ellr, chi)
    return "sketch", inp, ref, info


def _two_sided(N, cap, decay, ell, chi):
    """Sums of MPO-applied chains whose spectra run well past the sketch width,
    so the range finder and the truncation both cut real weight."""
    caps = [min(2 ** n, 2 ** (N - n), cap) for n in range(N + 1)]
    xc = random_tt(caps, 61, decay=decay)
    yc = random_tt(caps, 62, decay=decay)
    Wc = random_mpo(N, 2, 63)
    Z, _ = gaussian_sketch(N, ell, 64)
    Zl, _ = gaussian_sketch(N, ell, 65)
    inp = {"coeffs": [1.0, -0.25, 0.5], "mpos": [Wc, Wc, None], "xs": [xc, yc, xc], "Z": Z, "Zl": Zl,
           "chi": chi}
    ref, info = tt.round_sketch_two_sided(list(zip(inp["coeffs"], inp["mpos"], inp["xs"])), Z, Zl, chi)
    return "two_sided", inp, ref, info


ROUNDING_CASES = {
    "det_chi3": lambda: _det(3),
    "det_chi6": lambda: _det(6),
    "sketch_N10_chi12": _sketch,
    "large_ell144_chi128": lambda: _large(144, 128),
    "large_ell80_chi64": lambda: _large(80, 64),
    "large_ell40_chi32": lambda: _large(40, 32),
    "two_sided_N10_chi12": lambda: _two_sided(10, 24, 0.7, 20, 12),
    "two_sided_N12_chi32": lambda: _two_sided(12, 64, 0.9, 40, 32),
    "two_sided_N16_chi128": lambda: _two_sided(16, 160, 0.97, 144, 128),
}

# ------------------------------------------------------------ truncated steps
# (workload name, integrator, steps, with the flow-case x-fields)
STEP_CASES = [
    ("t_5d_M8_chi16", "rk4", 3, False),
    ("c1_2d_M64", "rk4", 3, False),
    ("t_2d_M64_serial", "rk2", 3, False),
    ("t_5d_M8_chi16", "rk2", 3, True),
    ("t_5d_M16_chi32", "rk4", 3, True),
]
# initial states built on the host and rounded (tt_from_separable)
IC_CASES = ["c1_2d_M64", "t_5d_M8_chi16"]


def small_batch(count):
    """Uneven 5-D instances of the batched parity tests (M <= 16, chi <= 32)."""
    import workloads
    return workloads.batch_workloads(count=count, seed=7, bits=(3, 4), chis=(8, 16, 32))


def field_stepper(w, rounding="sketch"):
    """Oracle stepper with the seeded flow-case x-fields G(x), Omega(x)."""
    import workloads
    from oracle import stepper
    st0 = stepper.MPSStepper(w)
    xo = st0._x_order()
    fields = {k: st0._separable(terms, xo, 3) for k, terms in workloads.flow_field_terms(w).items()}
    return stepper.MPSStepper(w, fields, rounding=rounding)


# instances of the 64-instance ensemble (workloads.batch_workloads()) checked
# against the oracle at their real shapes: 64^5 with chi = 64 and 128, 128^5
# with chi = 64
C4_INSTANCES = [3, 13, 2]


def c4_instances():
    import workloads
    ws = workloads.batch_workloads()
    return [ws[i] for i in C4_INSTANCES]


# workloads with the mean compositions kept whole (chi_mean at the bond cap of
# their x chains): (name, chi_mean, steps)
UNCAPPED_MEAN_CASES = [("t_5d_M8_chi16", 16, 3), ("t_5d_M16_chi32", 32, 2)]


def uncapped(name, chi_mean):
    import workloads
    return workloads.get_workload(name).replace(chi_mean=chi_mean, oversample_mean=8)
