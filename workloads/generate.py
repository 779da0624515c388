"""Seeded inputs: grid coordinates, 1-D sample vectors, Gaussian sketch cores.

Nothing here is arithmetic of the method (no operators, no tensor-train
algebra, no time stepping).  The functions return plain float64 arrays:

* ``ic_terms``: the initial PDF as a short sum of separable terms,
  f0 = sum_t c_t * v_t[0](i_0) * v_t[1](i_1) * ...  (one 1-D vector per
  dimension, ``None`` meaning the all-ones vector).  This follows the
  "Gaussian step function" of eq. initPDF (two composition Gaussians of width
  1/8 switched by a window in x1 that is smoothed in x), with seeded centres
  and window edge; ``ic="paper"`` gives the exact paper values.  Each
  composition Gaussian is normalised on the discrete grid so that the
  integral of f over composition space is exactly one at every x.
* ``velocity_terms``: the three velocity components on the x grid as sums of
  separable terms: a Taylor-Green family (a1 C1 S2 S3, a2 S1 C2 S3,
  a3 S1 S2 C3 with a1 + a2 + a3 = 0, hence divergence free) minus the
  Gaussian jet of eq. velField along x1.  ``ic="paper"`` gives a = (1, 1, -2)
  and zero phases, i.e. eq. velField itself.
* ``sketch_cores`` / ``mean_sketch_cores`` (read from the right end) and
  ``left_sketch_cores`` / ``left_mean_sketch_cores`` (read from the left end):
  i.i.d. Gaussian tensor-train cores used as the random sketches of the
  randomized rounding.  They are inputs: both sides of a comparison receive
  the same numbers.
"""
from __future__ import annotations

import numpy as np

from .configs import Workload

KAPPA_TG = 4.0 * np.pi       # Taylor-Green wavenumber k = 4 pi / l0 (eq. velField)
SIGMA_PHI_5D = 1.0 / 8.0     # width of the composition Gaussians (eq. initPDF)
SIGMA_PHI_2D = 0.05
JET_WIDTH = 1.0 / 6.0        # jet profile width (eq. velField)


def phi_points(M: int) -> np.ndarray:
    """Cell-centred composition nodes phi_i = (i + 1/2) / M on [0, 1)."""
    return (np.arange(M, dtype=np.float64) + 0.5) / M


def x_points(M: int) -> np.ndarray:
    """Periodic physical nodes x_j = j / M on [0, 1)."""
    return np.arange(M, dtype=np.float64) / M


def site_order(w: Workload) -> list[tuple[int, int]]:
    """(dimension, bit) of every chain site; bit 0 is the most significant."""
    if w.ordering == "serial":
        return [(d, b) for d in range(w.ndims) for b in range(w.bits)]
    if w.ordering == "interleaved":
        return [(d, b) for b in range(w.bits) for d in range(w.ndims)]
    raise ValueError(w.ordering)


def _phi_gaussian(M: int, mu: float, sigma: float) -> np.ndarray:
    p = phi_points(M)
    g = np.exp(-((p - mu) ** 2) / (2.0 * sigma * sigma))
    return g / (g.sum() / M)


def _smoothed_window(M: int, edge: float) -> np.ndarray:
    """Indicator of [edge, edge + 1/2) on the periodic x grid, smoothed by a
    periodic discrete Gaussian of width two grid spacings (circular FFT
    convolution)."""
    x = x_points(M)
    ind = (np.mod(x - edge, 1.0) < 0.5).astype(np.float64)
    j = np.arange(M)
    dist = np.minimum(j, M - j) / M
    ker = np.exp(-(dist ** 2) / (2.0 * (2.0 / M) ** 2))
    ker /= ker.sum()
    return np.real(np.fft.ifft(np.fft.fft(ind) * np.fft.fft(ker)))


def ic_terms(w: Workload):
    """Initial PDF as [(coeff, [vec per dimension or None]), ...]."""
    M = w.M
    rng = np.random.default_rng([w.seed, 1])
    if w.ndims == 2:
        if w.ic == "paper":
            c1, c2 = (0.75, 0.25), (0.25, 0.75)
        else:
            c1 = tuple(rng.uniform(0.25, 0.75, 2))
            c2 = tuple(rng.uniform(0.25, 0.75, 2))
        s = SIGMA_PHI_2D
        return [
            (0.5, [_phi_gaussian(M, c1[0], s), _phi_gaussian(M, c1[1], s)]),
            (0.5, [_phi_gaussian(M, c2[0], s), _phi_gaussian(M, c2[1], s)]),
        ]
    if w.ndims != 5:
        raise ValueError("ndims must be 2 or 5")
    if w.ic == "paper":
        cA, cB, edge = (0.75, 0.25), (0.25, 0.75), 0.25
    else:
        cA = tuple(rng.uniform(0.2, 0.8, 2))
        cB = tuple(rng.uniform(0.2, 0.8, 2))
        edge = float(rng.uniform(0.0, 0.5))
    s = SIGMA_PHI_5D
    win = _smoothed_window(M, edge)
    return [
        (1.0, [_phi_gaussian(M, cA[0], s), _phi_gaussian(M, cA[1], s), win, None, None]),
        (1.0, [_phi_gaussian(M, cB[0], s), _phi_gaussian(M, cB[1], s), 1.0 - win, None, None]),
    ]


def velocity_terms(w: Workload):
    """[U1_terms, U2_terms, U3_terms], each [(coeff, [v_x1, v_x2, v_x3]), ...]."""
    if w.ndims != 5:
        return []
    M = w.M
    x = x_points(M)
    rng = np.random.default_rng([w.seed, 2])
    if w.ic == "paper":
        th = np.zeros(3)
        a1, a2 = 1.0, 1.0
    else:
        th = rng.uniform(0.0, 2.0 * np.pi, 3)
        a1, a2 = rng.uniform(0.5, 1.5, 2)
    a3 = -(a1 + a2)
    S = [np.sin(KAPPA_TG * x + th[i]) for i in range(3)]
    C = [np.cos(KAPPA_TG * x + th[i]) for i in range(3)]
    jet = np.exp(-((x - 0.5) ** 2) / (2.0 * JET_WIDTH ** 2))
    return [
        [(float(a1), [C[0], S[1], S[2]]), (-1.0, [None, jet, jet])],
        [(float(a2), [S[0], C[1], S[2]])],
        [(float(a3), [S[0], S[1], C[2]])],
    ]


def flow_field_terms(w: Workload):
    """Seeded smooth x-fields standing in for the flow case's variable
    coefficients, as separable terms over (x1, x2, x3):
    {"G": gamma (1 + a sin(2 pi x1 + t1) cos(2 pi x3 + t3)),
     "Omega": omega (1 + b cos(2 pi x2 + t2))}, 0 < a, b < 1/2."""
    x = x_points(w.M)
    rng = np.random.default_rng([w.seed, 3])
    t = rng.uniform(0.0, 2.0 * np.pi, 3)
    a, b = rng.uniform(0.2, 0.5, 2)
    tp = 2.0 * np.pi
    return {
        "G": [(w.gamma, [None, None, None]),
              (w.gamma * a, [np.sin(tp * x + t[0]), None, np.cos(tp * x + t[2])])],
        "Omega": [(w.omega, [None, None, None]), (w.omega * b, [None, np.cos(tp * x + t[1]), None])],
    }


def _chain_ranks(n_sites: int, cap: int) -> list[int]:
    return [min(cap, 1 << n, 1 << (n_sites - n)) for n in range(n_sites + 1)]


def sketch_ranks(w: Workload) -> list[int]:
    """ell_n = min(ell, 2^n, 2^(N-n)) for n = 0..N."""
    return _chain_ranks(w.n_sites, w.ell)


def mean_sketch_ranks(w: Workload) -> list[int]:
    return _chain_ranks(w.n_x_sites, w.ell_mean)


def _gaussian_tt(ranks: list[int], seed) -> list[np.ndarray]:
    rng = np.random.default_rng(seed)
    cores = []
    for n in range(1, len(ranks)):
        rl, rr = ranks[n - 1], ranks[n]
        cores.append(rng.standard_normal((rl, 2, rr)) / np.sqrt(rl))
    return cores


def sketch_cores(w: Workload) -> list[np.ndarray]:
    """Gaussian sketch cores Z_n, shape (ell_{n-1}, 2, ell_n), n = 1..N."""
    return _gaussian_tt(sketch_ranks(w), [w.seed, 3])


def mean_sketch_cores(w: Workload) -> list[np.ndarray]:
    """Gaussian sketch cores for the x-only mean-composition fields."""
    if w.n_x_sites == 0:
        return []
    return _gaussian_tt(mean_sketch_ranks(w), [w.seed, 4])


def left_sketch_cores(w: Workload) -> list[np.ndarray]:
    """Second, independent Gaussian sketch (same ranks as sketch_cores), read
    from the left end by the two-sided rounding."""
    return _gaussian_tt(sketch_ranks(w), [w.seed, 5])


def left_mean_sketch_cores(w: Workload) -> list[np.ndarray]:
    """Second Gaussian sketch for the mean-composition fields."""
    if w.n_x_sites == 0:
        return []
    return _gaussian_tt(mean_sketch_ranks(w), [w.seed, 6])
