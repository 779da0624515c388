"""Prolongation of periodic fields to finer grids -- oracle (test infrastructure).

The paper's cost paragraph ("Computational complexity") prepares the input
fields (the mean velocity, the SGS diffusivity, the initial PDF) either by
tensor cross interpolation or by prolongation from a coarser grid.  The
oracle of the prolongation is its plain definition on dense arrays:
periodic linear interpolation onto the grid of twice the resolution along
every axis, x'_(2j) = x_j, x'_(2j+1) = (x_j + x_(j+1 mod M)) / 2, then, for a
result in tensor-train form, the TT-SVD of the fine array cut to a bond cap.

Pins (tests/test_oracle_fields.py): the closed form of the interpolated
Fourier mode cos(2 pi k x) (odd points carry cos(pi k / M) times the mode),
invariance of constants, second-order convergence on a smooth field, and
separability (interpolating a product of 1-D vectors interpolates each).
"""
from __future__ import annotations

import numpy as np

from . import tt


def prolong_dense(F, axes=None):
    """Periodic linear interpolation of the array F onto twice the resolution
    along each axis in `axes` (default: all)."""
    out = np.asarray(F, dtype=np.float64)
    for ax in range(out.ndim) if axes is None else axes:
        nxt = np.roll(out, -1, axis=ax)
        shape = list(out.shape)
        shape[ax] *= 2
        fine = np.empty(shape)
        idx = [slice(None)] * out.ndim
        idx[ax] = slice(0, None, 2)
        fine[tuple(idx)] = out
        idx[ax] = slice(1, None, 2)
        fine[tuple(idx)] = 0.5 * (out + nxt)
        out = fine
    return out


def prolong_tt(F, chi):
    """The prolonged field of the dense array F (every axis of length 2^b)
    as an MPS in serial site order, cut to bond chi by TT-SVD; returns the
    cores and the dense prolonged array."""
    G = prolong_dense(F)
    N = int(round(np.log2(G.size)))
    return tt.tt_svd(G.reshape((2,) * N), rel_tol=0.0, chi=chi), G
