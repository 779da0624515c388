"""Moment equation, Smagorinsky closure and error measures -- oracle (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the bench use this
module; the GPU library never calls it.

What it computes (plain numpy, FP64, dense grids of shape (M, M, M) over
(x1, x2, x3), x_j = j h, h = 1/M, periodic):

* ``gamma_total``: the total diffusivity gamma + gamma_SGS of eq. FP0, with
  the Smagorinsky closure of the paragraph after eq. FP0: C_s (Delta^2 / 2)
  times the square root of the sum over i, j of (dU_i/dx_j + dU_j/dx_i)^2.
  The velocity derivatives are the CFD2 periodic differences of the grid
  values ("Finite-difference discretisation").
* ``omega_field``: the LMSE mixing frequency C_Omega (gamma + gamma_SGS) /
  Delta^2 (same paragraph).
* ``rhs`` / ``step``: eq. FPMoms with S = 0 (Da = 0), RK2 (Heun) in time and
  CFD2 in space.  The variable-coefficient diffusion d/dx_i (G dm/dx_i) is
  written in expanded form, G D2_i m + (D1_i G)(D1_i m), the form in which a
  diagonal field times a difference operator expresses it.
* ``error_measures``: the four RMSE measures of eq. RMSE0 with the averages of
  eq. RMSE1 taken as the mean over the time samples (17 samples from 0 to
  2 T0 in the paper) and the mean over all grid points.

Pins: tests/test_oracle_moments.py (closed-form Fourier-mode amplification
under diffusion and under advection, second-order convergence of the
variable-coefficient operator and of the Smagorinsky field against analytic
derivatives, agreement with the first composition moment of the dense
Fokker-Planck solver when the composition-space terms vanish, and closed
forms of the error measures).
"""
from __future__ import annotations

import numpy as np

from .dense import apply_axis, d1_periodic, d2_periodic


def _d1(g: np.ndarray, axis: int) -> np.ndarray:
    return apply_axis(d1_periodic(g.shape[axis]), g, axis)


def _d2(g: np.ndarray, axis: int) -> np.ndarray:
    return apply_axis(d2_periodic(g.shape[axis]), g, axis)


def strain_norm(U) -> np.ndarray:
    """sqrt(sum_ij (dU_i/dx_j + dU_j/dx_i)^2) with CFD2 periodic differences."""
    grad = [[_d1(U[i], j) for j in range(3)] for i in range(3)]  # grad[i][j] = dU_i/dx_j
    s = np.zeros_like(U[0])
    for i in range(3):
        for j in range(3):
            s += (grad[i][j] + grad[j][i]) ** 2
    return np.sqrt(s)


def gamma_total(U, gamma: float, c_s: float, delta: float) -> np.ndarray:
    """gamma + gamma_SGS with the Smagorinsky closure (C_s Delta^2 / 2) |S|."""
    return gamma + c_s * delta * delta / 2.0 * strain_norm(U)


def omega_field(G: np.ndarray, c_omega: float, delta: float) -> np.ndarray:
    """LMSE mixing frequency Omega_mix = C_Omega (gamma + gamma_SGS) / Delta^2."""
    return c_omega * G / (delta * delta)


def rhs(m: np.ndarray, U, G) -> np.ndarray:
    """Right-hand side of eq. FPMoms at S = 0:
    -U_i D1_i m + G D2_i m + (D1_i G)(D1_i m), summed over i."""
    out = np.zeros_like(m)
    for i in range(3):
        dm = _d1(m, i)
        out += -U[i] * dm + G * _d2(m, i) + _d1(G, i) * dm
    return out


def step(m: np.ndarray, U, G, dt: float) -> np.ndarray:
    """One RK2 step in Heun form: m1 = m + dt L(m); m+ = m + dt/2 (L(m) + L(m1))."""
    k1 = rhs(m, U, G)
    m1 = m + dt * k1
    k2 = rhs(m1, U, G)
    return m + 0.5 * dt * (k1 + k2)


def rhs_at(m: np.ndarray, U, G, pts: np.ndarray) -> np.ndarray:
    """The right-hand side of ``rhs`` at the grid points pts (k x 3 integer
    indices), each evaluated on its own from its periodic neighbours: for
    checks of large grids at sampled points."""
    M = m.shape[0]
    h = 1.0 / M
    pts = np.asarray(pts) % M
    out = np.zeros(len(pts))
    for q, (a, b, c) in enumerate(pts):
        idx = (a, b, c)
        for i in range(3):
            p1 = list(idx)
            m1 = list(idx)
            p1[i] = (idx[i] + 1) % M
            m1[i] = (idx[i] - 1) % M
            p1, m1 = tuple(p1), tuple(m1)
            d1 = (m[p1] - m[m1]) / (2 * h)
            d2 = (m[p1] - 2 * m[idx] + m[m1]) / (h * h)
            dG = (G[p1] - G[m1]) / (2 * h)
            out[q] += -U[i][idx] * d1 + G[idx] * d2 + dG * d1
    return out


def step_at(m: np.ndarray, U, G, dt: float, pts: np.ndarray) -> np.ndarray:
    """One Heun step (as ``step``) at the grid points pts only: the first
    stage is evaluated at the points and their six neighbours."""
    M = m.shape[0]
    pts = np.asarray(pts) % M
    offs = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    nb = np.concatenate([(pts + np.array(o)) % M for o in offs])
    m1_nb = m[tuple(nb.T)] + dt * rhs_at(m, U, G, nb)
    m1 = m.copy()  # only the stencil points of m1 are used below
    m1[tuple(nb.T)] = m1_nb
    k1 = rhs_at(m, U, G, pts)
    k2 = rhs_at(m1, U, G, pts)
    return m[tuple(pts.T)] + 0.5 * dt * (k1 + k2)


def time_mean_sq(g, g0) -> float:
    """E_t of eq. RMSE1: the mean over the time samples of (g - g0)^2."""
    g = np.asarray(g, dtype=np.float64)
    g0 = np.broadcast_to(np.asarray(g0, dtype=np.float64), g.shape)
    return float(np.mean((g - g0) ** 2))


def space_time_mean_sq(g, g0) -> float:
    """E_{t,x} of eq. RMSE1: the mean over time samples and grid points of
    (g - g0)^2; g has shape (n_samples, ...) and g0 broadcasts to it."""
    g = np.asarray(g, dtype=np.float64)
    g0 = np.broadcast_to(np.asarray(g0, dtype=np.float64), g.shape)
    return float(np.mean((g - g0) ** 2))


def error_measures(mean_bar, mean_x, mean_x_exact, norm_x):
    """The four RMSE measures of eq. RMSE0.

    mean_bar:      (2, T) space averages of <Phi_a> at the T time samples
    mean_x:        (2, T, ...) <Phi_a>(x) of the MPS solution
    mean_x_exact:  (2, T, ...) <Phi_a>(x) of the moment equation (or None)
    norm_x:        (T, ...) <1>(x) of the MPS solution
    Returns (E2b_up, E2b_down, E2c_up, E2c_down); E2b_down is NaN without an
    exact solution.
    """
    mean_bar = np.asarray(mean_bar, dtype=np.float64)
    e2b_up = np.sqrt(0.5 * sum(time_mean_sq(mean_bar[a], 0.5) for a in range(2)))
    if mean_x_exact is None:
        e2b_dn = float("nan")
    else:
        e2b_dn = np.sqrt(0.5 * sum(space_time_mean_sq(mean_x[a], mean_x_exact[a]) for a in range(2)))
    e2c_up = np.sqrt(time_mean_sq(mean_bar[0] - mean_bar[1], 0.0))
    e2c_dn = np.sqrt(space_time_mean_sq(norm_x, 1.0))
    return float(e2b_up), float(e2b_dn), float(e2c_up), float(e2c_dn)
