"""Full-grid finite-difference solver of eq. FP2 -- oracle (test infrastructure).

Discretisation ("Finite-difference discretisation" section, eq. FP2, eq.
compBCs):

* equidistant grids with M = 2**bits points per dimension; composition nodes
  are cell-centred, phi_i = (i + 1/2) h, physical nodes x_j = j h, h = 1/M;
* second-order central differences (CFD2) for first and second derivatives;
* periodic boundaries in x;
* composition-space ghost points chosen so that the sum over the grid of any
  discrete derivative vanishes (eq. compBCs): g_{-1} = -g_0, g_M = -g_{M-1}
  for first derivatives and g_{-1} = g_0, g_M = g_{M-1} for second ones;
* the LMSE drift plus the artificial dissipation of eq. FP2 in composition
  space, read as D1g[Omega (phi_a - <Phi_a>) f] + nu_phi D2g f (the
  dissipation written with the compact second-difference stencil);
* the bilinear reaction S_1 = S_2 = -k phi1 phi2 of the binary scheme
  A + B -> P, entering as -D1g(S_a f) = +k D1g(phi1 phi2 f);
* convection -U_i D1p f and diffusion Gamma D2p f in x (constant Gamma);
* the mean composition <Phi_a>(x) = h^2 sum_{i1,i2} phi_a f is the raw
  integral (no division by <1>), recomputed at every Runge-Kutta stage;
* explicit RK4 (classic) or RK2 in Heun form.

Array layout: f has shape (M,) * ndims with axes (phi1, phi2[, x1, x2, x3]).
Velocity components U_i are arrays of shape (M, M, M) over (x1, x2, x3).

Pins: tests/test_oracle_dense.py (ghost rules, eq. compBCs column sums, the
Ornstein-Uhlenbeck moment law of the 2-D mixing model, a Fourier mode of the
periodic advection-diffusion operator under RK4, the normalisation and
species-symmetry invariants, reaction consumption, separability at
C_Omega = 0).
"""
from __future__ import annotations

import numpy as np


# ----------------------------------------------------------------------------
# 1-D operators
# ----------------------------------------------------------------------------
def _stencil(M: int, offsets: dict[int, float], boundary) -> np.ndarray:
    """Matrix of sum_o c_o g_{i+o} with the given boundary treatment.

    boundary == "periodic": indices wrap.  boundary == ("ghost", sign): the
    out-of-range neighbours are ghost values g_{-1} = sign*g_0 and
    g_M = sign*g_{M-1}.
    """
    A = np.zeros((M, M))
    for i in range(M):
        for o, c in offsets.items():
            j = i + o
            if boundary == "periodic":
                A[i, j % M] += c
                continue
            _, sign = boundary
            if j < 0:
                A[i, 0] += sign * c
            elif j >= M:
                A[i, M - 1] += sign * c
            else:
                A[i, j] += c
    return A


def d1_ghost(M: int) -> np.ndarray:
    """First derivative, composition space (ghosts g_{-1}=-g_0, g_M=-g_{M-1})."""
    h = 1.0 / M
    return _stencil(M, {1: 1.0 / (2 * h), -1: -1.0 / (2 * h)}, ("ghost", -1.0))


def d2_ghost(M: int) -> np.ndarray:
    """Second derivative, composition space (ghosts g_{-1}=g_0, g_M=g_{M-1})."""
    h = 1.0 / M
    return _stencil(M, {1: 1.0 / h**2, 0: -2.0 / h**2, -1: 1.0 / h**2}, ("ghost", 1.0))


def d1_periodic(M: int) -> np.ndarray:
    h = 1.0 / M
    return _stencil(M, {1: 1.0 / (2 * h), -1: -1.0 / (2 * h)}, "periodic")


def d2_periodic(M: int) -> np.ndarray:
    h = 1.0 / M
    return _stencil(M, {1: 1.0 / h**2, 0: -2.0 / h**2, -1: 1.0 / h**2}, "periodic")


def phi_nodes(M: int) -> np.ndarray:
    return (np.arange(M) + 0.5) / M


def apply_axis(A: np.ndarray, f: np.ndarray, axis: int) -> np.ndarray:
    return np.moveaxis(np.tensordot(A, f, axes=(1, axis)), 0, axis)


# ----------------------------------------------------------------------------
# Problem and right-hand side
# ----------------------------------------------------------------------------
class DenseProblem:
    """Parameters and operators of eq. FP2 on the full grid."""

    def __init__(self, ndims, M, omega, k_react, nu_phi, gamma=0.0, U=None, G=None, Omega=None):
        """G, Omega: optional (M, M, M) x-fields of the flow case (section
        "Materials and Methods"): the total diffusivity gamma + gamma_SGS, which
        replaces the constant gamma in the expanded variable-coefficient form
        G D2_i f + (D1_i G)(D1_i f), and the LMSE frequency Omega_mix(x), which
        replaces the constant omega."""
        if ndims not in (2, 5):
            raise ValueError("ndims must be 2 or 5")
        self.ndims, self.M = ndims, M
        self.omega, self.k_react, self.nu_phi, self.gamma = omega, k_react, nu_phi, gamma
        self.U = U  # list of three (M, M, M) arrays or None
        self.G, self.Omega = G, Omega
        if (G is not None or Omega is not None) and ndims != 5:
            raise ValueError("x-fields need a 5-D problem")
        if ndims == 5 and U is None:
            raise ValueError("5-D problem needs a velocity field")
        self.D1g, self.D2g = d1_ghost(M), d2_ghost(M)
        self.D1p, self.D2p = d1_periodic(M), d2_periodic(M)
        phi = phi_nodes(M)
        shp1 = [M] + [1] * (ndims - 1)
        shp2 = [1, M] + [1] * (ndims - 2)
        self.phi = (phi.reshape(shp1), phi.reshape(shp2))
        self.h = 1.0 / M

    # <Phi_a>(x) = h^2 sum_{phi1, phi2} phi_a f   (raw integral)
    def mean_field(self, f, a):
        return self.h**2 * np.sum(self.phi[a] * f, axis=(0, 1), keepdims=True)

    def rhs(self, f):
        out = np.zeros_like(f)
        p1, p2 = self.phi
        react = self.k_react * p1 * p2 * f
        om = self.omega if self.Omega is None else self.Omega[None, None]
        for a in (0, 1):
            m = self.mean_field(f, a)
            flux = om * (self.phi[a] - m) * f + react
            out += apply_axis(self.D1g, flux, a)
            out += self.nu_phi * apply_axis(self.D2g, f, a)
        if self.ndims == 5:
            for i in range(3):
                Ui = self.U[i][None, None]
                d1f = apply_axis(self.D1p, f, 2 + i)
                out -= Ui * d1f
                if self.G is None:
                    out += self.gamma * apply_axis(self.D2p, f, 2 + i)
                else:
                    dG = apply_axis(self.D1p, self.G, i)[None, None]
                    out += self.G[None, None] * apply_axis(self.D2p, f, 2 + i) + dG * d1f
        return out

    def rhs_tangent(self, f, df, param=None):
        if self.G is not None or self.Omega is not None:
            raise NotImplementedError("derivatives are defined for constant coefficients")
        """Directional derivative of rhs at (f, theta) along (df, e_param):
        the right-hand side linearised in f (the mean composition m_a depends
        on f, so d(m_a f) = m_a df + m_a(df) f) applied to df, plus the partial
        derivative with respect to the parameter "omega" or "k_react" (None:
        no parameter direction)."""
        out = np.zeros_like(f)
        p1, p2 = self.phi
        for a in (0, 1):
            m = self.mean_field(f, a)
            dm = self.mean_field(df, a)
            dflux = self.omega * ((self.phi[a] - m) * df - dm * f) + self.k_react * p1 * p2 * df
            if param == "omega":
                dflux = dflux + (self.phi[a] - m) * f
            elif param == "k_react":
                dflux = dflux + p1 * p2 * f
            elif param is not None:
                raise ValueError(param)
            out += apply_axis(self.D1g, dflux, a)
            out += self.nu_phi * apply_axis(self.D2g, df, a)
        if self.ndims == 5:
            for i in range(3):
                Ui = self.U[i][None, None]
                out -= Ui * apply_axis(self.D1p, df, 2 + i)
                out += self.gamma * apply_axis(self.D2p, df, 2 + i)
        return out

    def step_tangent(self, f, df, dt, param=None, integrator="rk4"):
        """One step and its derivative: returns (f+, df+) with df+ the
        derivative of the explicit Runge-Kutta map along (df, e_param), stage
        by stage in the order of the step."""
        L, dL = self.rhs, self.rhs_tangent
        if integrator == "rk4":
            k1, d1 = L(f), dL(f, df, param)
            g, dg = f + 0.5 * dt * k1, df + 0.5 * dt * d1
            k2, d2 = L(g), dL(g, dg, param)
            g, dg = f + 0.5 * dt * k2, df + 0.5 * dt * d2
            k3, d3 = L(g), dL(g, dg, param)
            g, dg = f + dt * k3, df + dt * d3
            k4, d4 = L(g), dL(g, dg, param)
            return (f + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4),
                    df + dt / 6.0 * (d1 + 2 * d2 + 2 * d3 + d4))
        if integrator == "rk2":
            k1, d1 = L(f), dL(f, df, param)
            g, dg = f + dt * k1, df + dt * d1
            k2, d2 = L(g), dL(g, dg, param)
            return f + 0.5 * dt * (k1 + k2), df + 0.5 * dt * (d1 + d2)
        raise ValueError(integrator)

    def with_params(self, **kw):
        """Copy with some of omega / k_react / nu_phi / gamma replaced."""
        q = DenseProblem(self.ndims, self.M, kw.get("omega", self.omega), kw.get("k_react", self.k_react),
                         kw.get("nu_phi", self.nu_phi), kw.get("gamma", self.gamma), self.U)
        return q

    def step(self, f, dt, integrator="rk4"):
        L = self.rhs
        if integrator == "rk4":
            k1 = L(f)
            k2 = L(f + 0.5 * dt * k1)
            k3 = L(f + 0.5 * dt * k2)
            k4 = L(f + dt * k3)
            return f + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
        if integrator == "rk2":
            k1 = L(f)
            k2 = L(f + dt * k1)
            return f + 0.5 * dt * (k1 + k2)
        raise ValueError(integrator)

    # ---------------- observables ----------------
    def norm_field(self, f):
        """<1>(x) = h^2 sum_phi f  (should equal one everywhere)."""
        return self.h**2 * np.sum(f, axis=(0, 1))

    def observables(self, f):
        """Space averages (eq. spaceAvg), R12 (eq. RACov), Y12 (eq. SGSCov)."""
        h = self.h
        nx = self.ndims - 2
        xavg = (lambda g: np.mean(g)) if nx > 0 else (lambda g: float(np.asarray(g).reshape(-1)[0]))
        p1, p2 = self.phi
        m1 = h**2 * np.sum(p1 * f, axis=(0, 1))
        m2 = h**2 * np.sum(p2 * f, axis=(0, 1))
        m12 = h**2 * np.sum(p1 * p2 * f, axis=(0, 1))
        mass = h**2 * np.sum(f, axis=(0, 1))
        out = {
            "mass": xavg(mass),
            "mean1": xavg(m1),
            "mean2": xavg(m2),
            "mean12": xavg(m12),
            "R12": xavg(m1 * m2) - xavg(m1) * xavg(m2),
            "Y12": xavg(m12 - m1 * m2),
            "product": xavg(mass - m1 - m2),
        }
        return out


def dense_from_terms(terms, ndims, M):
    """Sum of separable terms (coeff, [vec or None per dim]) on the full grid."""
    f = np.zeros((M,) * ndims)
    for c, vecs in terms:
        t = np.array(c, dtype=np.float64)
        for d in range(ndims):
            v = np.ones(M) if vecs[d] is None else np.asarray(vecs[d], dtype=np.float64)
            t = np.multiply.outer(t, v)
        f += t
    return f
