"""Problem sizes and physical parameters of the synthetic workloads.

Units follow the paper's flow case with l0 = u0 = T0 = 1, so the Peclet number
Pe = 1e3 gives the molecular diffusivity gamma = 1e-3, the Damkohler number is
the reaction rate k_react, and the artificial composition-space dissipation is
nu_phi = C_Omega * mu with mu = 4e-3 (Materials and Methods, "Flow case
definition" and "Finite-difference discretisation", eq. FP2).

Dimension order is always phi1, phi2, then x1, x2, x3 (section "Matrix product
state encoding").  ``ordering`` selects how the bits of the dimensions are laid
out along the chain: "serial" puts all bits of phi1 first, then phi2, ... (the
paper's choice); "interleaved" alternates bit b of every dimension.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass


@dataclass(frozen=True)
class Workload:
    name: str
    ndims: int                 # 2 (phi1, phi2) or 5 (phi1, phi2, x1, x2, x3)
    bits: int                  # M = 2**bits grid points per dimension
    ordering: str              # "serial" | "interleaved"
    chi: int                   # maximum MPS bond dimension
    oversample: int = 16       # sketch rank ell = chi + oversample
    chi_mean: int = 16         # bond cap of the mean-composition x-field
    oversample_mean: int = 8
    vel_rank: int = 8          # bond cap of each velocity component
    omega: float = 1.0         # Omega_mix (constant)
    k_react: float = 0.0       # reaction rate C_r (= Da in these units)
    nu_phi: float = 4e-3       # C_Omega * mu
    gamma: float = 1e-3        # gamma = 1/Pe (constant diffusivity)
    integrator: str = "rk4"    # "rk4" | "rk2" (Heun)
    dt: float = 1e-4
    steps: int = 100
    seed: int = 0
    ic: str = "seeded"         # "seeded" | "paper" (exact eq. initPDF / eq. velField)
    rel_tol: float = 0.0       # > 0: also drop singular values below rel_tol * sigma_1

    @property
    def M(self) -> int:
        return 1 << self.bits

    @property
    def n_sites(self) -> int:
        return self.ndims * self.bits

    @property
    def n_phi_sites(self) -> int:
        return 2 * self.bits

    @property
    def n_x_sites(self) -> int:
        return (self.ndims - 2) * self.bits

    @property
    def ell(self) -> int:
        return self.chi + self.oversample

    @property
    def ell_mean(self) -> int:
        return self.chi_mean + self.oversample_mean

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


_W = [
    # 2-D composition PDF, M = 64, 12 interleaved cores, chi <= 16, RK4 dt = 1e-4, 100 steps.
    Workload("c1_2d_M64", ndims=2, bits=6, ordering="interleaved", chi=16, oversample=16,
             omega=1.0, k_react=0.0, nu_phi=4e-3, gamma=0.0, integrator="rk4",
             dt=1e-4, steps=100, seed=0),
    # Same, untruncated (chi = 2**6 covers every bond of a 12-core chain).
    Workload("c1_2d_M64_exact", ndims=2, bits=6, ordering="interleaved", chi=64, oversample=0,
             omega=1.0, k_react=0.0, nu_phi=4e-3, gamma=0.0, integrator="rk4",
             dt=1e-4, steps=100, seed=0),
    # 5-D PDF, M = 128, 35 serial cores, chi = 64, 200 RK4 steps.
    Workload("c2_5d_M128_chi64", ndims=5, bits=7, ordering="serial", chi=64, oversample=16,
             omega=1.0, k_react=0.0, dt=1e-3, steps=200, seed=1),
    # 5-D PDF, M = 1024, 50 serial cores, chi = 128 / 256, reaction k = 10.
    Workload("c3_5d_M1024_chi128", ndims=5, bits=10, ordering="serial", chi=128, oversample=16,
             chi_mean=8, omega=1.0, k_react=10.0, dt=3e-5, steps=50, seed=2),
    Workload("c3_5d_M1024_chi256", ndims=5, bits=10, ordering="serial", chi=256, oversample=32,
             chi_mean=8, omega=1.0, k_react=10.0, dt=3e-5, steps=50, seed=2),
    # 5-D PDF, M = 256, 40 serial cores, chi = 64: gradients of the final product mean
    # with respect to Omega and k over 200 RK4 steps.
    Workload("c5_5d_M256_chi64", ndims=5, bits=8, ordering="serial", chi=64, oversample=16,
             chi_mean=16, omega=1.0, k_react=10.0, dt=2e-4, steps=200, seed=5),
    # Small 5-D cases that a dense full-grid solver can follow (tests).
    Workload("t_5d_M8_exact", ndims=5, bits=3, ordering="serial", chi=128, oversample=0,
             chi_mean=64, oversample_mean=0, vel_rank=64,
             omega=1.0, k_react=10.0, dt=2e-3, steps=10, seed=3),
    Workload("t_5d_M8_chi16", ndims=5, bits=3, ordering="serial", chi=16, oversample=8,
             chi_mean=8, oversample_mean=8, vel_rank=8,
             omega=1.0, k_react=10.0, dt=2e-3, steps=10, seed=3),
    Workload("t_5d_M16_chi32", ndims=5, bits=4, ordering="serial", chi=32, oversample=16,
             chi_mean=16, oversample_mean=8,
             omega=1.0, k_react=10.0, dt=1e-3, steps=4, seed=4),
    Workload("t_2d_M64_serial", ndims=2, bits=6, ordering="serial", chi=8, oversample=8,
             omega=1.0, k_react=5.0, nu_phi=4e-3, gamma=0.0, dt=1e-4, steps=20, seed=5),
]

WORKLOADS = {w.name: w for w in _W}


def get_workload(name: str, **overrides) -> Workload:
    w = WORKLOADS[name]
    return w.replace(**overrides) if overrides else w


# Upper bound of |<U_i>| for the seeded velocity family (a1, a2 in [0.5, 1.5],
# a3 = -(a1 + a2), unit jet): |U1| <= 2.5, |U2| <= 1.5, |U3| <= 3.
U_MAX = 3.0


def stable_dt(ndims: int, bits: int, omega: float, k_react: float, nu_phi: float = 4e-3,
              gamma: float = 1e-3, safety: float = 0.5) -> float:
    """Explicit RK4 step from a Gershgorin bound of the spectral radius of the
    discrete operator: rho = sum over the two composition axes of
    (4 nu_phi / h^2 + (Omega + k) / h) plus, in 5-D, sum over the three
    physical axes of (4 Gamma / h^2 + U_max / h); dt = safety * 2.78 / rho
    (2.78 is where RK4's stability region meets the negative real axis)."""
    h = 1.0 / (1 << bits)
    rho = 2 * (4.0 * nu_phi / h ** 2 + (omega + k_react) / h)
    if ndims == 5:
        rho += 3 * (4.0 * gamma / h ** 2 + U_MAX / h)
    return safety * 2.78 / rho


def batch_workloads(count: int = 64, seed: int = 4, bits=(6, 7, 8, 9), chis=(16, 32, 64, 128),
                    omega=(0.5, 4.0), k_react=(1.0, 50.0)) -> list:
    """The batched ensemble of 5-D problems: instance i draws its grid level
    (bits), bond cap chi, Omega and k from the seeded generator [seed, i] and
    uses seed 1000 + i for its own initial PDF, velocity and sketches; dt
    follows stable_dt."""
    import numpy as np
    out = []
    for i in range(count):
        rng = np.random.default_rng([seed, i])
        b = int(rng.choice(bits))
        chi = int(rng.choice(chis))
        om = float(rng.uniform(*omega))
        k = float(rng.uniform(*k_react))
        out.append(Workload(f"batch{i:02d}_M{1 << b}_chi{chi}", ndims=5, bits=b, ordering="serial",
                            chi=chi, oversample=16, chi_mean=min(16, chi), oversample_mean=8,
                            omega=om, k_react=k, dt=stable_dt(5, b, om, k), steps=20,
                            seed=1000 + i))
    return out
