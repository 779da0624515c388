"""The flow case's accuracy protocol (section "Materials and Methods", "Moment
equations" and "Error measures"): the MPS solution of eq. FP2 and the moment
equation eq. FPMoms advanced side by side, sampled at equally spaced times,
and reduced to the four RMSE measures of eq. RMSE0.

Every step runs in the HIP library: the MPS step (tt_step), the composition
moments of the state as x-MPSs and their dense evaluation (tt_moment_field,
tt_to_dense), the moment equation (fd_moment_steps), the squared-difference
sums (fd_sq_diff_sum) and the final measures (flow_error_measures).  This
module only sequences the calls and holds device tensors.

The moment equation sees the same velocity as the MPS problem (its velocity
MPSs evaluated on the grid) and the same diffusivity (the constant gamma, or
the problem's x-field G(x) evaluated on the grid); its initial condition is
the first composition moment of the initial PDF.  Exact means exist only without reaction (Da =
0); with reaction the measure Error_2b down is NaN.
"""
from __future__ import annotations

import numpy as np

from . import (TT_SERIAL, axpby, from_dense, from_separable, error_measures, moment_steps,
               setup_workload, smagorinsky, sq_diff_sum, to_dense)

C_S = 0.11  # Smagorinsky constant of the flow case


def smagorinsky_fields(ctx, w, chi_field, c_omega=1.0):
    """The paper's closure fields as x-MPSs: G = gamma + gamma_SGS from the
    velocity of w (its velocity MPSs on the grid, Delta = 3 / M) by
    fd_smagorinsky, cut to chi_field by tt_from_dense, and Omega_mix =
    C_Omega G / Delta^2.  Returns ({"G": TT, "Omega": TT}, discarded weight
    of G, the dense G of the cut MPS)."""
    import torch
    import workloads
    bits, M = w.bits, w.M
    n = M ** 3
    dev = torch.device("cuda", ctx.device)
    U = torch.empty(3 * n, dtype=torch.float64, device=dev)
    for i, comp in enumerate(workloads.velocity_terms(w)):
        v = from_separable(ctx, 3, bits, TT_SERIAL, comp, w.vel_rank)
        to_dense(ctx, v, U[i * n:(i + 1) * n])
        v.free()
    delta = 3.0 / M
    G = torch.empty(n, dtype=torch.float64, device=dev)
    smagorinsky(ctx, bits, U, G, C_S, delta, w.gamma)
    g, disc = from_dense(ctx, G, chi_field)
    om = axpby(ctx, [c_omega / (delta * delta)], [g])
    to_dense(ctx, g, G)
    return {"G": g, "Omega": om}, disc, G


def run(ctx, w, n_samples=17, steps_per_sample=1, dtype="f64", exact=None, fields=False,
        chi_field=16, c_omega=1.0, on_sample=None, sketch_seed=None):
    """Advances workload w (5-D) for (n_samples - 1) * steps_per_sample steps,
    sampling at every steps_per_sample steps from t = 0.

    Returns a dict with the four measures ("E2b_up", "E2b_down", "E2c_up",
    "E2c_down") and the per-sample series they come from: "mean_bar" (2, T),
    "sq_mean_x" (2, T) and "sq_norm_x" (T) (grid means of the squared
    differences).  exact: None (solve the moment equation when k_react == 0)
    or False (skip it).  fields=True runs the problem with the seeded x-fields
    G(x) and Omega(x) (setup_workload), fields="smagorinsky" with the paper's
    closure (smagorinsky_fields, G cut to chi_field, Omega = c_omega G /
    Delta^2); the moment equation then uses the same G(x).  on_sample(t, T),
    if given, is called after sample t of T has been taken; sketch_seed draws
    the Gaussian sketches from another seed (setup_workload)."""
    import torch
    import workloads

    if w.ndims != 5:
        raise ValueError("the flow case is 5-D")
    if exact is None:
        exact = w.k_react == 0.0
    bits, M = w.bits, w.M
    n = M ** 3
    dev = torch.device("cuda", ctx.device)
    G_closure = None
    fdisc = None
    if fields == "smagorinsky":
        fx, fdisc, G_closure = smagorinsky_fields(ctx, w, chi_field, c_omega)
        prob, f = setup_workload(ctx, w, dtype, fields=fx, sketch_seed=sketch_seed)
    else:
        prob, f = setup_workload(ctx, w, dtype, fields=fields, sketch_seed=sketch_seed)
    phi = (np.arange(M) + 0.5) / M
    dense = torch.empty(n, dtype=torch.float64, device=dev)
    m = work = U = G = None
    if exact:
        U = torch.empty(3 * n, dtype=torch.float64, device=dev)
        for i, comp in enumerate(workloads.velocity_terms(w)):
            v = from_separable(ctx, 3, bits, TT_SERIAL, comp, w.vel_rank)
            to_dense(ctx, v, U[i * n:(i + 1) * n])
            v.free()
        G = torch.full((n,), w.gamma, dtype=torch.float64, device=dev)
        if G_closure is not None:
            G = G_closure
        elif fields:
            g = from_separable(ctx, 3, bits, TT_SERIAL, workloads.flow_field_terms(w)["G"], 16)
            to_dense(ctx, g, G)
            g.free()
        m = torch.empty(2 * n, dtype=torch.float64, device=dev)
        work = torch.empty(2 * n, dtype=torch.float64, device=dev)
        for a in range(2):
            x = prob.moment_field(f, phi if a == 0 else None, phi if a == 1 else None)
            to_dense(ctx, x, m[a * n:(a + 1) * n])
            x.free()
    T = n_samples
    mean_bar = np.zeros((2, T))
    sq_mean_x = np.zeros((2, T))
    sq_norm_x = np.zeros(T)
    for t in range(T):
        if t > 0:
            prob.step(f, steps_per_sample)
            if exact:
                moment_steps(ctx, bits, U, G, m, work, w.dt, steps_per_sample)
        mean_bar[0, t] = prob.observable(f, "mean1")
        mean_bar[1, t] = prob.observable(f, "mean2")
        x = prob.moment_field(f, None, None)
        to_dense(ctx, x, dense)
        x.free()
        sq_norm_x[t] = sq_diff_sum(ctx, dense, None, 1.0) / n
        if exact:
            for a in range(2):
                x = prob.moment_field(f, phi if a == 0 else None, phi if a == 1 else None)
                to_dense(ctx, x, dense)
                x.free()
                sq_mean_x[a, t] = sq_diff_sum(ctx, dense, m[a * n:(a + 1) * n]) / n
        if on_sample is not None:
            on_sample(t, T)
    e = error_measures(mean_bar, sq_mean_x if exact else None, sq_norm_x)
    _, max_bond = prob.info()
    f.free()
    prob.close()
    return {"E2b_up": e[0], "E2b_down": e[1], "E2c_up": e[2], "E2c_down": e[3],
            "mean_bar": mean_bar, "sq_mean_x": sq_mean_x if exact else None,
            "sq_norm_x": sq_norm_x, "field_discarded": fdisc, "max_mpo_bond": max_bond}
