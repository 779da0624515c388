"""Seeded synthetic workloads for the QTT Fokker-Planck time step.

This package is the ONE piece shared by the CPU oracle (``oracle/``) and the
HIP product path (``paper_2407_09169_amd``).  It holds no arithmetic of the
method: it only defines problem sizes and parameters and draws the seeded
numbers (1-D sample vectors of the initial PDF and of the velocity field, and
the Gaussian sketch cores used by randomized rounding).  Each side builds its
own tensor-train representation from these numbers.
"""
from .configs import WORKLOADS, Workload, batch_workloads, get_workload, stable_dt  # noqa: F401
from .generate import (  # noqa: F401
    phi_points, x_points, ic_terms, velocity_terms, sketch_ranks, sketch_cores,
    mean_sketch_ranks, mean_sketch_cores, left_sketch_cores, left_mean_sketch_cores, site_order,
    flow_field_terms,
)
