"""QTT Fokker-Planck time steps per second on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype bf16|f32|f64]
                    [--workload c3_5d_M1024_chi128] [--no-cpu-baseline]

A step is one full RK4 step (4 stage evaluations with their mean-field
updates and roundings, plus the rounded stage combination) of the 5-D PDF on
the 1024^5 grid (50 quantics cores) at chi = 128, with synthetic seeded
inputs (workloads.c3_5d_M1024_chi128).  Inputs are resident in HBM before the
timed region.  The MFMA path (FP32 by default) and the plain FP64 path run the
same schedule from the same initial state; the line reports the MFMA path's
steps/s as `value`, the FP64 path's steps/s and the L2 distance between the
two states after the run.  Four more timed regions of K steps continue the
same trajectory afterwards (`repeats_steps_per_s`, `median_steps_per_s`): the
Jacobi sweeps of the truncations, and with them the step time, grow as the
state evolves.

Other workloads print their own line: batch64 (64 uneven problems stepped
together), --gradient (steps carrying parameter derivatives), fpmoms_M<M>
(the moment equation on an M^3 grid), flow_c2_5d_M128_chi64 (the flow
case's accuracy protocol on the 128^5 grid), prolong_smag_M1024 (the closure
field on 1024^3 by prolongation against the direct TT-SVD), --drift
(precision over 200 steps) and --chi-mean-study.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QTT time steps/sec, 5D PDF chi=128 (MFMA FP32/BF16 vs FP64 plain) at L2 err"
PEAKS_TFLOPS = {"bf16": 2500.0, "f32": 157.3, "f64": 78.6}
N_CU = 256  # compute units of an MI355X
HBM_GBS = 8000.0


def _time_steps(torch, prob, f, K):
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    prob.step(f, K)
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1)


KERNEL_SOURCES = {"qr_": "factor.hip", "eig_": "factor.hip", "tc_": "tc_gemm.hip",
                  "moment_": "moments.hip"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.txt")


def _source_hash(kernel):
    """sha1 (first 12 hex digits) of the source file that holds `kernel`."""
    import hashlib
    for prefix, src in KERNEL_SOURCES.items():
        if kernel.startswith(prefix):
            path = os.path.join(ROOT, "paper_2407_09169_amd", "csrc", src)
            return hashlib.sha1(open(path, "rb").read()).hexdigest()[:12]
    return None


def _traffic(kernel, shape):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by the plain-copy
    calibration) recorded in profiles/traffic.txt for this kernel and shape,
    or None when absent or taken on a different version of its source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    h = _source_hash(kernel)
    for line in open(TRAFFIC_FILE):
        if line.startswith("#") or not line.strip():
            continue
        parts = line.rstrip("\n").split("\t")
        if len(parts) >= 5 and parts[0] == kernel and parts[1] == shape and parts[4] == h:
            return float(parts[2]) + float(parts[3])
    return None


def _op_log(prob, f):
    """One eager step with a pair of HIP events around every launch, on the
    stream of its lane; returns [(index, class, ms, flops, bytes, description,
    lane)], lane fork / join events included (class -2, no time)."""
    import tempfile
    fd, path = tempfile.mkstemp(suffix=".txt")
    os.close(fd)
    os.environ["QTTPDF_PROFILE_LOG"] = path
    try:
        prob.profile(f, 1, "all")
    finally:
        del os.environ["QTTPDF_PROFILE_LOG"]
    rows = []
    for line in open(path):
        i, k, ms, fl, by, what, lane = line.rstrip("\n").split("\t")
        rows.append((int(i), int(k), float(ms), float(fl), float(by), what, int(lane)))
    os.unlink(path)
    return rows


def _roofline(rows):
    """Roofline of the dominant kernel: the (kernel, shape) group with the
    most event time in one step; achieved = its algorithmic flops (bytes) per
    launch / its average launch duration."""
    groups = {}
    for _, k, ms, fl, by, what, _lane in rows:
        if k < 0:  # copies, fills and lane events are not kernels of the method
            continue
        g = groups.setdefault(what, [0, 0.0, 0.0, 0.0])
        g[0] += 1
        g[1] += ms
        g[2] += fl
        g[3] += by
    what = max(groups, key=lambda w: groups[w][1])
    n, ms, fl, by = groups[what]
    kernel, shape = what.split("|", 1) if "|" in what else (what, "")
    avg_s = ms / n / 1e3
    if kernel.startswith("tc_mfma_kernel<false"):
        roof = {"bound": "mfma", "achieved": fl / n / avg_s / 1e12, "peak": PEAKS_TFLOPS["f32"], "unit": "TFLOP/s"}
    elif kernel.startswith("tc_mfma_kernel<true"):
        roof = {"bound": "mfma", "achieved": fl / n / avg_s / 1e12, "peak": PEAKS_TFLOPS["bf16"], "unit": "TFLOP/s"}
    elif fl > 0:
        roof = {"bound": "alu", "achieved": fl / n / avg_s / 1e12, "peak": PEAKS_TFLOPS["f64"], "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": by / n / avg_s / 1e9, "peak": HBM_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = _traffic(kernel, shape)
    roof["kernel"] = kernel
    roof["shape"] = shape
    roof["launches_per_step"] = n
    roof["avg_launch_us"] = 1e6 * avg_s
    roof["algorithmic_per_launch"] = (fl / n) if fl > 0 else (by / n)
    roof["share_of_step_kernel_time"] = ms / sum(r[2] for r in rows)
    if kernel.startswith(("qr_", "eig_")) and kernel != "qr_blocked":
        # one workgroup (one CU) per matrix: the fraction of the peak of the
        # CUs such a launch occupies (the blocked QR spreads over the chip)
        m = re.match(r"b(\d+) ", shape)
        cus = int(m.group(1)) if m else 1
        if kernel.startswith("qr_q_kernel"):  # workgroups of 4 columns of Q
            cus = -(-int(re.search(r"n(\d+)", shape).group(1)) // 4)
        roof["cus_per_launch"] = cus
        roof["frac_of_cus_used"] = roof["achieved"] / (roof["peak"] * cus / N_CU)
    return roof


def _classes(rows):
    names = {0: "contract", 1: "qr", 2: "eig", 3: "stream", -1: "other"}
    out = {}
    for _, k, ms, fl, by, _w, _lane in rows:
        if k == -2:  # lane fork / join
            continue
        c = out.setdefault(names.get(k, "other"), {"ms": 0.0, "launches": 0, "flops": 0.0, "bytes": 0.0})
        c["ms"] += ms
        c["launches"] += 1
        c["flops"] += fl
        c["bytes"] += by
    return out


def _kernel_probe(spec):
    """One factorisation kernel alone, on the shape the step uses (counter
    runs): qr:MxN (one matrix, as in the sweeps) or eig:N (a batch of 49
    Gram-like PSD matrices with eigenvalues over 20 decades, as in a
    truncation)."""
    import numpy as np
    import paper_2407_09169_amd as q
    kind, shape = spec.split(":")
    ctx = q.Context(0)
    rng = np.random.default_rng(0)
    if kind == "qr":
        m, n = (int(v) for v in shape.lower().split("x"))
        A = rng.standard_normal((1, m, n))
        for _ in range(5):
            q.linalg_qr(ctx, A, with_r=False)
    elif kind == "eig":
        n = int(shape)
        Q, _ = np.linalg.qr(rng.standard_normal((49, n, n)))
        lam = 10.0 ** (-20.0 * np.arange(n) / (n - 1))
        G = np.einsum("bij,j,bkj->bik", Q, lam, Q)
        for _ in range(5):
            q.linalg_eigh(ctx, G, min(n, 128))
    else:
        raise SystemExit(f"unknown kernel probe {kind}")
    print(json.dumps({"kernel_probe": spec, "dispatches": 5}))


def _bench_batched(args, log):
    """The batched ensemble (64 uneven 5-D problems, FP32-MFMA contractions):
    instance-steps/s of the instances stepped together (one call per step;
    instances of equal structure fused into shared launches, the units on
    parallel branches), next to the same instances stepped one after
    another."""
    import torch
    import paper_2407_09169_amd as q
    import workloads
    ws = workloads.batch_workloads(count=64)
    ctx = q.Context(0)
    t0 = time.perf_counter()
    inst = [q.setup_workload(ctx, w, args.dtype) for w in ws]
    b = q.Batch(ctx, [p for p, _ in inst], [f for _, f in inst])
    binfo = b.info()
    log(f"batch of {len(ws)} set up in {time.perf_counter() - t0:.1f} s ({binfo}); warmup {args.warmup}")
    b.step(args.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.step(args.steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    value = len(ws) * args.steps / (ms / 1e3)
    log(f"batched: {args.steps} steps of {len(ws)} instances in {ms:.1f} ms ({value:.1f} instance-steps/s)")
    masses = [p.observable(f, "mass") for p, f in inst]
    b.close()  # releases the batch plan before the instances record their own
    if args.no_plain:  # the batch alone
        print(json.dumps({"metric": "instance-steps/s, 64 uneven 5-D QTT PDF problems stepped together",
                          "value": value, "unit": "instance-steps/s", "ms_per_step": ms / args.steps,
                          "batch": binfo}))
        return
    # one after another: each instance records its own graph, is timed over
    # one step, and releases its plan (all 64 step plans at once would not fit)
    ms1 = 0.0
    for p, f in inst:
        p.step(f, 1)
        torch.cuda.synchronize()
        e0.record()
        p.step(f, 1)
        e1.record()
        torch.cuda.synchronize()
        ms1 += e0.elapsed_time(e1)
        p.close()
    seq = len(ws) / (ms1 / 1e3)
    log(f"one after another: {seq:.1f} instance-steps/s")
    out = {
        "metric": "instance-steps/s, 64 uneven 5-D QTT PDF problems stepped together",
        "value": value, "unit": "instance-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": "batch64", "instances": len(ws),
                   "grid_levels": sorted({w.M for w in ws}), "chis": sorted({w.chi for w in ws}),
                   "total_cores": sum(w.n_sites for w in ws), "integrator": "rk4"},
        "sequential_instance_steps_per_s": seq,
        "batching_speedup": value / seq,
        "batch": binfo,
        "mass_range": [min(masses), max(masses)],
    }
    print(json.dumps(out))


def _bench_moments(args, log):
    """The moment equation of the flow case (eq. FPMoms at Da = 0, RK2-CFD2)
    for both mean compositions on an M^3 grid with the Smagorinsky
    diffusivity of eq. velField's flow: RK2 steps/s, and the roofline of the
    stage kernel.  Algorithmic bytes per grid point and step: the first stage
    reads the two fields, U (3 values) and G and writes two fields (8 values,
    64 bytes); the second also reads the two base fields (10 values, 80
    bytes)."""
    import numpy as np
    import torch
    import paper_2407_09169_amd as q
    import workloads
    bits = int(round(np.log2(int(args.workload.split("_M")[1]))))
    M, n = 1 << bits, 1 << (3 * bits)
    w = workloads.get_workload("t_5d_M8_chi16", bits=bits, ic="paper")
    ctx = q.Context(0)
    dev = torch.device("cuda", 0)
    U = torch.zeros((3, M, M, M), dtype=torch.float64, device=dev)
    one = torch.ones(M, dtype=torch.float64, device=dev)
    for i, comp in enumerate(workloads.velocity_terms(w)):
        for c, vecs in comp:
            v = [one if x is None else torch.as_tensor(x, device=dev) for x in vecs]
            U[i] += c * v[0][:, None, None] * v[1][None, :, None] * v[2][None, None, :]
    G = torch.empty(n, dtype=torch.float64, device=dev)
    delta = 3.0 / M
    q.smagorinsky(ctx, bits, U.view(-1), G, 0.11, delta, 1e-3)
    gen = torch.Generator(device=dev)
    gen.manual_seed(17)
    m = torch.rand(2 * n, dtype=torch.float64, device=dev, generator=gen)
    work = torch.empty_like(m)
    gmax = float(G.max())
    dt = 0.2 / (M * M * gmax * 6 + M * 4)
    q.moment_steps(ctx, bits, U.view(-1), G, m, work, dt, args.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    q.moment_steps(ctx, bits, U.view(-1), G, m, work, dt, args.steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    value = args.steps / (ms / 1e3)
    per_launch_bytes = (64 + 80) / 2 * n
    kernel = "moment_stage_col_kernel<2>" if bits >= 8 else "moment_stage_kernel<2>"
    avg_us = ms * 1e3 / (2 * args.steps)
    achieved = per_launch_bytes / (avg_us * 1e-6) / 1e9
    log(f"moments M={M}: {args.steps} RK2 steps in {ms:.2f} ms ({value:.1f} steps/s, "
        f"{achieved:.0f} GB/s per stage launch)")
    out = {
        "metric": "moment-equation RK2 steps/s (both mean compositions, Smagorinsky diffusivity)",
        "value": value, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "grid": f"{M}^3", "fields": 2, "dt": dt},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_GBS, "traffic": _traffic(kernel, f"M{M}"),
                     "kernel": kernel, "avg_launch_us": avg_us,
                     "algorithmic_bytes_per_launch": per_launch_bytes,
                     "timing": "events around the timed steps, divided by the launches"},
        "finite": bool(torch.isfinite(m).all()),
    }
    print(json.dumps(out))


def _bench_prolong(args, log):
    """The flow case's Smagorinsky diffusivity as a bond-16 x-MPS on the 1024^3
    grid, prepared two ways: directly (the velocity of eq. velField and the
    closure evaluated on the 1024^3 grid, 2^30 values, then the truncated
    TT-SVD of tt_from_dense) and by prolongation (the same on the 256^3 grid,
    then two tt_prolong refinements).  Wall time of each path (the closure
    field's set-up, not part of a step) and the relative L2 distance between
    the two fields, both with the filter width Delta = 3 / 1024."""
    import torch
    import paper_2407_09169_amd as q
    import workloads
    ctx = q.Context(0)
    dev = torch.device("cuda", 0)
    delta, chi = 3.0 / 1024, 16

    def closure(bits):
        M = 1 << bits
        w = workloads.get_workload("t_5d_M8_chi16", bits=bits, ic="paper")
        U = torch.zeros((3, M, M, M), dtype=torch.float64, device=dev)
        one = torch.ones(M, dtype=torch.float64, device=dev)
        for i, comp in enumerate(workloads.velocity_terms(w)):
            for c, vecs in comp:
                v = [one if x is None else torch.as_tensor(x, device=dev) for x in vecs]
                U[i] += c * v[0][:, None, None] * v[1][None, :, None] * v[2][None, None, :]
        G = torch.empty(M ** 3, dtype=torch.float64, device=dev)
        q.smagorinsky(ctx, bits, U.view(-1), G, 0.11, delta, 1e-3)
        del U
        return G

    for rep in range(2):  # the first pass pages in the kernels
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        G = closure(10)
        direct, d_direct = q.from_dense(ctx, G, chi)
        torch.cuda.synchronize()
        t_direct = time.perf_counter() - t0
        del G
        torch.cuda.empty_cache()
        t0 = time.perf_counter()
        G = closure(8)
        coarse, d_coarse = q.from_dense(ctx, G, chi)
        y1, d1 = q.prolong(ctx, coarse, 3, 8, chi)
        y2, d2 = q.prolong(ctx, y1, 3, 9, chi)
        torch.cuda.synchronize()
        t_prolong = time.perf_counter() - t0
        del G
    diff = q.l2_diff(ctx, y2, direct)
    log(f"direct {t_direct:.3f} s, prolonged {t_prolong:.3f} s, L2 between them {diff:.3e}")
    out = {"metric": "set-up time of the 1024^3 Smagorinsky x-MPS (bond 16): direct vs prolongation from 256^3",
           "value": t_direct / t_prolong, "unit": "speedup", "n_gpus": 1, "higher_is_better": True,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "prolong_smag_M1024", "chi": chi, "delta": delta, "coarse": "256^3"},
           "direct_s": t_direct, "prolonged_s": t_prolong, "l2_prolonged_vs_direct": diff,
           "discarded": {"direct": d_direct, "coarse": d_coarse, "prolong": d1 + d2}}
    print(json.dumps(out))


def _bench_flow(args, log):
    """The flow case's accuracy protocol on the paper's 128^5 grid: the MPS
    step (chi = 64, RK2, Da = 0, the Smagorinsky diffusivity cut to bond 16 and
    Omega_mix = C_Omega G / Delta^2 with C_Omega = 1) and the
    moment equation advanced side by side from the printed initial PDF and
    velocity (eq. initPDF, eq. velField), 17 samples, the four error measures
    of eq. RMSE0; protocol steps/s over the whole run."""
    import torch
    import paper_2407_09169_amd as q
    from paper_2407_09169_amd import flow
    import workloads
    w = workloads.get_workload("c2_5d_M128_chi64", k_react=0.0, integrator="rk2", ic="paper")
    if args.chi:
        w = w.replace(chi=args.chi)
    if args.dt:
        w = w.replace(dt=args.dt)
    if args.chi_mean:
        w = w.replace(chi_mean=args.chi_mean, oversample_mean=8)
    ctx = q.Context(0)
    k = max(1, args.steps // 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = flow.run(ctx, w, n_samples=17, steps_per_sample=k, dtype=args.dtype, fields="smagorinsky",
                 chi_field=16, c_omega=1.0,
                 on_sample=lambda t, T: log(f"flow sample {t + 1}/{T} at step {t * k}"),
                 sketch_seed=args.sketch_seed)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    steps = 16 * k
    log(f"flow protocol 128^5 chi={w.chi} chi_mean={w.chi_mean}: {steps} steps and 17 samples in {sec:.2f} s; "
        f"E2b up {r['E2b_up']:.3e} down {r['E2b_down']:.3e}, E2c up {r['E2c_up']:.3e} down {r['E2c_down']:.3e}")
    out = {
        "metric": "flow-protocol steps/s (MPS step + moment equation + 17 samples of the error measures)",
        "value": steps / sec, "unit": "steps/s", "n_gpus": 1, "steps": steps, "warmup": 0,
        "ms_per_step": 1e3 * sec / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": "flow_c2_5d_M128_chi64", "grid": "128^5", "chi": w.chi,
                   "integrator": "rk2", "k_react": 0.0, "dt": w.dt, "samples": 17, "chi_mean": w.chi_mean,
                   "steps_per_sample": k, "sketch_seed": w.seed if args.sketch_seed is None else args.sketch_seed,
                   "autotune": os.environ.get("QTTPDF_AUTOTUNE", "1")[:1] != "0",
                   "fields": "Smagorinsky G(x) (C_s 0.11, Delta 3/M, bond 16), Omega = G / Delta^2",
                   "initial_state": "eq. initPDF, eq. velField"},
        "errors": {"E2b_up": r["E2b_up"], "E2b_down": r["E2b_down"], "E2c_up": r["E2c_up"],
                   "E2c_down": r["E2c_down"]},
        "field_discarded_weight": r["field_discarded"],
        "max_stage_mpo_bond": r["max_mpo_bond"],
        "timing": "wall clock of the whole protocol, set-up and first-step recording included",
    }
    print(json.dumps(out))


def _bench_gradient(args, log):
    """Steps of the gradient workload carrying d f / d Omega and d f / d k
    (tt_step_tangent): gradient-steps/s and the final dJ/dtheta of the
    product mean."""
    import torch
    import paper_2407_09169_amd as q
    import workloads
    name = args.workload if args.workload != "c3_5d_M1024_chi128" else "c5_5d_M256_chi64"
    w = workloads.get_workload(name)
    ctx = q.Context(0)
    prob, f = q.setup_workload(ctx, w, args.dtype)
    tans = {"omega": prob.state(), "k_react": prob.state()}
    n = w.steps
    log(f"{w.name} {args.dtype}: {n} steps with two tangents")
    prob.step_tangent(f, tans, 1)  # records the graph
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    prob.step_tangent(f, tans, n - 1)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    J = prob.observable(f, "product")
    g = {p: prob.observable(t, "product") for p, t in tans.items()}
    log(f"{n - 1} steps in {ms:.1f} ms; J = {J:.6e}, dJ/dOmega = {g['omega']:.6e}, dJ/dk = {g['k_react']:.6e}")
    out = {
        "metric": "RK4 steps/s carrying dJ/dOmega and dJ/dk (forward-mode tangents), 5-D chi=64",
        "value": (n - 1) / (ms / 1e3), "unit": "steps/s", "n_gpus": 1, "steps": n - 1, "warmup": 1,
        "ms_per_step": ms / (n - 1), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": w.name, "grid": f"{w.M}^{w.ndims}", "n_cores": w.n_sites, "chi": w.chi,
                   "statistic": "product mean", "steps_total": n},
        "J": J, "dJ_dOmega": g["omega"], "dJ_dk": g["k_react"],
    }
    print(json.dumps(out))


def _copy_probe(nbytes):
    """A plain device copy of known size (torch's copy kernel), for scaling
    the HBM counters of rocprofv3 runs."""
    import torch
    n = nbytes // 8
    a = torch.rand(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": 8 * n, "dispatches": 5}))


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _cpu_baseline(w):
    """The CPU oracle (numpy / LAPACK, FP64) on bounded samples: one RK4 step
    of the same workload from the same initial state with every BLAS thread
    (the reported value), and, for a number of the kind the paper quotes for
    its single-core runs (the longest of the first steps of a run), the first
    two steps of the 128^5 chi = 64 workload on one thread."""
    from oracle import stepper
    import workloads
    st = stepper.MPSStepper(w)
    f = st.initial_state()
    t0 = time.perf_counter()
    st.step(f)
    el = time.perf_counter() - t0
    cores = os.cpu_count() or 1
    single = None
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max([i.get("num_threads", 1) for i in info] + [1])
        w2 = workloads.get_workload("c2_5d_M128_chi64")
        with threadpoolctl.threadpool_limits(1):
            st2 = stepper.MPSStepper(w2)
            g = st2.initial_state()
            longest = 0.0
            for _ in range(2):
                t1 = time.perf_counter()
                g, _ = st2.step(g)
                longest = max(longest, time.perf_counter() - t1)
        single = {"workload": w2.name, "threads": 1, "steps": 2, "longest_step_s": longest}
    except Exception as e:  # noqa: BLE001
        single = {"error": str(e)}
    return {"value": 1.0 / el, "unit": "steps/s", "cores": cores, "kind": "oracle",
            "cpu_model": _cpu_model(),
            "sample": f"1 RK4 step of {w.name} from the seeded initial state ({el:.1f} s)",
            "single_thread": single}


def _accuracy_series(q, ctx, w, runs, n):
    """Every run of `runs` ({name: (problem, state[, workload])}, "f64" among
    them; a run's own workload, when given, may differ from w in chi or in the
    sketch seeds) is restarted from the seeded initial state and advanced one
    step at a time for n steps; after each step the relative L2 distance of
    each state to the FP64 one (tt_l2_diff) and every run's mass deviation
    <1> - 1 are recorded."""
    import workloads
    ordering = q.TT_SERIAL if w.ordering == "serial" else q.TT_INTERLEAVED
    for r in runs.values():
        wr = r[2] if len(r) > 2 else w
        f0 = q.from_separable(ctx, w.ndims, w.bits, ordering, workloads.ic_terms(w), wr.chi)
        r[1].set_cores(f0.cores())
        f0.free()
    series = {k: {"l2_vs_f64": [], "mass_dev": []} for k in runs}
    f64 = runs["f64"][1]
    for _ in range(n):
        for r in runs.values():
            r[0].step(r[1], 1)
        for k, r in runs.items():
            if k != "f64":
                series[k]["l2_vs_f64"].append(q.l2_diff(ctx, r[1], f64))
            series[k]["mass_dev"].append(r[0].observable(r[1], "mass") - 1.0)
    del series["f64"]["l2_vs_f64"]
    return series


def _bench_chi_mean(args, log):
    """What the bond cap chi_mean of the mean compositions <Phi_a>(x) costs
    and changes: FP64 runs of the 128^5 chi = 64 and 1024^5 chi = 128
    workloads from the same initial state with chi_mean in {8, 16, 32, chi}
    (chi: the raw mean is kept whole), steps/s of each and the relative L2
    distance of each final state to the chi_mean = chi run."""
    import torch
    import paper_2407_09169_amd as q
    import workloads
    ctx = q.Context(0)
    out = {"metric": "chi_mean study: steps/s and L2 distance to the uncapped mean field", "runs": []}
    for name, n in (("c2_5d_M128_chi64", args.steps), ("c3_5d_M1024_chi128", max(2, args.steps // 2))):
        w0 = workloads.get_workload(name)
        states = {}
        for cm in (w0.chi, 8, 16, 32):
            w = w0.replace(chi_mean=cm, oversample_mean=8)
            prob, f = q.setup_workload(ctx, w, "f64")
            _, mb = prob.info()
            prob.step(f, 1)  # records the graph
            ms = _time_steps(torch, prob, f, n)
            states[cm] = (prob, f)
            d = 0.0 if cm == w0.chi else q.l2_diff(ctx, f, states[w0.chi][1])
            row = {"workload": name, "chi_mean": cm, "steps": n + 1, "steps_per_s": n / (ms / 1e3),
                   "l2_vs_uncapped": d, "stage_mpo_bond_x_sites": mb + 2 * cm}
            log(str(row))
            out["runs"].append(row)
        for prob, f in states.values():
            f.free()
            prob.close()
    print(json.dumps(out))


def _bench_drift(args, log):
    """Precision drift over a long run: the 128^5 chi = 64 workload (200 RK4
    steps) in FP32 and BF16 next to FP64 from the same initial state, the
    relative L2 distance to the FP64 state and the mass deviation after every
    step.  Two FP64 runs give the scale of what truncation alone leaves
    undetermined: the same schedule at twice the bond cap (the truncation
    error ||f_chi - f_2chi||), and at the same cap with other Gaussian sketches
    (another, equally valid truncated trajectory)."""
    import paper_2407_09169_amd as q
    import workloads
    w = workloads.get_workload("c2_5d_M128_chi64")
    ctx = q.Context(0)
    runs = {dt: q.setup_workload(ctx, w, dt) for dt in ("f64", "f32", "bf16")}
    w2 = w.replace(chi=2 * w.chi)
    runs["f64_2chi"] = (*q.setup_workload(ctx, w2, "f64"), w2)
    runs["f64_other_sketch"] = (*q.setup_workload(ctx, w, "f64", sketch_seed=w.seed + 100), w)
    n = args.steps
    t0 = time.perf_counter()
    series = _accuracy_series(q, ctx, w, runs, n)
    log(f"drift over {n} steps in {time.perf_counter() - t0:.1f} s")
    out = {"metric": "relative L2 distance to the FP64 run, per step", "workload": w.name,
           "steps": n, "dt": w.dt, "chi": w.chi,
           "final": {k: {"l2_vs_f64": v["l2_vs_f64"][-1] if "l2_vs_f64" in v else None,
                         "max_l2_vs_f64": max(v["l2_vs_f64"]) if "l2_vs_f64" in v else None,
                         "mass_dev": v["mass_dev"][-1]} for k, v in series.items()},
           "series": series}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--dtype", default="f32", choices=["bf16", "f32", "f64"])
    ap.add_argument("--workload", default="c3_5d_M1024_chi128")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-bf16", action="store_true",
                    help="skip the extra BF16-MFMA measurement made next to an FP32 run")
    ap.add_argument("--op-log", default=None,
                    help="also write the per-launch event times of one eager step to this file")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of this many bytes (counter calibration)")
    ap.add_argument("--chi-mean", type=int, default=0,
                    help="bond cap of the mean compositions in the flow protocol (default: the workload's)")
    ap.add_argument("--chi", type=int, default=0,
                    help="bond cap chi of the PDF in the flow protocol (default: the workload's, 64)")
    ap.add_argument("--dt", type=float, default=0.0,
                    help="time step of the flow protocol (default: the workload's, 1e-3)")
    ap.add_argument("--sketch-seed", type=int, default=None,
                    help="seed of the Gaussian sketches in the flow protocol (default: the workload's)")
    ap.add_argument("--chi-mean-study", action="store_true",
                    help="FP64 steps/s and L2 distance to the uncapped mean field for chi_mean in "
                         "{8, 16, 32, chi} on the 128^5 and 1024^5 workloads")
    ap.add_argument("--drift", action="store_true",
                    help="precision drift: FP32 and BF16 against FP64 after every step of the 128^5 "
                         "chi = 64 workload (--steps steps, 200 for the stated target)")
    ap.add_argument("--gradient", action="store_true",
                    help="time steps that also carry the derivatives with respect to Omega and k "
                         "(default workload for this mode: c5_5d_M256_chi64, all its steps)")
    ap.add_argument("--kernel-probe", default=None, metavar="qr:MxN|eig:N",
                    help="only run one FP64 factorisation kernel five times: the Householder QR "
                         "on one seeded M x N matrix, or the Jacobi eigensolver on a batch of "
                         "49 seeded N x N PSD matrices (counter runs)")
    args = ap.parse_args()
    if args.copy_probe:
        _copy_probe(args.copy_probe)
        return
    if args.kernel_probe:
        _kernel_probe(args.kernel_probe)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: there is no multi-GPU path (asked for {args.gpus}); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2407_09169_amd as q
    import workloads

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.workload == "batch64":
        _bench_batched(args, log)
        return
    if args.gradient:
        _bench_gradient(args, log)
        return
    if args.drift:
        _bench_drift(args, log)
        return
    if args.chi_mean_study:
        _bench_chi_mean(args, log)
        return
    if args.workload.startswith("fpmoms_M"):
        _bench_moments(args, log)
        return
    if args.workload == "flow_c2_5d_M128_chi64":
        _bench_flow(args, log)
        return
    if args.workload == "prolong_smag_M1024":
        _bench_prolong(args, log)
        return
    w = workloads.get_workload(args.workload)
    ctx = q.Context(0)
    K, W = args.steps, args.warmup

    prob, f = q.setup_workload(ctx, w, args.dtype)
    log(f"{w.name} {args.dtype}: set up; warmup {W}")
    t_rec = time.perf_counter()
    prob.step(f, W)
    t_rec = time.perf_counter() - t_rec
    ms = _time_steps(torch, prob, f, K)
    value = K / (ms / 1e3)
    log(f"{args.dtype}: {K} steps in {ms:.1f} ms ({value:.2f} steps/s)")

    plain = None
    l2 = None
    if not args.no_plain and args.dtype != "f64":
        prob64, f64 = q.setup_workload(ctx, w, "f64")
        prob64.step(f64, W)
        ms64 = _time_steps(torch, prob64, f64, K)
        plain = K / (ms64 / 1e3)
        l2 = q.l2_diff(ctx, f, f64)
        log(f"f64: {K} steps in {ms64:.1f} ms ({plain:.2f} steps/s); L2 vs f64 {l2:.3e}")
    extra = {}
    if args.dtype == "f32" and not args.no_bf16:
        prob16, f16 = q.setup_workload(ctx, w, "bf16")
        prob16.step(f16, W)
        ms16 = _time_steps(torch, prob16, f16, K)
        extra["bf16_steps_per_s"] = K / (ms16 / 1e3)
        extra["bf16_l2_err_vs_f64"] = q.l2_diff(ctx, f16, f64) if plain else None
        extra["bf16_mass_after"] = prob16.observable(f16, "mass")
        log(f"bf16: {K} steps in {ms16:.1f} ms; L2 vs f64 {extra['bf16_l2_err_vs_f64']}")
    mass = prob.observable(f, "mass")
    disc, norm2 = prob.step_info()
    accuracy = None
    if plain:
        runs = {"f64": (prob64, f64), args.dtype: (prob, f)}
        if "bf16_steps_per_s" in extra:
            runs["bf16"] = (prob16, f16)
        accuracy = _accuracy_series(q, ctx, w, runs, W + K)
        log(f"per-step accuracy: { {k: v.get('l2_vs_f64', [None])[-1] for k, v in accuracy.items()} }")

    oplog = _op_log(prob, f)
    if args.op_log:
        with open(args.op_log, "w") as fh:
            for r in oplog:
                fh.write("\t".join(str(x) for x in r) + "\n")
    roof = _roofline(oplog)
    rows = _classes(oplog)
    log(f"kernel classes: {rows}")
    log(f"dominant kernel: {roof}")
    # four more timed regions of K steps continuing the same trajectory: the
    # median of the five rates is reported beside value (which is the first)
    reps = [value] + [K / (_time_steps(torch, prob, f, K) / 1e3) for _ in range(4)]
    log(f"repeats (steps/s): {[round(r, 2) for r in reps]}")
    cpu = None if args.no_cpu_baseline else _cpu_baseline(w)
    if cpu:
        log(f"cpu baseline: {cpu}")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": w.name, "grid": f"{w.M}^{w.ndims}", "n_cores": w.n_sites,
                   "chi": w.chi, "ell": w.ell, "chi_mean": w.chi_mean, "integrator": w.integrator,
                   "dt": w.dt, "omega": w.omega, "k_react": w.k_react},
        "plain_f64_steps_per_s": plain,
        "speedup_vs_f64": (value / plain) if plain else None,
        "l2_err_vs_f64": l2,
        "mass_after": mass,
        "discarded_weight_last_rounding": float(sum(disc)),
        "repeats_steps_per_s": reps,
        "median_steps_per_s": statistics.median(reps),
        **extra,
        "per_step_accuracy": accuracy,
        "autotune": {"shapes_measured": q.autotune_info()[0], "seconds": q.autotune_info()[1],
                     "enabled": os.environ.get("QTTPDF_AUTOTUNE", "1") != "0",
                     "first_steps_with_recording_s": t_rec},
        "roofline": roof,
        "kernel_classes": rows,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
