"""The C-ABI library loads and exports every entry point include/qttpdf.h declares
(no device calls), and the host-side launch planning is bounds-checked."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qttpdf.h")
LIB = os.path.join(ROOT, "paper_2407_09169_amd", "libqttpdf.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:tt_status|const char\s*\*)\s*([a-z_0-9]+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        subprocess.run([sys.executable, "-m", "paper_2407_09169_amd.build"], cwd=ROOT, check=True)
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("tt_alloc", "mpo_build", "mps_apply_mpo", "mps_round", "tt_step", "tt_observable"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_declared_symbol():
    import paper_2407_09169_amd as q
    assert sorted(q.EXPORTS) == _declared()


def test_dry_run_planning_is_in_bounds():
    """Plans every entry point at the full 5-D M=1024 chi=128 and 256 shapes with host
    memory standing in for device memory: every contraction, QR, eigen and
    copy launch is checked against its buffers; no kernel runs."""
    code = r"""
import os, sys
os.environ["QTTPDF_DRYRUN"] = "1"
sys.path.insert(0, %r)
import paper_2407_09169_amd as q, workloads
ctx = q.Context(0, stream=0)
for name in ["c1_2d_M64", "t_5d_M8_chi16", "c3_5d_M1024_chi128", "c3_5d_M1024_chi256"]:
    w = workloads.get_workload(name)
    for dt in ("f64", "bf16"):
        prob, f = q.setup_workload(ctx, w, dt)
        prob.step(f, 1)
        for o in q.OBS:
            prob.observable(f, o)
    q.l2_diff(ctx, f, f)
    q.round_det(ctx, f, w.chi)
print("ok")
""" % ROOT
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr


def test_dry_run_batch_planning_is_in_bounds():
    """The batched step over uneven problems plans every launch in bounds
    (fused classes included), and a batch that repeats a problem is
    refused."""
    code = r"""
import os, sys
os.environ["QTTPDF_DRYRUN"] = "1"
sys.path.insert(0, %r)
import paper_2407_09169_amd as q, workloads
ctx = q.Context(0, stream=0)
ws = workloads.batch_workloads(count=4, seed=7, bits=(3, 4, 6), chis=(8, 16, 64))
inst = [q.setup_workload(ctx, w, "f32") for w in ws]
b = q.Batch(ctx, [p for p, _ in inst], [f for _, f in inst])
b.step(1)
# two 64^5 chi = 64 instances of equal structure share their launches: every
# fused launch checks that each instance's data stay inside its slab
info = b.info()
assert info["fused_classes"] == 1 and info["fused_instances"] == 2 and info["units"] == 3, info
ws6 = workloads.batch_workloads(count=6, seed=7, bits=(3, 4), chis=(8, 16, 32))
inst6 = [q.setup_workload(ctx, w, "f64") for w in ws6]
b6 = q.Batch(ctx, [p for p, _ in inst6], [f for _, f in inst6])
b6.step(2)
assert b6.info()["fused_classes"] == 2, b6.info()
os.environ["QTTPDF_BATCH_FUSE"] = "0"
assert q.Batch(ctx, [p for p, _ in inst6], [f for _, f in inst6]).info()["fused_classes"] == 0
try:
    q.Batch(ctx, [inst[0][0], inst[0][0]], [inst[0][1], inst[0][1]])
except q.QttError as e:
    assert "repeats" in str(e), e
else:
    raise SystemExit("no error for a repeated problem")
print("ok")
""" % ROOT
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr


def test_dry_run_tangent_planning_is_in_bounds():
    """The step with its two parameter derivatives plans every launch in
    bounds (5-D M = 16 and the M = 256, chi = 64 gradient size)."""
    code = r"""
import os, sys
os.environ["QTTPDF_DRYRUN"] = "1"
sys.path.insert(0, %r)
import paper_2407_09169_amd as q, workloads
ctx = q.Context(0, stream=0)
for w in [workloads.get_workload("t_5d_M16_chi32"),
          workloads.get_workload("c2_5d_M128_chi64").replace(bits=8, k_react=10.0, dt=2e-4)]:
    prob, f = q.setup_workload(ctx, w, "f32")
    tans = {"omega": prob.state(), "k_react": prob.state()}
    prob.step_tangent(f, tans, 1)
    prob.step(f, 1)
try:
    prob.step_tangent(f, {"omega": f}, 1)
except q.QttError as e:
    assert "aliases" in str(e), e
else:
    raise SystemExit("no error for a tangent that aliases the state")
print("ok")
""" % ROOT
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr


def test_errors_are_reported_not_thrown():
    code = r"""
import os, sys
os.environ["QTTPDF_DRYRUN"] = "1"
sys.path.insert(0, %r)
import paper_2407_09169_amd as q
ctx = q.Context(0, stream=0)
try:
    q.TT.alloc(ctx, [2, 4, 1])
except q.QttError as e:
    assert "boundary" in str(e), e
else:
    raise SystemExit("no error for a bad boundary bond")
x = q.TT.alloc(ctx, [1, 2, 1])
try:
    q.round_det(ctx, x, 0)
except q.QttError:
    pass
else:
    raise SystemExit("no error for chi = 0")
print("ok")
""" % ROOT
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr


def test_dry_run_field_problem_planning_is_in_bounds():
    """A problem with the x-fields G(x) and Omega(x) (5-D M = 8, 16 and the
    M = 128 flow grid) plans every launch in bounds, and refuses tangents."""
    code = r"""
import os, sys
os.environ["QTTPDF_DRYRUN"] = "1"
sys.path.insert(0, %r)
import paper_2407_09169_amd as q, workloads
ctx = q.Context(0, stream=0)
for w in [workloads.get_workload("t_5d_M8_chi16"), workloads.get_workload("t_5d_M16_chi32"),
          workloads.get_workload("c2_5d_M128_chi64")]:
    for dt in ("f64", "f32"):
        prob, f = q.setup_workload(ctx, w, dt, fields=True)
        prob.step(f, 1)
        prob.observable(f, "mass")
    try:
        prob.step_tangent(f, {"omega": prob.state()}, 1)
    except q.QttError as e:
        assert "status 5" in str(e), e
    else:
        raise SystemExit("tangent accepted for a field problem")
print("ok")
""" % ROOT
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr


def test_flow_error_measures_host_logic():
    """flow_error_measures is host code of the library: it runs without a GPU
    and gives the oracle's eq. RMSE0 measures."""
    import numpy as np
    from oracle import moments
    import paper_2407_09169_amd as q
    T = 17
    rng = np.random.default_rng(5)
    shape = (3, 3, 3)
    mean_bar = 0.5 + 0.02 * rng.standard_normal((2, T))
    ex = rng.random((2, T) + shape)
    mx = ex + 0.01 * rng.standard_normal((2, T) + shape)
    nx = 1.0 + 1e-3 * rng.standard_normal((T,) + shape)
    want = moments.error_measures(mean_bar, mx, ex, nx)
    got = q.error_measures(mean_bar, np.mean((mx - ex) ** 2, axis=(2, 3, 4)),
                           np.mean((nx - 1.0) ** 2, axis=(1, 2, 3)))
    assert np.allclose(got, want, rtol=1e-13, atol=0)
    with pytest.raises(ValueError):
        q.error_measures(mean_bar[:, :3], None, np.zeros(T))


def test_dry_run_flow_argument_checks():
    """The dense-field entry points validate their arguments on the host
    (grid size, field count, overlapping buffers) before any launch."""
    code = r"""
import os, sys, ctypes as C
os.environ["QTTPDF_DRYRUN"] = "1"
sys.path.insert(0, %r)
import numpy as np
import paper_2407_09169_amd as q
L = q.lib()
ctx = q.Context(0, stream=0)
bits = 3
n = 1 << (3 * bits)
U, G, m, w = (np.zeros(k * n) for k in (3, 1, 2, 2))
p = lambda a, off=0: C.c_void_p(a.ctypes.data + 8 * off)
assert L.fd_moment_steps(ctx.h, bits, 2, p(U), p(G), p(m), p(w), 1e-3, 1) == 0
assert L.fd_moment_steps(ctx.h, 2, 1, p(U), p(G), p(m), p(w), 1e-3, 1) == 1   # bits < 3
assert L.fd_moment_steps(ctx.h, bits, 3, p(U), p(G), p(m), p(w), 1e-3, 1) == 1  # count
assert L.fd_moment_steps(ctx.h, bits, 2, p(U), p(G), p(m), p(m, n), 1e-3, 1) == 1  # work overlaps m
assert L.fd_moment_steps(ctx.h, bits, 1, p(U), p(G), p(m), p(w), 1e-3, -1) == 1
assert L.fd_smagorinsky(ctx.h, bits, p(U), 0.11, 3.0 / 8, 1e-3, p(U, n)) == 1      # G overlaps U
assert L.fd_smagorinsky(ctx.h, bits, p(U), 0.11, 0.0, 1e-3, p(G)) == 1             # delta
assert L.fd_smagorinsky(ctx.h, 11, p(U), 0.11, 3.0 / 8, 1e-3, p(G)) == 1           # bits > 10
h = C.c_void_p(); d = C.c_double()
assert L.tt_from_dense(ctx.h, 1, p(m), 4, C.byref(h), C.byref(d)) == 1
assert L.tt_from_dense(ctx.h, 9, p(m), 0, C.byref(h), C.byref(d)) == 1
assert L.tt_from_dense(ctx.h, 9, p(m), 4, C.byref(h), C.byref(d)) == 0
print("ok")
""" % ROOT
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr


def test_dry_run_inner_noalloc():
    """tt_inner_noalloc plans its launches inside the static scratch buffer
    (host stand-in in a dry run): accepted for chains whose environments fit,
    refused with TT_ERR_INVALID_ARG for larger ones."""
    code = r"""
import os, sys, ctypes as C
os.environ["QTTPDF_DRYRUN"] = "1"
sys.path.insert(0, %r)
import paper_2407_09169_amd as q
from tests.helpers import random_tt
ctx = q.Context(0, stream=0)
out = (C.c_double * 1)()
def run(N, cap):
    caps = [min(2 ** n, 2 ** (N - n), cap) for n in range(N + 1)]
    a = q.TT.from_cores(ctx, random_tt(caps, 1))
    b = q.TT.from_cores(ctx, random_tt(caps, 2))
    return q.lib().tt_inner_noalloc(ctx.h, a.h, b.h, C.cast(out, C.c_void_p))
assert run(24, 160) == 0 and run(12, 24) == 0 and run(20, 512) == 0
assert run(22, 1024) == 1
assert b"static scratch" in q.lib().tt_last_error()
print("ok")
""" % ROOT
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr


def test_dry_run_nonfinite_reported():
    """A NaN put into a state through tt_set_cores is found by the checks that
    every step runs after its roundings (in a dry run on the host buffers that
    stand in for device memory): tt_step_ex returns TT_ERR_NONFINITE and the
    record says so; tt_step_info reports it after a plain tt_step."""
    code = r"""
import os, sys
os.environ["QTTPDF_DRYRUN"] = "1"
sys.path.insert(0, %r)
import numpy as np
import paper_2407_09169_amd as q, workloads
ctx = q.Context(0, stream=0)
w = workloads.get_workload("t_5d_M8_chi16")
p, f = q.setup_workload(ctx, w, "f64")
assert p.step_ex(f, 1)[0]["nonfinite"] == 0
c = f.cores(); c[3][0, 0, 0] = np.inf; f.set_cores(c)
try:
    p.step_ex(f, 1)
    raise SystemExit("no error")
except q.QttError as e:
    assert e.status == 4 and e.records[0]["nonfinite"] == 1, e
p.step(f, 1)
try:
    p.step_info()
    raise SystemExit("no error")
except q.QttError as e:
    assert "NaN or Inf" in str(e)
x, info = q.round_det(ctx, f, 4, 1e-3, with_info=True)
assert len(info["per_bond"]) == w.n_sites + 1
print("ok")
""" % ROOT
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr


def test_dry_run_prolong_planning():
    """tt_prolong at 256^3 -> 512^3 -> 1024^3 plans every launch in bounds
    (dry run) and gives 27 and 30 sites."""
    code = r"""
import os, sys
os.environ["QTTPDF_DRYRUN"] = "1"
sys.path.insert(0, %r)
import paper_2407_09169_amd as q, workloads
ctx = q.Context(0, stream=0)
w = workloads.get_workload("t_5d_M8_chi16", bits=8)
x = q.from_separable(ctx, 3, 8, q.TT_SERIAL, workloads.flow_field_terms(w)["G"], 16)
y, _ = q.prolong(ctx, x, 3, 8, 16)
z, _ = q.prolong(ctx, y, 3, 9, 16)
assert y.info()[1] == 27 and z.info()[1] == 30
print("ok")
""" % ROOT
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr


def test_plan_lane_rules(tmp_path):
    """The launch-plan rules that keep HIP graph capture on the forms that
    work on this runtime (every fork from lane 0, every join onto it; one
    lane on a fixed scratch buffer), exercised by a host program linked
    against the library (dry run), and no batched step captures a graph
    across its units: the batch launches recorded graphs on branch streams
    (the four-branch captured form crashed the host process), each fused
    class's graph captured from one plan as a single step's is."""
    exe = tmp_path / "plan_rules"
    src = os.path.join(ROOT, "tests", "cpp", "test_plan_rules.cpp")
    lib_dir = os.path.dirname(LIB)
    cmd = ["/opt/rocm/bin/hipcc", "-std=c++17", "-O1", "--offload-arch=gfx950", "-x", "hip", src,
           "-I", os.path.join(lib_dir, "csrc"), "-L", lib_dir, "-lqttpdf", "-Wl,-rpath," + lib_dir, "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60,
                       env={**os.environ, "QTTPDF_DRYRUN": "1"})
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr
    src = open(os.path.join(lib_dir, "csrc", "capi.cpp")).read()
    body = src[src.index("tt_status tt_step_batched("):]
    body = body[:body.index("\n}\n")]
    assert "hipStreamBeginCapture" not in body and "hipGraphInstantiate" not in body
    fused = src[src.index("static std::unique_ptr<FusedClass> build_fused_class("):]
    fused = fused[:fused.index("\n}\n")]
    cap = fused[fused.index("hipStreamBeginCapture"):fused.index("hipStreamEndCapture")]
    assert cap.count("->run(") == 1 and "hipStreamWaitEvent" not in cap
