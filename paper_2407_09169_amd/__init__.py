"""Python binding of libqttpdf (MI355X quantics tensor-train Fokker-Planck stepper).

Thin ctypes marshalling over the C ABI declared in include/qttpdf.h; every
step of the method runs in the HIP library.  PyTorch is only used to pass its
current HIP stream (optional).  Importing the package does not load the
library; ``lib()`` does, and raises if libqttpdf.so is missing or no GPU is
present -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqttpdf.so")

TT_MPS, TT_MPO = 0, 1
TT_F64, TT_F32, TT_BF16 = 0, 1, 2
TT_RK4, TT_RK2_HEUN = 0, 1
TT_SERIAL, TT_INTERLEAVED = 0, 1
OBS = {"mass": 0, "mean1": 1, "mean2": 2, "mean12": 3, "R12": 4, "Y12": 5, "product": 6}
OP = {"ID": 0, "D1G": 1, "D2G": 2, "D1P": 3, "D2P": 4, "PHI": 5, "D1G_PHI": 6}
DTYPES = {"f64": TT_F64, "f32": TT_F32, "bf16": TT_BF16}
PARAMS = {"omega": 0, "k_react": 1}
# statistics that are linear in f: their derivative is the statistic of df
LINEAR_OBS = ("mass", "mean1", "mean2", "mean12", "product")

# every entry point of include/qttpdf.h
EXPORTS = [
    "tt_set_allocator", "tt_autotune_info", "tt_ctx_create", "tt_ctx_destroy", "tt_ctx_set_stream", "tt_ctx_synchronize", "tt_last_error",
    "tt_alloc", "tt_free", "tt_info", "tt_set_cores", "tt_get_cores", "tt_from_separable",
    "mpo_build", "mps_apply_mpo", "mps_axpby", "mps_round", "mps_round_sketch",
    "mps_round_sketch_two_sided", "tt_l2_diff",
    "tt_inner", "tt_inner_noalloc", "tt_problem_create", "tt_problem_destroy", "tt_problem_info", "tt_problem_state",
    "tt_step", "tt_step_ex", "tt_profile", "tt_step_info", "tt_observable", "tt_mean_field",
    "tt_linalg_qr", "tt_linalg_eigh", "tt_batch_create", "tt_batch_info", "tt_step_batched", "tt_batch_destroy",
    "tt_step_tangent", "tt_moment_field", "tt_to_dense", "fd_smagorinsky", "fd_moment_steps",
    "fd_sq_diff_sum", "flow_error_measures", "tt_problem_create_flow", "tt_from_dense", "tt_prolong",
]
KERNELS = {"contract": 0, "qr": 1, "eig": 2, "stream": 3, "all": 4}


class TTParams(C.Structure):
    _fields_ = [
        ("ndims", C.c_int32), ("bits", C.c_int32), ("ordering", C.c_int32),
        ("chi", C.c_int32), ("ell", C.c_int32), ("chi_mean", C.c_int32), ("ell_mean", C.c_int32),
        ("integrator", C.c_int32), ("dtype", C.c_int32),
        ("omega", C.c_double), ("k_react", C.c_double), ("nu_phi", C.c_double),
        ("gamma", C.c_double), ("dt", C.c_double),
    ]


class TTTerm(C.Structure):
    _fields_ = [("coeff", C.c_double), ("op", C.c_int32 * 8), ("field", C.c_int32)]


class TTRoundInfo(C.Structure):
    _fields_ = [("max_bond", C.c_int32), ("discarded_weight", C.c_double), ("norm2", C.c_double),
                ("per_bond", C.POINTER(C.c_double))]


class TTStepRecord(C.Structure):
    _fields_ = [("mass_dev", C.c_double), ("discarded_weight", C.c_double), ("max_bond", C.c_int32),
                ("nonfinite", C.c_int32)]


class QttError(RuntimeError):
    pass


_LIB = None


def lib_path() -> str:
    return LIB_PATH


def lib():
    """Loads libqttpdf.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise QttError(f"{LIB_PATH} not built: run `python -m paper_2407_09169_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, dbl = C.c_void_p, C.c_int, C.c_double
    P = C.POINTER
    sig = {
        "tt_set_allocator": [vp, vp, vp],
        "tt_autotune_info": [P(i32), P(dbl)],
        "tt_ctx_create": [i32, vp, P(vp)],
        "tt_ctx_destroy": [vp],
        "tt_ctx_set_stream": [vp, vp],
        "tt_ctx_synchronize": [vp],
        "tt_alloc": [vp, i32, i32, P(C.c_int32), P(vp)],
        "tt_free": [vp],
        "tt_info": [vp, P(i32), P(i32), P(C.c_int32), P(C.c_int64)],
        "tt_set_cores": [vp, P(dbl)],
        "tt_get_cores": [vp, P(dbl)],
        "tt_from_separable": [vp, i32, i32, i32, i32, P(dbl), P(P(dbl)), i32, P(vp)],
        "mpo_build": [vp, i32, i32, i32, P(TTTerm), i32, P(vp), i32, i32, dbl, P(vp), P(i32)],
        "mps_apply_mpo": [vp, vp, vp, i32, P(vp)],
        "mps_axpby": [vp, i32, P(dbl), P(vp), P(vp)],
        "mps_round": [vp, vp, i32, dbl, P(TTRoundInfo), P(vp)],
        "mps_round_sketch": [vp, i32, P(dbl), P(vp), P(vp), vp, i32, i32, P(vp)],
        "mps_round_sketch_two_sided": [vp, i32, P(dbl), P(vp), P(vp), vp, vp, i32, i32, P(vp)],
        "tt_l2_diff": [vp, vp, vp, P(dbl)],
        "tt_inner": [vp, vp, vp, P(dbl)],
        "tt_inner_noalloc": [vp, vp, vp, vp],
        "tt_problem_create": [vp, P(TTParams), P(vp), vp, vp, vp, vp, P(vp)],
        "tt_problem_destroy": [vp],
        "tt_problem_info": [vp, P(i32), P(C.c_int32), P(i32)],
        "tt_problem_state": [vp, P(vp)],
        "tt_step": [vp, vp, vp, i32],
        "tt_step_ex": [vp, vp, vp, i32, P(TTStepRecord)],
        "tt_step_info": [vp, P(dbl), P(dbl)],
        "tt_profile": [vp, vp, vp, i32, i32, P(dbl), P(C.c_int64), P(dbl), P(dbl)],
        "tt_observable": [vp, vp, vp, i32, P(dbl)],
        "tt_mean_field": [vp, vp, vp, i32, P(vp), P(dbl)],
        "tt_linalg_qr": [vp, i32, i32, i32, P(dbl), P(dbl), P(dbl)],
        "tt_linalg_eigh": [vp, i32, i32, i32, P(dbl), P(dbl), P(dbl)],
        "tt_batch_create": [vp, i32, P(vp), P(vp), P(vp)],
        "tt_batch_info": [vp, P(i32), P(i32), P(i32), P(C.c_int64)],
        "tt_step_batched": [vp, i32],
        "tt_batch_destroy": [vp],
        "tt_step_tangent": [vp, vp, vp, i32, P(i32), P(vp), i32],
        "tt_moment_field": [vp, vp, vp, P(dbl), P(dbl), P(vp)],
        "tt_to_dense": [vp, vp, vp],
        "fd_smagorinsky": [vp, i32, vp, dbl, dbl, dbl, vp],
        "fd_moment_steps": [vp, i32, i32, vp, vp, vp, vp, dbl, i32],
        "fd_sq_diff_sum": [vp, C.c_int64, vp, vp, dbl, P(dbl)],
        "flow_error_measures": [i32, P(dbl), P(dbl), P(dbl), P(dbl)],
        "tt_problem_create_flow": [vp, P(TTParams), P(vp), vp, vp, vp, vp, vp, vp, P(vp)],
        "tt_from_dense": [vp, i32, vp, i32, P(vp), P(dbl)],
        "tt_prolong": [vp, vp, i32, i32, i32, P(vp), P(dbl)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.tt_last_error.argtypes = []
    L.tt_last_error.restype = C.c_char_p
    _LIB = L
    return L


def _check(status: int):
    if status != 0:
        msg = lib().tt_last_error().decode(errors="replace")
        raise QttError(f"qttpdf status {status}: {msg}")


def _torch_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:  # noqa: BLE001 - torch is optional plumbing
        pass
    return C.c_void_p(None)


def autotune_info():
    """(launch shapes measured by the contraction autotuner, seconds spent)."""
    n, t = C.c_int(), C.c_double()
    _check(lib().tt_autotune_info(C.byref(n), C.byref(t)))
    return n.value, t.value


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_int, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p, C.c_void_p)
_ALLOCATOR = None  # the registered callbacks (kept alive while registered)


def use_torch_allocator(enable: bool = True):
    """Routes the library's device allocations through PyTorch's caching
    allocator (tt_set_allocator), so that torch owns and accounts for the
    memory; enable=False restores hipMalloc.  Memory already allocated keeps
    its allocator."""
    global _ALLOCATOR
    if not enable:
        _check(lib().tt_set_allocator(None, None, None))
        _ALLOCATOR = None
        return
    import torch

    def _alloc(nbytes, device, stream, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device=int(device))
        except Exception:  # noqa: BLE001 - reported by the library as TT_ERR_OOM
            return None

    def _free(ptr, nbytes, device, stream, user):
        torch.cuda.caching_allocator_delete(int(ptr))

    cbs = (_ALLOC_FN(_alloc), _FREE_FN(_free))
    _check(lib().tt_set_allocator(C.cast(cbs[0], C.c_void_p), C.cast(cbs[1], C.c_void_p), None))
    _ALLOCATOR = cbs


class Context:
    def __init__(self, device: int = 0, stream=None):
        self.device = device
        self.h = C.c_void_p()
        s = _torch_stream() if stream is None else C.c_void_p(stream)
        _check(lib().tt_ctx_create(device, s, C.byref(self.h)))

    def synchronize(self):
        _check(lib().tt_ctx_synchronize(self.h))

    def close(self):
        if self.h:
            lib().tt_ctx_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


class TT:
    """An MPS or MPO in device memory (owned)."""

    def __init__(self, ctx: Context, handle: C.c_void_p):
        self.ctx = ctx
        self.h = handle

    @classmethod
    def alloc(cls, ctx, caps, kind=TT_MPS):
        caps = np.ascontiguousarray(caps, dtype=np.int32)
        h = C.c_void_p()
        _check(lib().tt_alloc(ctx.h, kind, len(caps) - 1, caps.ctypes.data_as(C.POINTER(C.c_int32)),
                              C.byref(h)))
        return cls(ctx, h)

    @classmethod
    def from_cores(cls, ctx, cores, kind=TT_MPS):
        """Uploads cores (list of arrays (rl, 2, rr) or (rl, 2, 2, rr))."""
        caps = [1] + [int(G.shape[-1]) for G in cores]
        t = cls.alloc(ctx, caps, kind)
        t.set_cores(cores)
        return t

    def info(self):
        kind, n = C.c_int(), C.c_int()
        _check(lib().tt_info(self.h, C.byref(kind), C.byref(n), None, None))
        caps = np.zeros(n.value + 1, dtype=np.int32)
        ne = C.c_int64()
        _check(lib().tt_info(self.h, None, None, caps.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(ne)))
        return kind.value, n.value, caps, ne.value

    @property
    def caps(self):
        return self.info()[2]

    def set_cores(self, cores):
        kind, n, caps, ne = self.info()
        p = 4 if kind == TT_MPO else 2
        buf = np.zeros(ne, dtype=np.float64)
        off = 0
        for k in range(n):
            G = np.asarray(cores[k], dtype=np.float64)
            shape = (caps[k], 2, caps[k + 1]) if p == 2 else (caps[k], 2, 2, caps[k + 1])
            full = np.zeros(shape)
            sl = tuple(slice(0, s) for s in G.shape)
            full[sl] = G
            sz = full.size
            buf[off:off + sz] = full.ravel()
            off += sz
        _check(lib().tt_set_cores(self.h, buf.ctypes.data_as(C.POINTER(C.c_double))))

    def cores(self):
        kind, n, caps, ne = self.info()
        buf = np.zeros(ne, dtype=np.float64)
        _check(lib().tt_get_cores(self.h, buf.ctypes.data_as(C.POINTER(C.c_double))))
        out, off = [], 0
        for k in range(n):
            shape = (caps[k], 2, caps[k + 1]) if kind == TT_MPS else (caps[k], 2, 2, caps[k + 1])
            sz = int(np.prod(shape))
            out.append(buf[off:off + sz].reshape(shape))
            off += sz
        return out

    def free(self):
        if self.h:
            lib().tt_free(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:  # noqa: BLE001
            pass


def _handles(ts):
    arr = (C.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = t.h if t is not None else None
    return arr


def from_separable(ctx, ndims, bits, ordering, terms, chi):
    """MPS of sum_t c_t prod_d v_t[d] rounded to chi (terms: [(c, [vec or None]*ndims)])."""
    n = len(terms)
    coeffs = (C.c_double * n)(*[float(c) for c, _ in terms])
    keep = []
    ptrs = (C.POINTER(C.c_double) * (n * ndims))()
    for t, (_, vecs) in enumerate(terms):
        for d in range(ndims):
            v = vecs[d]
            if v is None:
                ptrs[t * ndims + d] = C.POINTER(C.c_double)()
            else:
                a = np.ascontiguousarray(v, dtype=np.float64)
                keep.append(a)
                ptrs[t * ndims + d] = a.ctypes.data_as(C.POINTER(C.c_double))
    h = C.c_void_p()
    _check(lib().tt_from_separable(ctx.h, ndims, bits, ordering, n, coeffs, ptrs, chi, C.byref(h)))
    return TT(ctx, h)


def mpo_build(ctx, ndims, bits, ordering, terms, fields=(), field_ndims=0, rel_tol=0.0):
    """terms: [(coeff, {dim: op_name}, field_index or -1)]."""
    arr = (TTTerm * len(terms))()
    for i, (c, ops, fld) in enumerate(terms):
        arr[i].coeff = c
        for d in range(8):
            arr[i].op[d] = OP[ops.get(d, "ID")] if isinstance(ops, dict) else OP["ID"]
        arr[i].field = fld
    h = C.c_void_p()
    mb = C.c_int()
    _check(lib().mpo_build(ctx.h, ndims, bits, ordering, arr, len(terms), _handles(list(fields)),
                           len(fields), field_ndims, rel_tol, C.byref(h), C.byref(mb)))
    return TT(ctx, h), mb.value


def apply_mpo(ctx, W, x, dtype="f64"):
    h = C.c_void_p()
    _check(lib().mps_apply_mpo(ctx.h, W.h, x.h, DTYPES[dtype], C.byref(h)))
    return TT(ctx, h)


def axpby(ctx, coeffs, xs):
    c = (C.c_double * len(xs))(*coeffs)
    h = C.c_void_p()
    _check(lib().mps_axpby(ctx.h, len(xs), c, _handles(xs), C.byref(h)))
    return TT(ctx, h)


def round_det(ctx, x, chi, rel_tol=0.0, with_info=False):
    """mps_round; with_info also returns {"max_bond", "discarded_weight",
    "norm2", "per_bond"}."""
    h = C.c_void_p()
    if not with_info:
        _check(lib().mps_round(ctx.h, x.h, chi, rel_tol, None, C.byref(h)))
        return TT(ctx, h)
    n = x.info()[1]
    per = (C.c_double * (n + 1))()
    info = TTRoundInfo(0, 0.0, 0.0, per)
    _check(lib().mps_round(ctx.h, x.h, chi, rel_tol, C.byref(info), C.byref(h)))
    return TT(ctx, h), {"max_bond": info.max_bond, "discarded_weight": info.discarded_weight,
                        "norm2": info.norm2, "per_bond": list(per)}


def round_sketch(ctx, coeffs, mpos, xs, sketch, chi, dtype="f64", sketch_left=None):
    """mps_round_sketch, or with a left sketch mps_round_sketch_two_sided."""
    c = (C.c_double * len(xs))(*coeffs)
    h = C.c_void_p()
    if sketch_left is None:
        _check(lib().mps_round_sketch(ctx.h, len(xs), c, _handles(mpos), _handles(xs), sketch.h, chi,
                                      DTYPES[dtype], C.byref(h)))
    else:
        _check(lib().mps_round_sketch_two_sided(ctx.h, len(xs), c, _handles(mpos), _handles(xs),
                                                sketch.h, sketch_left.h, chi, DTYPES[dtype],
                                                C.byref(h)))
    return TT(ctx, h)


def l2_diff(ctx, a, b):
    r = C.c_double()
    _check(lib().tt_l2_diff(ctx.h, a.h, b.h, C.byref(r)))
    return r.value


def inner(ctx, a, b):
    r = C.c_double()
    _check(lib().tt_inner(ctx.h, a.h, b.h, C.byref(r)))
    return r.value


def inner_noalloc(ctx, a, b, out):
    """tt_inner_noalloc: <a, b> written to out (a float64 CUDA tensor owned by
    the caller; its first element), asynchronously on the context's stream."""
    if out.dtype.itemsize != 8 or out.numel() < 1 or not out.is_cuda:
        raise ValueError("out must be a float64 CUDA tensor with at least one element")
    _check(lib().tt_inner_noalloc(ctx.h, a.h, b.h, C.c_void_p(out.data_ptr())))


def linalg_qr(ctx, A, with_r=True):
    """Householder QR of a stack of matrices A (count, m, n) on the device."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    cnt, m, n = A.shape
    Q = np.zeros((cnt, m, n))
    R = np.zeros((cnt, n, n)) if with_r else None
    dp = C.POINTER(C.c_double)
    _check(lib().tt_linalg_qr(ctx.h, cnt, m, n, A.ctypes.data_as(dp), Q.ctypes.data_as(dp),
                              R.ctypes.data_as(dp) if with_r else None))
    return Q, R


def linalg_eigh(ctx, G, keep):
    """Leading eigenpairs of a stack of PSD matrices G (count, n, n) on the device."""
    G = np.ascontiguousarray(G, dtype=np.float64)
    cnt, n, _ = G.shape
    P = np.zeros((cnt, n, keep))
    lam = np.zeros((cnt, n))
    dp = C.POINTER(C.c_double)
    _check(lib().tt_linalg_eigh(ctx.h, cnt, n, keep, G.ctypes.data_as(dp), P.ctypes.data_as(dp),
                                lam.ctypes.data_as(dp)))
    return P, lam


class Problem:
    """One eq. FP2 problem: fixed operator, sketches and the recorded step."""

    def __init__(self, ctx, params: TTParams, velocity=None, sketch=None, sketch_left=None,
                 sketch_mean=None, sketch_mean_left=None, diffusivity=None, mixing=None):
        """diffusivity / mixing: optional x-MPS fields G(x) and Omega_mix(x)
        (tt_problem_create_flow)."""
        self.ctx = ctx
        self.params = params
        self._keep = (velocity, sketch, sketch_left, sketch_mean, sketch_mean_left)
        h = C.c_void_p()
        vel = _handles(velocity) if velocity else None
        opt = lambda t: t.h if t is not None else None  # noqa: E731
        if diffusivity is None and mixing is None:
            _check(lib().tt_problem_create(ctx.h, C.byref(params), vel, sketch.h, sketch_left.h,
                                           opt(sketch_mean), opt(sketch_mean_left), C.byref(h)))
        else:
            _check(lib().tt_problem_create_flow(ctx.h, C.byref(params), vel, opt(diffusivity),
                                                opt(mixing), sketch.h, sketch_left.h,
                                                opt(sketch_mean), opt(sketch_mean_left), C.byref(h)))
        self.h = h

    def info(self):
        n = C.c_int()
        _check(lib().tt_problem_info(self.h, C.byref(n), None, None))
        bonds = np.zeros(n.value + 1, dtype=np.int32)
        mb = C.c_int()
        _check(lib().tt_problem_info(self.h, None, bonds.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(mb)))
        return bonds, mb.value

    def state(self):
        h = C.c_void_p()
        _check(lib().tt_problem_state(self.h, C.byref(h)))
        return TT(self.ctx, h)

    def step(self, f, n_steps=1):
        _check(lib().tt_step(self.ctx.h, self.h, f.h, n_steps))

    def step_ex(self, f, n_steps=1):
        """tt_step_ex: steps with one record per step, [{"mass_dev",
        "discarded_weight", "max_bond", "nonfinite"}]; raises QttError on a
        NaN or Inf (the records up to that step in its .records)."""
        recs = (TTStepRecord * max(1, n_steps))()
        st = lib().tt_step_ex(self.ctx.h, self.h, f.h, n_steps, recs)
        out = [{"mass_dev": r.mass_dev, "discarded_weight": r.discarded_weight, "max_bond": r.max_bond,
                "nonfinite": r.nonfinite} for r in recs[:n_steps]]
        if st != 0:
            err = QttError(f"qttpdf status {st}: {lib().tt_last_error().decode(errors='replace')}")
            err.status = st
            err.records = out
            raise err
        return out

    def profile(self, f, n_steps, kernel):
        """(ms, launches, flops, bytes) of one kernel class over n_steps eager steps."""
        ms, n, fl, by = C.c_double(), C.c_int64(), C.c_double(), C.c_double()
        _check(lib().tt_profile(self.ctx.h, self.h, f.h, n_steps, KERNELS[kernel], C.byref(ms),
                                C.byref(n), C.byref(fl), C.byref(by)))
        return ms.value, n.value, fl.value, by.value

    def step_info(self):
        n = int(self.info()[0].size)
        disc = np.zeros(n, dtype=np.float64)
        nrm = C.c_double()
        _check(lib().tt_step_info(self.h, disc.ctypes.data_as(C.POINTER(C.c_double)), C.byref(nrm)))
        return disc, nrm.value

    def step_tangent(self, f, tangents, n_steps=1):
        """Advances f and the parameter derivatives tangents = {"omega": df,
        "k_react": dk} (states of this problem) by n_steps steps."""
        names = list(tangents)
        n = len(names)
        params = (C.c_int * n)(*[PARAMS[k] for k in names])
        dfs = (C.c_void_p * n)(*[tangents[k].h for k in names])
        _check(lib().tt_step_tangent(self.ctx.h, self.h, f.h, n, params, dfs, n_steps))

    def observable(self, f, which):
        r = C.c_double()
        _check(lib().tt_observable(self.ctx.h, self.h, f.h, OBS[which], C.byref(r)))
        return r.value

    def mean_field(self, f, a):
        h = C.c_void_p()
        sc = C.c_double()
        _check(lib().tt_mean_field(self.ctx.h, self.h, f.h, a, C.byref(h), C.byref(sc)))
        if h.value is None:
            return sc.value
        return TT(self.ctx, h)

    def moment_field(self, f, w1=None, w2=None):
        """h^2 sum w1(phi1) w2(phi2) f as an x-MPS (tt_moment_field); w1, w2 are
        arrays of M weights or None (all ones)."""
        M = 1 << self.params.bits
        ws = []
        for w in (w1, w2):
            if w is None:
                ws.append(None)
                continue
            a = np.ascontiguousarray(w, dtype=np.float64)
            if a.shape != (M,):
                raise ValueError(f"weights must have shape ({M},)")
            ws.append(a)
        h = C.c_void_p()
        ptr = [None if a is None else a.ctypes.data_as(C.POINTER(C.c_double)) for a in ws]
        _check(lib().tt_moment_field(self.ctx.h, self.h, f.h, ptr[0], ptr[1], C.byref(h)))
        return TT(self.ctx, h)

    def close(self):
        if self.h:
            lib().tt_problem_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


class Batch:
    """Many (problem, state) instances advanced together (tt_batch_create /
    tt_step_batched): instances of equal structure share every launch of
    their step (fused classes), the others step with their own graphs."""

    def __init__(self, ctx, problems, states):
        self.ctx = ctx
        self._keep = (list(problems), list(states))
        n = len(problems)
        P = (C.c_void_p * n)(*[p.h for p in problems])
        S = (C.c_void_p * n)(*[f.h for f in states])
        h = C.c_void_p()
        _check(lib().tt_batch_create(ctx.h, n, P, S, C.byref(h)))
        self.h = h

    def step(self, n_steps=1):
        _check(lib().tt_step_batched(self.h, n_steps))

    def info(self):
        """{"units", "fused_classes", "fused_instances", "slab_bytes"} (tt_batch_info)."""
        u, c, fi = C.c_int32(), C.c_int32(), C.c_int32()
        sb = C.c_int64()
        _check(lib().tt_batch_info(self.h, C.byref(u), C.byref(c), C.byref(fi), C.byref(sb)))
        return {"units": u.value, "fused_classes": c.value, "fused_instances": fi.value,
                "slab_bytes": sb.value}

    def close(self):
        if getattr(self, "h", None):
            lib().tt_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


def statistic_and_gradient(ctx, w, n_steps, statistic="product", dtype="f64",
                           params=("omega", "k_react")):
    """J = statistic(f(T)) after n_steps steps of workload w from its initial
    PDF, and dJ/dtheta for theta in params (forward-mode tangents carried
    along the step).  statistic must be linear in f."""
    if statistic not in LINEAR_OBS:
        raise ValueError(f"derivatives are provided for the linear statistics {LINEAR_OBS}")
    prob, f = setup_workload(ctx, w, dtype)
    tans = {p: prob.state() for p in params}
    prob.step_tangent(f, tans, n_steps)
    J = prob.observable(f, statistic)
    grads = {p: prob.observable(tans[p], statistic) for p in params}
    for t in tans.values():
        t.free()
    f.free()
    prob.close()
    return J, grads


def setup_workload(ctx, w, dtype="f64", fields=False, sketch_seed=None):
    """Builds (problem, f0) for a workloads.Workload with the seeded inputs;
    fields=True adds the seeded x-fields G(x) and Omega(x)
    (workloads.flow_field_terms, built exactly from their separable terms); a
    dict {"G": TT, "Omega": TT} passes given x-MPSs.  sketch_seed draws the
    Gaussian sketches from another seed (same initial state and velocity)."""
    import workloads
    ws = w if sketch_seed is None else w.replace(seed=sketch_seed)

    ordering = TT_SERIAL if w.ordering == "serial" else TT_INTERLEAVED
    velocity = None
    if w.ndims == 5:
        velocity = [from_separable(ctx, 3, w.bits, TT_SERIAL, comp, w.vel_rank)
                    for comp in workloads.velocity_terms(w)]
    sketch = TT.from_cores(ctx, workloads.sketch_cores(ws))
    sketch_left = TT.from_cores(ctx, workloads.left_sketch_cores(ws))
    sketch_mean = TT.from_cores(ctx, workloads.mean_sketch_cores(ws)) if w.ndims == 5 else None
    sketch_mean_left = TT.from_cores(ctx, workloads.left_mean_sketch_cores(ws)) if w.ndims == 5 else None
    p = TTParams(ndims=w.ndims, bits=w.bits, ordering=ordering, chi=w.chi, ell=w.ell,
                 chi_mean=w.chi_mean, ell_mean=w.ell_mean,
                 integrator=TT_RK4 if w.integrator == "rk4" else TT_RK2_HEUN,
                 dtype=DTYPES[dtype], omega=w.omega, k_react=w.k_react, nu_phi=w.nu_phi,
                 gamma=w.gamma, dt=w.dt)
    fx = dict(fields) if isinstance(fields, dict) else {}
    if fields is True:
        for k, terms in workloads.flow_field_terms(w).items():
            fx[k] = from_separable(ctx, 3, w.bits, TT_SERIAL, terms, 16)
    prob = Problem(ctx, p, velocity, sketch, sketch_left, sketch_mean, sketch_mean_left,
                   diffusivity=fx.get("G"), mixing=fx.get("Omega"))
    f0 = from_separable(ctx, w.ndims, w.bits, ordering, workloads.ic_terms(w), w.chi)
    return prob, f0


# ---------------------------------------------------------------------------
# flow case: dense x fields (float64 torch tensors on the GPU, row-major
# [x1][x2][x3]); the arithmetic runs in the library
# ---------------------------------------------------------------------------
def _dense_arg(t, n, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be contiguous with {n} elements (has {t.numel()})")
    return C.c_void_p(t.data_ptr())


def to_dense(ctx, x, out):
    """Writes every entry of the MPS x (N <= 30 sites) into the tensor out (2^N values)."""
    _, n_sites, _, _ = x.info()
    _check(lib().tt_to_dense(ctx.h, x.h, _dense_arg(out, 1 << n_sites, "out")))
    return out


def from_dense(ctx, values, chi):
    """(MPS, discarded weight) of a dense float64 CUDA tensor of 2^N values
    (tt_from_dense: truncated TT-SVD, bonds capped at chi)."""
    n = values.numel()
    N = n.bit_length() - 1
    if n != 1 << N:
        raise ValueError("the number of values must be a power of two")
    h = C.c_void_p()
    disc = C.c_double()
    _check(lib().tt_from_dense(ctx.h, N, _dense_arg(values, n, "values"), chi, C.byref(h),
                               C.byref(disc)))
    return TT(ctx, h), disc.value


def prolong(ctx, x, ndims, bits, chi):
    """tt_prolong: (the field on the grid of twice the resolution, rounded to
    chi; the discarded weight of the roundings)."""
    h = C.c_void_p()
    d = C.c_double()
    _check(lib().tt_prolong(ctx.h, x.h, ndims, bits, chi, C.byref(h), C.byref(d)))
    return TT(ctx, h), d.value


def smagorinsky(ctx, bits, U, G, c_s, delta, gamma):
    """G = gamma + c_s delta^2 / 2 |S(U)| (fd_smagorinsky); U has 3 M^3 values."""
    n = 1 << (3 * bits)
    _check(lib().fd_smagorinsky(ctx.h, bits, _dense_arg(U, 3 * n, "U"), c_s, delta, gamma,
                                _dense_arg(G, n, "G")))
    return G


def moment_steps(ctx, bits, U, G, m, work, dt, n_steps=1):
    """n_steps RK2 steps of the moment equation on m (1 or 2 fields) in place."""
    n = 1 << (3 * bits)
    count = m.numel() // n
    if count not in (1, 2):
        raise ValueError("m must hold one or two fields of M^3 values")
    _check(lib().fd_moment_steps(ctx.h, bits, count, _dense_arg(U, 3 * n, "U"),
                                 _dense_arg(G, n, "G"), _dense_arg(m, count * n, "m"),
                                 _dense_arg(work, count * n, "work"), dt, n_steps))
    return m


def sq_diff_sum(ctx, a, b=None, c=0.0):
    """sum (a - b - c)^2 over the entries of a (b optional, same size)."""
    n = a.numel()
    out = C.c_double()
    bp = None if b is None else _dense_arg(b, n, "b")
    _check(lib().fd_sq_diff_sum(ctx.h, n, _dense_arg(a, n, "a"), bp, c, C.byref(out)))
    return out.value


def error_measures(mean_bar, sq_mean_x, sq_norm_x):
    """(Error_2b up, Error_2b down, Error_2c up, Error_2c down) of eq. RMSE0."""
    mb = np.ascontiguousarray(mean_bar, dtype=np.float64)
    T = mb.shape[1]
    if mb.shape != (2, T):
        raise ValueError("mean_bar must have shape (2, T)")
    sn = np.ascontiguousarray(sq_norm_x, dtype=np.float64)
    if sn.shape != (T,):
        raise ValueError("sq_norm_x must have shape (T,)")
    dp = C.POINTER(C.c_double)
    sm = None
    if sq_mean_x is not None:
        sm = np.ascontiguousarray(sq_mean_x, dtype=np.float64)
        if sm.shape != (2, T):
            raise ValueError("sq_mean_x must have shape (2, T)")
    out = np.zeros(4)
    _check(lib().flow_error_measures(T, mb.ctypes.data_as(dp),
                                     None if sm is None else sm.ctypes.data_as(dp),
                                     sn.ctypes.data_as(dp), out.ctypes.data_as(dp)))
    return tuple(float(v) for v in out)
