"""Python binding of libellsp2.so (include/ellsp2.h): argument marshalling only.

Every function here has the name of the C entry point it calls.  No step of
the computation runs in Python: if the HIP library is missing, loading fails
with an error instead of falling back to anything else.

torch is imported before the library so that the process has a single HIP
runtime (torch ships its own libamdhip64 with the same soname); torch is used
for streams and, optionally, for device memory handed over via ellpack_wrap.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libellsp2.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "ellsp2.h")

ELL_OK, ELL_EINVAL, ELL_ENOMEM, ELL_EOVERFLOW, ELL_ENOCONV = 0, -1, -2, -3, -4
ELL_EDEVICE, ELL_ENODEV, ELL_ENONFINITE, ELL_EDEGENERATE = -5, -6, -7, -8
ELL_F64, ELL_F32 = 0, 1
SP2_F64, SP2_MIXED = 0, 1
DENSE_F64, DENSE_BF16X3 = 0, 1

i32p = C.POINTER(C.c_int32)
i8p = C.POINTER(C.c_int8)
i64p = C.POINTER(C.c_int64)
f64p = C.POINTER(C.c_double)
vp = C.c_void_p


class SP2Params(C.Structure):
    _fields_ = [("n_occ", C.c_double), ("tau", C.c_double), ("idem_target", C.c_double),
                ("max_iter", C.c_int32), ("precision", C.c_int32), ("fp64_tail_steps", C.c_int32),
                ("poll_every", C.c_int32), ("tau_fp32", C.c_double), ("switch_eta", C.c_double),
                ("stall_stop", C.c_int32), ("profile", C.c_int32), ("prune_once", C.c_int32)]


class SP2Report(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("fp32_iterations", C.c_int32),
                ("final_M", C.c_int32), ("eta", C.c_double), ("trace_x", C.c_double),
                ("emin", C.c_double), ("emax", C.c_double), ("seconds", C.c_double),
                ("hist_trx", f64p), ("hist_trx2", f64p), ("hist_eta2", f64p), ("hist_up", i8p),
                ("hist_maxw", i32p), ("hist_prec", i8p), ("x2_seconds", C.c_double),
                ("x2_bytes", C.c_int64), ("x2_launches", C.c_int32), ("hist_x2_seconds", f64p),
                ("hist_x2_bytes", i64p), ("batch_k", C.c_int32), ("batch_kernel", C.c_int32)]


_lib = None


def load():
    """Load libellsp2.so (built by paper_2102_08505_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  -- one HIP runtime per process, see module docstring
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_2102_08505_amd/build.py")
    L = C.CDLL(LIB_PATH)
    L.ellpack_check_host.argtypes = [C.c_int32, C.c_int32, i32p, i32p, f64p]
    L.ellpack_alloc.argtypes = [C.POINTER(vp), C.c_int32, C.c_int32, C.c_int, vp]
    L.ellpack_wrap.argtypes = [C.POINTER(vp), C.c_int32, C.c_int32, C.c_int, vp, vp, vp, vp]
    L.ellpack_free.argtypes = [vp]
    L.ellpack_info.argtypes = [vp, i32p, i32p, i32p]
    L.ellpack_upload.argtypes = [vp, i32p, i32p, f64p]
    L.ellpack_download.argtypes = [vp, i32p, i32p, f64p]
    L.ellpack_x2_threshold.argtypes = [vp, vp, C.c_double, f64p, i32p]
    L.ellpack_x2_step.argtypes = [vp, vp, vp, C.c_double, f64p, i32p]
    L.ellpack_x2_step_noalloc.argtypes = [vp, vp, vp, C.c_double, f64p, i32p]
    L.ellpack_trace.argtypes = [vp, f64p]
    L.ellpack_trace_product.argtypes = [vp, vp, f64p]
    L.sp2_solve.argtypes = [vp, vp, C.POINTER(SP2Params), C.POINTER(SP2Report)]
    L.sp2_solve_batched.argtypes = [C.c_int32, C.POINTER(vp), C.POINTER(vp), C.POINTER(SP2Params),
                                    C.POINTER(SP2Report)]
    L.dense_sp2_solve.argtypes = [vp, C.c_int32, vp, C.c_int32, C.POINTER(SP2Params),
                                  C.POINTER(SP2Report), vp]
    L.dense_x2.argtypes = [vp, vp, C.c_int32, C.c_int32, vp]
    L.ellpack_strerror.restype = C.c_char_p
    L.ellpack_strerror.argtypes = [C.c_int]
    L.ellpack_last_device_error.restype = C.c_char_p
    L.ellpack_last_device_error.argtypes = []
    _lib = L
    return L


def header_functions():
    """Names of the functions include/ellsp2.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t):
    return a.ctypes.data_as(t)


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream  # a torch.cuda.Stream


class Error(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = load().ellpack_strerror(status).decode()
        dev = load().ellpack_last_device_error().decode()
        super().__init__(f"{where}: {msg} ({status}); last device error: {dev}")


def _check(rc, where):
    if rc != ELL_OK:
        raise Error(rc, where)
    return rc


# ---- handles --------------------------------------------------------------------------
def ellpack_check_host(N, M, nnz, index, value=None):
    nnz, index = _i32(nnz), _i32(index)
    v = _f64(value) if value is not None else None
    return load().ellpack_check_host(int(N), int(M), _ptr(nnz, i32p), _ptr(index, i32p),
                                     _ptr(v, f64p) if v is not None else None)


def ellpack_alloc(N, M, prec=ELL_F64, stream=None):
    """Returns (status, handle)."""
    h = vp()
    rc = load().ellpack_alloc(C.byref(h), int(N), int(M), int(prec), _stream(stream))
    return rc, h


def ellpack_wrap(N, M, prec, d_nnz, d_index, d_value, stream=None):
    """Wrap device pointers (ints, e.g. torch tensor data_ptr()).  Returns (status, handle)."""
    h = vp()
    rc = load().ellpack_wrap(C.byref(h), int(N), int(M), int(prec), vp(d_nnz), vp(d_index), vp(d_value),
                             _stream(stream))
    return rc, h


def ellpack_free(h):
    return load().ellpack_free(h)


def ellpack_info(h):
    N, M, p = C.c_int32(), C.c_int32(), C.c_int32()
    rc = load().ellpack_info(h, C.byref(N), C.byref(M), C.byref(p))
    return rc, N.value, M.value, p.value


def ellpack_upload(h, nnz, index, value):
    nnz, index, value = _i32(nnz), _i32(index), _f64(value)
    return load().ellpack_upload(h, _ptr(nnz, i32p), _ptr(index, i32p), _ptr(value, f64p))


def ellpack_download(h):
    """Returns (status, nnz, index, value) as row-major host arrays."""
    rc, N, M, _ = ellpack_info(h)
    nnz = np.zeros(N, np.int32)
    index = np.zeros(N * M, np.int32)
    value = np.zeros(N * M, np.float64)
    if rc == ELL_OK:
        rc = load().ellpack_download(h, _ptr(nnz, i32p), _ptr(index, i32p), _ptr(value, f64p))
    return rc, nnz, index, value


# ---- operations -----------------------------------------------------------------------
def ellpack_x2_threshold(X, X2, tau):
    """Returns (status, (TrX, TrX2), max_row_width)."""
    tr = np.zeros(2)
    w = C.c_int32(0)
    rc = load().ellpack_x2_threshold(X, X2, float(tau), _ptr(tr, f64p), C.byref(w))
    return rc, (tr[0], tr[1]), w.value


def ellpack_x2_step(X, X2, U, tau):
    """Returns (status, (TrX, TrX2, eta2), (width X2, width U))."""
    out = np.zeros(3)
    w = np.zeros(2, np.int32)
    rc = load().ellpack_x2_step(X, X2, U, float(tau), _ptr(out, f64p), _ptr(w, i32p))
    return rc, tuple(out), tuple(int(x) for x in w)


def ellpack_x2_step_noalloc(X, X2, U, tau):
    """ellpack_x2_step with its intermediates in the library's fixed device
    scratch (no device allocation).  Returns as ellpack_x2_step."""
    out = np.zeros(3)
    w = np.zeros(2, np.int32)
    rc = load().ellpack_x2_step_noalloc(X, X2, U, float(tau), _ptr(out, f64p), _ptr(w, i32p))
    return rc, tuple(out), tuple(int(x) for x in w)


def ellpack_trace(h):
    t = C.c_double(0)
    rc = load().ellpack_trace(h, C.byref(t))
    return rc, t.value


def ellpack_trace_product(a, b):
    """Tr(AB) = sum_ij A_ij B_ji."""
    t = C.c_double(0)
    rc = load().ellpack_trace_product(a, b, C.byref(t))
    return rc, t.value


def sp2_params(n_occ, tau, idem_target, max_iter=100, precision=SP2_F64, fp64_tail_steps=2,
               poll_every=4, tau_fp32=1e-7, switch_eta=1e-3, stall_stop=1, profile=0, prune_once=0):
    return SP2Params(float(n_occ), float(tau), float(idem_target), int(max_iter), int(precision),
                     int(fp64_tail_steps), int(poll_every), float(tau_fp32), float(switch_eta),
                     int(stall_stop), int(profile), int(prune_once))


class _Hist:
    def __init__(self, n):
        n = max(1, n)
        self.trx = np.zeros(n)
        self.trx2 = np.zeros(n)
        self.eta2 = np.zeros(n)
        self.up = np.zeros(n, np.int8)
        self.maxw = np.zeros(n, np.int32)
        self.prec = np.zeros(n, np.int8)
        self.x2_seconds = np.zeros(n)
        self.x2_bytes = np.zeros(n, np.int64)

    def attach(self, r):
        r.hist_trx = _ptr(self.trx, f64p)
        r.hist_trx2 = _ptr(self.trx2, f64p)
        r.hist_eta2 = _ptr(self.eta2, f64p)
        r.hist_up = _ptr(self.up, i8p)
        r.hist_maxw = _ptr(self.maxw, i32p)
        r.hist_prec = _ptr(self.prec, i8p)
        r.hist_x2_seconds = _ptr(self.x2_seconds, f64p)
        r.hist_x2_bytes = _ptr(self.x2_bytes, i64p)


def _report(r, h):
    n = r.iterations
    d = {k: getattr(r, k) for k, _ in SP2Report._fields_ if not k.startswith("hist_")}
    if h is not None:
        d.update(trx=h.trx[:n].copy(), trx2=h.trx2[:n].copy(), eta2=h.eta2[:n].copy(), up=h.up[:n].copy(),
                 maxw=h.maxw[:n].copy(), prec=h.prec[:n].copy(),
                 x2_seconds_each=h.x2_seconds[:r.x2_launches].copy(), x2_bytes_each=h.x2_bytes[:n].copy())
    return d


def sp2_solve(H, D, params, history=True):
    """Returns (status, report dict)."""
    r = SP2Report()
    h = _Hist(params.max_iter) if history else None
    if h is not None:
        h.attach(r)
    rc = load().sp2_solve(H, D, C.byref(params), C.byref(r))
    return rc, _report(r, h)


def sp2_solve_batched(Hs, Ds, params, history=True):
    """params: one SP2Params for every instance, or a list of n."""
    n = len(Hs)
    Ha = (vp * n)(*[h.value if isinstance(h, vp) else h for h in Hs])
    Da = (vp * n)(*[d.value if isinstance(d, vp) else d for d in Ds])
    plist = list(params) if isinstance(params, (list, tuple)) else [params] * n
    if len(plist) != n:
        raise ValueError("one parameter set per instance")
    pa = (SP2Params * max(n, 1))(*plist)
    reps = (SP2Report * n)()
    hs = []
    for q in range(n):
        h = _Hist(plist[q].max_iter) if history else None
        if h is not None:
            h.attach(reps[q])
        hs.append(h)
    rc = load().sp2_solve_batched(n, Ha, Da, pa, reps)
    return rc, [_report(reps[q], hs[q]) for q in range(n)]


def dense_x2(d_A, d_C, N, mode, stream=None):
    return load().dense_x2(vp(d_A), vp(d_C), int(N), int(mode), _stream(stream))


def dense_sp2_solve(d_H, N, d_D, mode, params, stream=None, history=True):
    r = SP2Report()
    h = _Hist(params.max_iter) if history else None
    if h is not None:
        h.attach(r)
    rc = load().dense_sp2_solve(vp(d_H), int(N), vp(d_D), int(mode), C.byref(params), C.byref(r),
                                _stream(stream))
    return rc, _report(r, h)


def ellpack_strerror(status):
    return load().ellpack_strerror(int(status)).decode()


def ellpack_last_device_error():
    return load().ellpack_last_device_error().decode()


# ---- convenience: an owned device matrix ------------------------------------------------
class DeviceEll:
    """An ellpack_alloc'ed matrix that frees itself."""

    def __init__(self, N, M, prec=ELL_F64, stream=None):
        rc, self.h = ellpack_alloc(N, M, prec, stream)
        _check(rc, "ellpack_alloc")
        self.N, self.M, self.prec = int(N), int(M), prec

    @classmethod
    def from_host(cls, N, M, nnz, index, value, prec=ELL_F64, capacity=None, stream=None):
        cap = int(capacity or M)
        obj = cls(N, cap, prec, stream)
        if cap != M:
            idx2 = np.full((N, cap), -1, np.int32)
            val2 = np.zeros((N, cap))
            w = min(M, cap)
            idx2[:, :w] = np.asarray(index).reshape(N, M)[:, :w]
            val2[:, :w] = np.asarray(value).reshape(N, M)[:, :w]
            index, value = idx2.reshape(-1), val2.reshape(-1)
        _check(ellpack_upload(obj.h, nnz, index, value), "ellpack_upload")
        return obj

    def download(self):
        rc, nnz, idx, val = ellpack_download(self.h)
        _check(rc, "ellpack_download")
        _, N, M, _ = ellpack_info(self.h)
        return N, M, nnz, idx, val

    def free(self):
        if self.h:
            ellpack_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
