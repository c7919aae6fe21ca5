"""ctypes binding of the CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports this
package and this package never imports the GPU library.

Parity status of each function (what pins it is in tests/test_oracle_pins.py):
  pairwise, x2 (f64 and f32), trace, norm2, update, gershgorin, x0, sp2 (f64):
      pinned (brute force / exact rational arithmetic / closed forms /
      eigendecomposition / invariants);
  sp2 mixed mode: pinned by invariants and by the FP64 projector within the
      FP32 error scale;
  dense_x2_bf16x3, dense_sp2: pinned by the exact-rational bound on the split
      product and by the FP64 projector.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ENOMEM, EOVERFLOW, ENOCONV, ENONFINITE, EDEGENERATE = 0, -1, -2, -3, -4, -7, -8
PREC_F64, PREC_MIXED = 0, 1
DENSE_F64, DENSE_BF16X3 = 0, 1


def build(force=True):
    """Compile liboracle.so with gcc (plain C11, no FP contraction, OpenMP row loops)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-o", tmp, _SRC, os.path.join(_HERE, "host_stream.c"), "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None

i32p = C.POINTER(C.c_int32)
i8p = C.POINTER(C.c_int8)
f64p = C.POINTER(C.c_double)
f32p = C.POINTER(C.c_float)


class SP2Params(C.Structure):
    _fields_ = [("n_occ", C.c_double), ("tau", C.c_double), ("idem_target", C.c_double),
                ("max_iter", C.c_int32), ("precision", C.c_int32), ("fp64_tail_steps", C.c_int32),
                ("stall_stop", C.c_int32), ("tau_fp32", C.c_double), ("switch_eta", C.c_double),
                ("prune_once", C.c_int32)]


class SP2Report(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("fp32_iterations", C.c_int32),
                ("final_M", C.c_int32), ("eta", C.c_double), ("trace_x", C.c_double),
                ("emin", C.c_double), ("emax", C.c_double),
                ("hist_trx", f64p), ("hist_trx2", f64p), ("hist_eta2", f64p),
                ("hist_up", i8p), ("hist_maxw", i32p), ("hist_prec", i8p)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        L.orc_pairwise.restype = C.c_double
        L.orc_pairwise.argtypes = [C.c_int64, f64p]
        L.orc_check_ell.argtypes = [C.c_int32, C.c_int32, i32p, i32p]
        L.orc_x2_fma_count.restype = C.c_int64
        L.orc_x2_fma_count.argtypes = [C.c_int32, C.c_int32, i32p, i32p]
        L.orc_x2_rows_f64.argtypes = [C.c_int32, C.c_int32, i32p, i32p, f64p, C.c_double, C.c_int32, i32p,
                                      C.c_int32, i32p, i32p, f64p, f64p]
        L.orc_prune_f64.argtypes = [C.c_int32, C.c_int32, i32p, i32p, f64p, C.c_double, C.c_int32,
                                    i32p, i32p, f64p, i32p]
        L.orc_prune_f32.argtypes = [C.c_int32, C.c_int32, i32p, i32p, f32p, C.c_float, C.c_int32,
                                    i32p, i32p, f32p, i32p]
        L.orc_threads.restype = C.c_int32
        L.orc_threads.argtypes = [C.c_int32]
        L.orc_rows_init.restype = None
        L.orc_rows_init.argtypes = [C.c_int32, C.c_int32, i32p, i32p, C.c_void_p, C.c_int32]
        L.orc_stream_triad.restype = C.c_double
        L.orc_stream_triad.argtypes = [C.c_int64, C.c_int32]
        L.orc_x2_f64.argtypes = [C.c_int32, C.c_int32, i32p, i32p, f64p, C.c_double, C.c_int32,
                                 i32p, i32p, f64p, f64p, f64p, i32p]
        L.orc_x2_f32.argtypes = [C.c_int32, C.c_int32, i32p, i32p, f32p, C.c_float, C.c_int32,
                                 i32p, i32p, f32p, f64p, f64p, i32p]
        L.orc_trace_f64.restype = C.c_double
        L.orc_trace_f64.argtypes = [C.c_int32, C.c_int32, i32p, i32p, f64p]
        L.orc_trace_product_f64.restype = C.c_double
        L.orc_trace_product_f64.argtypes = [C.c_int32, C.c_int32, i32p, i32p, f64p, C.c_int32, i32p, i32p, f64p]
        L.orc_norm2_f64.restype = C.c_double
        L.orc_norm2_f64.argtypes = [C.c_int32, C.c_int32, i32p, i32p, f64p, C.c_int32, i32p, i32p,
                                    f64p, f64p]
        L.orc_norm2_f32.restype = C.c_double
        L.orc_norm2_f32.argtypes = [C.c_int32, C.c_int32, i32p, i32p, f32p, C.c_int32, i32p, i32p,
                                    f32p, f64p]
        L.orc_update_f64.argtypes = [C.c_int32, C.c_int32, i32p, i32p, f64p, C.c_int32, i32p, i32p,
                                     f64p, C.c_double, C.c_int32, i32p, i32p, f64p, i32p]
        L.orc_update_f32.argtypes = [C.c_int32, C.c_int32, i32p, i32p, f32p, C.c_int32, i32p, i32p,
                                     f32p, C.c_float, C.c_int32, i32p, i32p, f32p, i32p]
        L.orc_gershgorin.argtypes = [C.c_int32, C.c_int32, i32p, i32p, f64p, f64p, f64p]
        L.orc_x0_f64.argtypes = [C.c_int32, C.c_int32, i32p, i32p, f64p, C.c_double, C.c_double,
                                 C.c_double, C.c_int32, i32p, i32p, f64p, i32p]
        L.orc_x0_f32.argtypes = [C.c_int32, C.c_int32, i32p, i32p, f64p, C.c_double, C.c_double,
                                 C.c_float, C.c_int32, i32p, i32p, f32p, i32p]
        L.orc_sp2.argtypes = [C.c_int32, C.c_int32, i32p, i32p, f64p, C.POINTER(SP2Params), C.c_int32,
                              i32p, i32p, f64p, C.POINTER(SP2Report)]
        L.orc_dense_x2_f64.restype = None
        L.orc_dense_x2_f64.argtypes = [C.c_int32, f64p, f64p]
        L.orc_bf16_rne.restype = C.c_float
        L.orc_bf16_rne.argtypes = [C.c_float]
        L.orc_dense_x2_bf16x3.restype = None
        L.orc_dense_x2_bf16x3.argtypes = [C.c_int32, f32p, f32p]
        L.orc_dense_sp2.argtypes = [C.c_int32, f64p, C.c_int32, C.POINTER(SP2Params), f64p,
                                    C.POINTER(SP2Report)]
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


class Ell:
    """Row-major ELLPACK matrix held in numpy arrays (oracle side)."""

    def __init__(self, N, M, nnz, idx, val):
        self.N, self.M = int(N), int(M)
        self.nnz = _i32(nnz)
        self.idx = _i32(idx).reshape(-1)
        self.val = np.ascontiguousarray(val).reshape(-1)

    @property
    def dtype(self):
        return self.val.dtype

    def rows(self):
        ix = self.idx.reshape(self.N, self.M)
        vx = self.val.reshape(self.N, self.M)
        return [(ix[i, : self.nnz[i]].copy(), vx[i, : self.nnz[i]].copy()) for i in range(self.N)]

    def dense(self):
        D = np.zeros((self.N, self.N), dtype=np.float64)
        for i, (c, v) in enumerate(self.rows()):
            D[i, c] = v
        return D

    def max_width(self):
        return int(self.nnz.max()) if self.N else 0


def pairwise(d):
    d = _f64(d)
    return lib().orc_pairwise(d.size, _p(d, f64p))


def check_ell(A):
    return lib().orc_check_ell(A.N, A.M, _p(A.nnz, i32p), _p(A.idx, i32p))


def fma_count(A):
    return int(lib().orc_x2_fma_count(A.N, A.M, _p(A.nnz, i32p), _p(A.idx, i32p)))


def x2_rows(A, tau, rows, M2):
    """(status, nnz[nr], idx[nr, M2], val[nr, M2], d2[nr]): rows `rows` of the
    FP64 prune(A.A, tau), each as x2 computes it."""
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    nr = rows.size
    nnz2 = np.zeros(nr, np.int32)
    idx2 = np.full(nr * M2, -1, np.int32)
    val2 = np.zeros(nr * M2, np.float64)
    d2 = np.zeros(nr)
    rc = lib().orc_x2_rows_f64(A.N, A.M, _p(A.nnz, i32p), _p(A.idx, i32p), _p(_f64(A.val), f64p), float(tau), nr,
                               _p(rows, i32p), M2, _p(nnz2, i32p), _p(idx2, i32p), _p(val2, f64p), _p(d2, f64p))
    return rc, nnz2, idx2.reshape(nr, M2), val2.reshape(nr, M2), d2


def threads(n=0):
    """Sets the oracle's OpenMP thread count when n > 0; returns the count in use."""
    return int(lib().orc_threads(int(n)))


def stream_triad(n, reps=10):
    """Host memory bandwidth (GB/s), best of `reps` STREAM triads over n doubles."""
    return float(lib().orc_stream_triad(int(n), int(reps)))


def empty_rows(N, M, dtype):
    """(nnz, idx, val) of an N x M ELLPACK matrix with nothing stored, first
    touched row by row in the oracle's static row schedule."""
    nnz = np.empty(N, np.int32)
    idx = np.empty(N * M, np.int32)
    val = np.empty(N * M, dtype)
    lib().orc_rows_init(N, M, _p(nnz, i32p), _p(idx, i32p), val.ctypes.data, val.itemsize)
    return nnz, idx, val


def x2(A, tau, M2=None):
    """Returns (status, X2 Ell, d1, d2, maxw).  FP64 or FP32 by A's value dtype."""
    L = lib()
    N = A.N
    if M2 is None:
        M2 = N
    nnz2, idx2, val2 = empty_rows(N, M2, A.val.dtype)
    d1 = np.zeros(N)
    d2 = np.zeros(N)
    w = C.c_int32(0)
    if A.val.dtype == np.float32:
        rc = L.orc_x2_f32(N, A.M, _p(A.nnz, i32p), _p(A.idx, i32p), _p(A.val, f32p), C.c_float(tau),
                          M2, _p(nnz2, i32p), _p(idx2, i32p), _p(val2, f32p), _p(d1, f64p),
                          _p(d2, f64p), C.byref(w))
    else:
        rc = L.orc_x2_f64(N, A.M, _p(A.nnz, i32p), _p(A.idx, i32p), _p(A.val, f64p), float(tau), M2,
                          _p(nnz2, i32p), _p(idx2, i32p), _p(val2, f64p), _p(d1, f64p),
                          _p(d2, f64p), C.byref(w))
    return rc, Ell(N, M2, nnz2, idx2, val2), d1, d2, int(w.value)


def trace(A):
    return lib().orc_trace_f64(A.N, A.M, _p(A.nnz, i32p), _p(A.idx, i32p), _p(_f64(A.val), f64p))


def trace_product(A, B):
    """Tr(AB) = sum_ij A_ij B_ji (FP32 values widened to double)."""
    assert A.N == B.N
    return lib().orc_trace_product_f64(A.N, A.M, _p(A.nnz, i32p), _p(A.idx, i32p), _p(_f64(A.val), f64p),
                                       B.M, _p(B.nnz, i32p), _p(B.idx, i32p), _p(_f64(B.val), f64p))


def norm2(X, Y):
    """(eta^2, row terms e) for ||Y - X||_F^2 over the union pattern."""
    e = np.zeros(X.N)
    L = lib()
    if X.val.dtype == np.float32:
        s = L.orc_norm2_f32(X.N, X.M, _p(X.nnz, i32p), _p(X.idx, i32p), _p(X.val, f32p), Y.M,
                            _p(Y.nnz, i32p), _p(Y.idx, i32p), _p(Y.val, f32p), _p(e, f64p))
    else:
        s = L.orc_norm2_f64(X.N, X.M, _p(X.nnz, i32p), _p(X.idx, i32p), _p(X.val, f64p), Y.M,
                            _p(Y.nnz, i32p), _p(Y.idx, i32p), _p(Y.val, f64p), _p(e, f64p))
    return s, e


def update(X, Y, tau, Mo=None):
    """(status, prune(2X - Y), maxw)."""
    N = X.N
    if Mo is None:
        Mo = N
    nnzo, idxo, valo = empty_rows(N, Mo, X.val.dtype)
    w = C.c_int32(0)
    L = lib()
    if X.val.dtype == np.float32:
        rc = L.orc_update_f32(N, X.M, _p(X.nnz, i32p), _p(X.idx, i32p), _p(X.val, f32p), Y.M,
                              _p(Y.nnz, i32p), _p(Y.idx, i32p), _p(Y.val, f32p), C.c_float(tau), Mo,
                              _p(nnzo, i32p), _p(idxo, i32p), _p(valo, f32p), C.byref(w))
    else:
        rc = L.orc_update_f64(N, X.M, _p(X.nnz, i32p), _p(X.idx, i32p), _p(X.val, f64p), Y.M,
                              _p(Y.nnz, i32p), _p(Y.idx, i32p), _p(Y.val, f64p), float(tau), Mo,
                              _p(nnzo, i32p), _p(idxo, i32p), _p(valo, f64p), C.byref(w))
    return rc, Ell(N, Mo, nnzo, idxo, valo), int(w.value)


def prune(Y, tau, Mo=None):
    """(status, prune(Y, tau), maxw): the entries with |v| > tau."""
    N = Y.N
    if Mo is None:
        Mo = max(Y.M, 1)
    nnzo, idxo, valo = empty_rows(N, Mo, Y.val.dtype)
    w = C.c_int32(0)
    L = lib()
    if Y.val.dtype == np.float32:
        rc = L.orc_prune_f32(N, Y.M, _p(Y.nnz, i32p), _p(Y.idx, i32p), _p(Y.val, f32p), C.c_float(tau), Mo,
                             _p(nnzo, i32p), _p(idxo, i32p), _p(valo, f32p), C.byref(w))
    else:
        rc = L.orc_prune_f64(N, Y.M, _p(Y.nnz, i32p), _p(Y.idx, i32p), _p(Y.val, f64p), float(tau), Mo,
                             _p(nnzo, i32p), _p(idxo, i32p), _p(valo, f64p), C.byref(w))
    return rc, Ell(N, Mo, nnzo, idxo, valo), int(w.value)


def gershgorin(H):
    lo, hi = C.c_double(0), C.c_double(0)
    rc = lib().orc_gershgorin(H.N, H.M, _p(H.nnz, i32p), _p(H.idx, i32p), _p(_f64(H.val), f64p),
                              C.byref(lo), C.byref(hi))
    return rc, lo.value, hi.value


def x0(H, emin, emax, tau, Mo=None, fp32=False):
    N = H.N
    if Mo is None:
        Mo = H.M + 1
    nnzo = np.zeros(N, np.int32)
    idxo = np.full(N * Mo, -1, np.int32)
    w = C.c_int32(0)
    L = lib()
    if fp32:
        valo = np.zeros(N * Mo, np.float32)
        rc = L.orc_x0_f32(N, H.M, _p(H.nnz, i32p), _p(H.idx, i32p), _p(_f64(H.val), f64p), emin, emax,
                          C.c_float(tau), Mo, _p(nnzo, i32p), _p(idxo, i32p), _p(valo, f32p), C.byref(w))
    else:
        valo = np.zeros(N * Mo, np.float64)
        rc = L.orc_x0_f64(N, H.M, _p(H.nnz, i32p), _p(H.idx, i32p), _p(_f64(H.val), f64p), emin, emax,
                          float(tau), Mo, _p(nnzo, i32p), _p(idxo, i32p), _p(valo, f64p), C.byref(w))
    return rc, Ell(N, Mo, nnzo, idxo, valo), int(w.value)


def make_params(n_occ, tau, idem_target, max_iter=100, precision=PREC_F64, fp64_tail_steps=2,
                stall_stop=1, tau_fp32=1e-7, switch_eta=1e-3, prune_once=0):
    return SP2Params(float(n_occ), float(tau), float(idem_target), int(max_iter), int(precision),
                     int(fp64_tail_steps), int(stall_stop), float(tau_fp32), float(switch_eta),
                     int(prune_once))


class _Hist:
    def __init__(self, n):
        self.trx = np.zeros(n)
        self.trx2 = np.zeros(n)
        self.eta2 = np.zeros(n)
        self.up = np.zeros(n, np.int8)
        self.maxw = np.zeros(n, np.int32)
        self.prec = np.zeros(n, np.int8)

    def report(self):
        r = SP2Report()
        r.hist_trx = _p(self.trx, f64p)
        r.hist_trx2 = _p(self.trx2, f64p)
        r.hist_eta2 = _p(self.eta2, f64p)
        r.hist_up = _p(self.up, i8p)
        r.hist_maxw = _p(self.maxw, i32p)
        r.hist_prec = _p(self.prec, i8p)
        return r


def _report_dict(r, h):
    n = r.iterations
    return dict(status=r.status, iterations=n, fp32_iterations=r.fp32_iterations, final_M=r.final_M,
                eta=r.eta, trace_x=r.trace_x, emin=r.emin, emax=r.emax,
                trx=h.trx[:n].copy(), trx2=h.trx2[:n].copy(), eta2=h.eta2[:n].copy(),
                up=h.up[:n].copy(), maxw=h.maxw[:n].copy(), prec=h.prec[:n].copy())


def sp2(H, params, Mo=None):
    """(status, D Ell, report dict)."""
    N = H.N
    if Mo is None:
        Mo = N
    nnzD = np.zeros(N, np.int32)
    idxD = np.full(N * Mo, -1, np.int32)
    valD = np.zeros(N * Mo, np.float64)
    h = _Hist(max(1, params.max_iter))
    r = h.report()
    rc = lib().orc_sp2(N, H.M, _p(H.nnz, i32p), _p(H.idx, i32p), _p(_f64(H.val), f64p),
                       C.byref(params), Mo, _p(nnzD, i32p), _p(idxD, i32p), _p(valD, f64p), C.byref(r))
    return rc, Ell(N, Mo, nnzD, idxD, valD), _report_dict(r, h)


def dense_x2_f64(A):
    A = _f64(A)
    Cm = np.zeros_like(A)
    lib().orc_dense_x2_f64(A.shape[0], _p(A, f64p), _p(Cm, f64p))
    return Cm


def bf16_rne(x):
    return np.float32(lib().orc_bf16_rne(C.c_float(x)))


def dense_x2_bf16x3(A):
    A = _f32(A)
    Cm = np.zeros_like(A)
    lib().orc_dense_x2_bf16x3(A.shape[0], _p(A, f32p), _p(Cm, f32p))
    return Cm


def dense_sp2(H, mode, params):
    H = _f64(H)
    N = H.shape[0]
    D = np.zeros_like(H)
    h = _Hist(max(1, params.max_iter))
    r = h.report()
    rc = lib().orc_dense_sp2(N, _p(H, f64p), int(mode), C.byref(params), _p(D, f64p), C.byref(r))
    return rc, D, _report_dict(r, h)
