"""Shared helpers of the GPU tests: upload/download through the C ABI and
bitwise comparisons against the oracle's row-major ELLPACK matrices."""
import numpy as np

import oracle
from paper_2102_08505_amd import ellsp2 as E


def dev_from_oracle(A, prec=E.ELL_F64, capacity=None):
    """Upload an oracle.Ell (values given to the library in double)."""
    cap = capacity or max(1, A.M)
    return E.DeviceEll.from_host(A.N, A.M, A.nnz, A.idx, A.val.astype(np.float64), prec=prec, capacity=cap)


def oracle_from_dev(D, f32=False):
    N, M, nnz, idx, val = D.download()
    if f32:
        val = val.astype(np.float32)
    return oracle.Ell(N, M, nnz, idx, val)


def assert_same_rows(got, want, what=""):
    """Bitwise equality of two oracle.Ell matrices (patterns and values)."""
    assert got.N == want.N
    assert np.array_equal(got.nnz, want.nnz), f"{what}: row widths differ at rows " \
        f"{np.nonzero(got.nnz != want.nnz)[0][:10]}"
    gi = got.idx.reshape(got.N, got.M)
    wi = want.idx.reshape(want.N, want.M)
    gv = got.val.reshape(got.N, got.M)
    wv = want.val.reshape(want.N, want.M)
    w = int(want.nnz.max()) if want.N else 0
    mask = np.arange(w)[None, :] < want.nnz[:, None]
    gi, wi, gv, wv = gi[:, :w], wi[:, :w], gv[:, :w], wv[:, :w]
    bad = mask & ((gi != wi) | (gv.view(np.uint64 if gv.dtype == np.float64 else np.uint32)
                                != wv.view(np.uint64 if wv.dtype == np.float64 else np.uint32)))
    if bad.any():
        r, c = np.argwhere(bad)[0]
        raise AssertionError(f"{what}: first difference at row {r} slot {c}: got ({gi[r, c]}, {gv[r, c]!r}) "
                             f"want ({wi[r, c]}, {wv[r, c]!r}); {bad.sum()} differing entries")


def same_float(a, b):
    """Bitwise equality of two floats, treating +0 and -0 as equal."""
    a, b = float(a), float(b)
    return a == b and (a != a) == (b != b) or (a != a and b != b)
