"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds no arithmetic of the method itself (no product, pruning,
trace, norm or purification step).  It only produces Hamiltonians in the
shape of the paper's workloads and moves matrices between storage forms.

Random numbers come from a counter-based generator, so every entry is a pure
function of (seed, stream, i, j, tag):

* splitmix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014) is used as a 64-bit mixing function;
* a 53-bit uniform in [0, 1) is the top 53 bits of the hash times 2^-53;
* normals use the Box-Muller transform of two such uniforms.

Workload (the paper measures model Hamiltonians from an external library that
is not available, section "On the Generation of Model Hamiltonian System
Matrices"; these banded matrices stand in for them):

* H_ii ~ N(0, 1);
* H_ij = H_ji = exp(-0.5 |i - j|) * U(-1, 1) for 0 < |i - j| <= b;
* zero elsewhere.

Matrices are returned in row-major ELLPACK form (the field set of the paper's
ELLPACK listings in the NUMA-aware-data section: N, M, nnz[N], index[N*M],
value[N*M]); row i occupies slots i*M .. i*M + nnz[i] - 1, columns strictly
ascending, unused slots hold index -1 and value 0.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

TAG_DIAG_U1 = 1
TAG_DIAG_U2 = 2
TAG_OFFDIAG = 3
TAG_INSTANCE = 4


def splitmix64(x):
    """splitmix64 finaliser applied elementwise to a uint64 array (wrapping arithmetic)."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def counter_hash(seed, stream, i, j, tag):
    """64-bit hash of the counter tuple (seed, stream, i, j, tag); array-broadcasting."""
    h = splitmix64(np.uint64(seed))
    h = splitmix64(h ^ np.uint64(stream))
    h = splitmix64(h ^ np.uint64(tag))
    i = np.asarray(i, dtype=np.uint64)
    j = np.asarray(j, dtype=np.uint64)
    h = splitmix64(h ^ ((i << np.uint64(32)) | j))
    return h


def uniform01(h):
    """Top 53 bits of a uint64 hash -> float64 in [0, 1)."""
    return (np.asarray(h, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def _normal(seed, stream, i):
    u1 = 1.0 - uniform01(counter_hash(seed, stream, i, i, TAG_DIAG_U1))  # (0, 1]
    u2 = uniform01(counter_hash(seed, stream, i, i, TAG_DIAG_U2))
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def banded_hamiltonian(N, b, seed=0, stream=0, M=None):
    """Symmetric banded H in row-major ELLPACK form.

    Returns (nnz int32[N], index int32[N*M], value float64[N*M], M).  M defaults
    to the band capacity min(N, 2b+1).  All band entries are stored.
    """
    N = int(N)
    b = int(b)
    if N <= 0 or b < 0:
        raise ValueError("N must be positive and b non-negative")
    width = min(N, 2 * b + 1)
    if M is None:
        M = width
    if M < width:
        raise ValueError(f"M={M} is smaller than the band width {width}")
    rows = np.arange(N, dtype=np.int64)
    offs = np.arange(-b, b + 1, dtype=np.int64)
    cols = rows[:, None] + offs[None, :]              # N x (2b+1)
    valid = (cols >= 0) & (cols < N)
    lo = np.minimum(rows[:, None], cols)
    hi = np.maximum(rows[:, None], cols)
    lo_c = np.where(valid, lo, 0)
    hi_c = np.where(valid, hi, 0)
    u = uniform01(counter_hash(seed, stream, lo_c, hi_c, TAG_OFFDIAG))
    off = np.exp(-0.5 * np.abs(offs[None, :]).astype(np.float64)) * (2.0 * u - 1.0)
    diag = _normal(seed, stream, rows)
    vals = np.where(offs[None, :] == 0, diag[:, None], off)
    nnz = valid.sum(axis=1).astype(np.int32)
    index = np.full((N, M), -1, dtype=np.int32)
    value = np.zeros((N, M), dtype=np.float64)
    # pack valid band entries left-aligned per row, ascending columns
    order = np.argsort(~valid, axis=1, kind="stable")
    packed_cols = np.take_along_axis(cols, order, axis=1)[:, :width]
    packed_vals = np.take_along_axis(vals, order, axis=1)[:, :width]
    slot = np.arange(width)[None, :] < nnz[:, None]
    index[:, :width] = np.where(slot, packed_cols, -1).astype(np.int32)
    value[:, :width] = np.where(slot, packed_vals, 0.0)
    return nnz, index.reshape(-1), value.reshape(-1), int(M)


def dense_hamiltonian(N, b, seed=0, stream=0):
    """The same H as banded_hamiltonian, as a dense row-major float64 N x N array."""
    nnz, idx, val, M = banded_hamiltonian(N, min(b, max(N - 1, 0)), seed, stream)
    return ell_to_dense(N, M, nnz, idx, val)


def batched_instances(count=256, seed=0, n_min=64, n_max=2048):
    """Sizes of the batched workload: N_m uniform in [n_min, n_max], b_m = max(4, N_m // 32)."""
    m = np.arange(count, dtype=np.uint64)
    h = counter_hash(seed, 0, m, 0, TAG_INSTANCE)
    span = np.uint64(n_max - n_min + 1)
    n = (h % span).astype(np.int64) + n_min
    b = np.maximum(4, n // 32)
    return [(int(n[k]), int(b[k])) for k in range(count)]


# ---- storage moves (no arithmetic) -------------------------------------------------

def ell_to_dense(N, M, nnz, idx, val, dtype=np.float64):
    nnz = np.asarray(nnz)
    idx = np.asarray(idx).reshape(N, M)
    val = np.asarray(val).reshape(N, M)
    D = np.zeros((N, N), dtype=dtype)
    slot = np.arange(M)[None, :] < nnz[:, None]
    r = np.repeat(np.arange(N)[:, None], M, axis=1)
    D[r[slot], idx[slot]] = val[slot]
    return D


def dense_to_ell(D, M=None, dtype=np.float64):
    """Row-major ELLPACK of the nonzero entries of a dense matrix (exact zeros dropped)."""
    D = np.asarray(D)
    N = D.shape[0]
    nz = D != 0
    nnz = nz.sum(axis=1).astype(np.int32)
    if M is None:
        M = max(1, int(nnz.max()) if N else 1)
    if N and nnz.max() > M:
        raise ValueError("M too small for this matrix")
    index = np.full((N, M), -1, dtype=np.int32)
    value = np.zeros((N, M), dtype=dtype)
    for i in range(N):
        c = np.nonzero(nz[i])[0]
        index[i, : c.size] = c
        value[i, : c.size] = D[i, c]
    return nnz, index.reshape(-1), value.reshape(-1), int(M)


def ell_rows(N, M, nnz, idx, val):
    """List of (columns, values) per row, for readable comparisons in tests."""
    idx = np.asarray(idx).reshape(N, M)
    val = np.asarray(val).reshape(N, M)
    return [(idx[i, : nnz[i]].copy(), val[i, : nnz[i]].copy()) for i in range(N)]
