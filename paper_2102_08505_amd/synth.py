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

Workloads: the paper's own model Hamiltonians (model_hamiltonian: metals,
semiconductors and soft matter, section "On the Generation of Model
Hamiltonian System Matrices", rebuilt from the text since the generator it used
is not available), and the banded matrices the benchmark and most tests use:

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
TAG_MODEL_ONSITE = 5
TAG_MODEL_COUPLING = 6


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


# ---- the paper's model Hamiltonians -----------------------------------------------
#
# Section "On the Generation of Model Hamiltonian System Matrices": a chain of
# two-level systems, each with an A and a B orbital (onsite energies eps_A,
# eps_B); orbitals of the same type couple with delta_AA or delta_BB, of
# different types with delta_AB; every coupling is damped by exp(k |j - i|) for
# orbital positions i, j; a noise parameter r turns each onsite energy and
# coupling `param` into param * (1 + r * RAND), RAND uniform in [-1, 1].  The
# section's three parameter sets follow; parameters it does not name are 0.
#
# Readings where the text leaves a choice: orbital i is of type A for even i and
# B for odd i (site i // 2), positions are orbital indices; RAND is drawn once
# per orbital (onsite) and once per unordered pair (coupling), so H is
# symmetric; an entry is stored when its magnitude exceeds the drop threshold
# `thr` (the coupling decays but never vanishes, and the printed sparsities do
# not fix a cut-off), default 1e-5.
MODEL_PARAMS = {
    "metal": dict(eps_a=0.0, eps_b=0.0, d_aa=-1.0, d_bb=-1.0, d_ab=0.0, k=-0.01, r=0.0),
    "semiconductor": dict(eps_a=0.0, eps_b=0.0, d_aa=0.0, d_bb=-1.0, d_ab=-2.0, k=-0.01, r=0.0),
    "soft_matter": dict(eps_a=-10.0, eps_b=0.0, d_aa=0.0, d_bb=-1.0, d_ab=-1.0, k=-0.1, r=1.0),
}


def model_reach(kind, thr=1e-5):
    """Largest |j - i| at which a coupling of `kind` can exceed thr."""
    p = MODEL_PARAMS[kind]
    top = max(abs(p["d_aa"]), abs(p["d_bb"]), abs(p["d_ab"])) * (1.0 + p["r"])
    if top <= thr:
        return 0
    return int(np.floor(np.log(top / thr) / -p["k"]))


def _model_rows(kind, N, r0, r1, seed, stream, reach):
    """Dense candidate block of rows r0 .. r1 - 1 over columns i - reach .. i + reach."""
    p = MODEL_PARAMS[kind]
    rows = np.arange(r0, r1, dtype=np.int64)
    offs = np.arange(-reach, reach + 1, dtype=np.int64)
    cols = rows[:, None] + offs[None, :]
    valid = (cols >= 0) & (cols < N)
    cc = np.where(valid, cols, 0)
    lo = np.minimum(rows[:, None], cc)
    hi = np.maximum(rows[:, None], cc)
    ti = (rows[:, None] & 1).astype(bool)  # True: B
    tj = (cc & 1).astype(bool)
    delta = np.where(ti == tj, np.where(ti, p["d_bb"], p["d_aa"]), p["d_ab"])
    val = delta * np.exp(p["k"] * np.abs(offs[None, :]).astype(np.float64))
    onsite = np.where((rows & 1).astype(bool), p["eps_b"], p["eps_a"]).astype(np.float64)
    if p["r"] != 0.0:  # noise: param * (1 + r RAND)
        rnd = 2.0 * uniform01(counter_hash(seed, stream, lo, hi, TAG_MODEL_COUPLING)) - 1.0
        val = val * (1.0 + p["r"] * rnd)
        ron = 2.0 * uniform01(counter_hash(seed, stream, rows, rows, TAG_MODEL_ONSITE)) - 1.0
        onsite = onsite * (1.0 + p["r"] * ron)
    val = np.where(offs[None, :] == 0, onsite[:, None], val)
    return cols, valid, val


def model_hamiltonian(kind, N, seed=0, stream=0, thr=1e-5, M=None, chunk=1024):
    """One of the paper's model Hamiltonians ("metal", "semiconductor",
    "soft_matter") of N orbitals in row-major ELLPACK form.

    Returns (nnz, index, value, M) like banded_hamiltonian; M defaults to the
    widest row.  Rows are built `chunk` at a time over the columns within
    model_reach(kind, thr) of the diagonal.
    """
    if kind not in MODEL_PARAMS:
        raise ValueError(f"unknown model Hamiltonian {kind!r}")
    N = int(N)
    if N <= 0:
        raise ValueError("N must be positive")
    reach = min(model_reach(kind, thr), N - 1)
    counts, flat_cols, flat_vals = [], [], []
    for r0 in range(0, N, chunk):
        r1 = min(N, r0 + chunk)
        cols, valid, val = _model_rows(kind, N, r0, r1, seed, stream, reach)
        keep = valid & (np.abs(val) > thr)
        counts.append(keep.sum(axis=1).astype(np.int32))
        flat_cols.append(cols[keep])  # row by row, ascending columns
        flat_vals.append(val[keep])
    nnz = np.concatenate(counts)
    wmax = int(nnz.max())
    if M is None:
        M = max(1, wmax)
    if M < wmax:
        raise ValueError(f"M={M} is smaller than the widest row {wmax}")
    cols = np.concatenate(flat_cols)
    vals = np.concatenate(flat_vals)
    row = np.repeat(np.arange(N, dtype=np.int64), nnz)
    start = np.concatenate(([0], np.cumsum(nnz, dtype=np.int64)[:-1]))
    slot = np.arange(cols.size, dtype=np.int64) - start[row]
    index = np.full(N * M, -1, dtype=np.int32)
    value = np.zeros(N * M, dtype=np.float64)
    index[row * M + slot] = cols.astype(np.int32)
    value[row * M + slot] = vals
    return nnz, index, value, int(M)


def grid3d_hamiltonian(n, delta=1.0, t=1.0, r=0.1, seed=0, stream=0, M=None):
    """A non-banded pattern: the nearest-neighbour Hamiltonian of an n x n x n
    cubic lattice in lexicographic order (site i = x + n y + n^2 z), onsite
    +delta on sites with x + y + z even and -delta on the others, hopping
    -t (1 + r RAND) to the six neighbours (open boundaries), RAND uniform in
    [-1, 1] once per bond.  Row i holds columns i, i +- 1, i +- n, i +- n^2:
    seven entries spread over 2 n^2 + 1 positions.  For even n the spectrum has
    no eigenvalue in (-delta, delta) and N_occ = n^3 / 2 at the Fermi level 0."""
    n = int(n)
    if n <= 0:
        raise ValueError("n must be positive")
    N = n ** 3
    i = np.arange(N, dtype=np.int64)
    x, y, z = i % n, (i // n) % n, i // (n * n)
    onsite = np.where((x + y + z) % 2 == 0, delta, -delta).astype(np.float64)
    cols = [i]
    vals = [onsite]
    valid = [np.ones(N, dtype=bool)]
    for step, coord in ((1, x), (n, y), (n * n, z)):
        for sgn in (-1, 1):
            j = i + sgn * step
            ok = (coord + sgn >= 0) & (coord + sgn < n)
            jc = np.where(ok, j, 0)
            lo, hi = np.minimum(i, jc), np.maximum(i, jc)
            rnd = 2.0 * uniform01(counter_hash(seed, stream, lo, hi, TAG_MODEL_COUPLING)) - 1.0
            cols.append(jc)
            vals.append(-t * (1.0 + r * rnd))
            valid.append(ok)
    cols = np.stack(cols, axis=1)
    vals = np.stack(vals, axis=1)
    valid = np.stack(valid, axis=1) & (vals != 0.0)
    cols = np.where(valid, cols, np.iinfo(np.int64).max)
    order = np.argsort(cols, axis=1, kind="stable")
    cols = np.take_along_axis(cols, order, axis=1)
    vals = np.take_along_axis(vals, order, axis=1)
    valid = np.take_along_axis(valid, order, axis=1)
    nnz = valid.sum(axis=1).astype(np.int32)
    if M is None:
        M = 7
    if M < 7:
        raise ValueError("M must hold the seven stencil slots")
    index = np.full((N, M), -1, dtype=np.int32)
    value = np.zeros((N, M), dtype=np.float64)
    index[:, :7] = np.where(valid, cols, -1).astype(np.int32)
    value[:, :7] = np.where(valid, vals, 0.0)
    return nnz, index.reshape(-1), value.reshape(-1), int(M)


def fermi_occupation(nnz, idx, val, M, mu=0.0):
    """Number of eigenvalues of the (symmetric) ELLPACK matrix below the Fermi
    level mu -- the occupation N_occ that SP2 is given.  The section on the model
    Hamiltonians sets the Fermi level at 0 eV.  Dense eigenvalues: for the sizes
    the tests and the benchmark run (N up to a few thousand)."""
    N = len(nnz)
    w = np.linalg.eigvalsh(ell_to_dense(N, M, nnz, idx, val))
    return int((w < mu).sum()), w


def fermi_occupation_banded(nnz, idx, val, M, mu=0.0):
    """N_occ without the spectrum, for banded sizes a dense eigensolver does
    not reach (the model Hamiltonians at 32000 orbitals): by Sylvester's law
    of inertia the number of eigenvalues of H below mu equals the number of
    negative eigenvalues of D in any congruence H - mu I = L D L^T.  Rows are
    cut into blocks of the half-bandwidth w, so H - mu I is block tridiagonal
    (diagonal blocks A_k, couplings B_k to the next block) and its block
    LDL^T has the Schur complements S_1 = A_1, S_k = A_k - B_{k-1}^T
    S_{k-1}^{-1} B_{k-1} as D (Haynsworth's inertia additivity).  Costs about
    N w^2 flops against N^3 for the spectrum.

    Returns (N_occ, smallest |eigenvalue| over all S_k): the second is a
    conditioning check; it stays of the order of the gap at mu when mu lies
    in a gap."""
    N = len(nnz)
    nnz = np.asarray(nnz)
    idx2 = np.asarray(idx).reshape(N, M)
    val2 = np.asarray(val).reshape(N, M)
    slot = np.arange(M)[None, :] < nnz[:, None]
    rows = np.repeat(np.arange(N)[:, None], M, axis=1)[slot]  # row-major: rows ascend
    cols = idx2[slot].astype(np.int64)
    vals = val2[slot]
    start = np.concatenate(([0], np.cumsum(nnz, dtype=np.int64)))
    w = max(1, int(np.abs(cols - rows).max(initial=0)))
    count, smallest = 0, np.inf
    C = None  # B_{k-1}^T S_{k-1}^{-1} B_{k-1}
    for s in range(0, N, w):
        e = min(N, s + w)
        e2 = min(N, e + w)
        r, c, v = (a[start[s]:start[e]] for a in (rows, cols, vals))
        sel = c >= s  # the entries left of the block belong to B_{k-1}^T
        blk = np.zeros((e - s, e2 - s))
        blk[r[sel] - s, c[sel] - s] = v[sel]
        S = blk[:, :e - s] - mu * np.eye(e - s)
        if C is not None:
            S = S - C
        S = 0.5 * (S + S.T)
        ev, V = np.linalg.eigh(S)
        count += int((ev < 0).sum())
        smallest = min(smallest, float(np.abs(ev).min()))
        B = blk[:, e - s:]
        if B.shape[1]:
            VB = V.T @ B
            C = VB.T @ (VB / ev[:, None])
    return count, smallest


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
