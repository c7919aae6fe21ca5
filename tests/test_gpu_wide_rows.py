"""Rows wider than 4096 entries (up to the 65536-entry row capacity), on the
GPU against the oracle, bit for bit: products whose output rows are dense
over 5000 columns (span form, matrix cores) and scattered over 20000
(ELLPACK kernels), an SP2 solve whose first product is wider than 4096, and
the paper's semiconductor Hamiltonian squared at its 32000 orbitals (sampled
rows: the whole product is too large for the oracle here)."""
import numpy as np
import pytest

import oracle
from paper_2102_08505_amd import ellsp2 as E
from paper_2102_08505_amd import synth
from tests.gpu_helpers import assert_same_rows, dev_from_oracle, oracle_from_dev, same_float
from tests.test_gpu_parity import random_ell

pytestmark = pytest.mark.gpu


def scattered_symmetric(N, per_row, seed):
    """Symmetric matrix with about 2 per_row random off-diagonal entries per
    row spread over all N columns, plus the diagonal."""
    rng = np.random.default_rng(seed)
    i = np.repeat(np.arange(N), per_row)
    j = rng.integers(0, N, size=N * per_row)
    keep = i != j
    i, j = i[keep], j[keep]
    lo, hi = np.minimum(i, j), np.maximum(i, j)
    key = np.unique(lo.astype(np.int64) * N + hi)
    lo, hi = (key // N).astype(np.int64), (key % N).astype(np.int64)
    v = rng.uniform(-1, 1, size=lo.size) * 0.1
    rows = np.concatenate([lo, hi, np.arange(N)])
    cols = np.concatenate([hi, lo, np.arange(N)])
    vals = np.concatenate([v, v, rng.uniform(-1, 1, size=N)])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    nnz = np.bincount(rows, minlength=N).astype(np.int32)
    M = int(nnz.max())
    start = np.concatenate([[0], np.cumsum(nnz)[:-1]])
    slot = np.arange(rows.size) - start[rows]
    idx = np.full(N * M, -1, np.int32)
    val = np.zeros(N * M)
    idx[rows * M + slot] = cols
    val[rows * M + slot] = vals
    return oracle.Ell(N, M, nnz, idx, val)


def check_step(A, tau, cap):
    rc, Y, d1, d2, wy = oracle.x2(A, tau, M2=cap)
    assert rc == 0 and wy > 4096, wy
    X = dev_from_oracle(A)
    Yd = E.DeviceEll(A.N, cap)
    U = E.DeviceEll(A.N, cap)
    rc_g, out, widths = E.ellpack_x2_step(X.h, Yd.h, U.h, tau)
    assert rc_g == E.ELL_OK, E.ellpack_strerror(rc_g)
    assert_same_rows(oracle_from_dev(Yd), Y, "X^2")
    assert widths[0] == wy
    assert same_float(out[0], oracle.pairwise(d1)) and same_float(out[1], oracle.pairwise(d2))
    eta2, _ = oracle.norm2(A, Y)
    assert same_float(out[2], eta2)
    rcu, Uo, wu = oracle.update(A, Y, tau, Mo=cap)
    assert rcu == 0
    assert_same_rows(oracle_from_dev(U), Uo, "2X - X^2")
    assert widths[1] == wu


def test_x2_step_dense_rows_wider_than_4096():
    A = random_ell(5000, 0.12, seed=31, symmetric=True)
    check_step(A, 0.02, 5056)


def test_x2_step_scattered_rows_wider_than_4096():
    A = scattered_symmetric(20000, 50, seed=32)
    check_step(A, 1e-4, 12288)


def test_sp2_first_product_wider_than_4096():
    """X0 has about 80 entries per row spread over 15000 columns, so the
    first X^2 has rows of about 5500: the working capacity grows past 4096
    (the solve is cut after that product; its traces, norm and width history
    and X0 itself are compared)."""
    H = scattered_symmetric(15000, 40, seed=33)
    po = oracle.make_params(H.N // 4, 1e-6, 1e-6, max_iter=1)
    o = oracle.sp2(H, po, Mo=H.M + 1)
    assert o[2]["maxw"][0] > 4096
    Hd = dev_from_oracle(H)
    Dd = E.DeviceEll(H.N, H.M + 1)
    rc, rep = E.sp2_solve(Hd.h, Dd.h, E.sp2_params(H.N // 4, 1e-6, 1e-6, max_iter=1))
    assert rc == o[0] == E.ELL_ENOCONV
    for k in ("trx", "trx2", "eta2"):
        assert rep[k][0] == o[2][k][0], k
    assert rep["maxw"][0] == o[2]["maxw"][0]
    assert_same_rows(oracle_from_dev(Dd), o[1], "D")


def test_semiconductor_x2_at_32000_orbitals_sampled_rows():
    N, tau = 32000, 1e-5
    nnz, idx, val, M = synth.model_hamiltonian("semiconductor", N)
    H = oracle.Ell(N, M, nnz, idx, val)
    X = dev_from_oracle(H)
    Yd = E.DeviceEll(N, 4096)
    rc_g, out, w = E.ellpack_x2_threshold(X.h, Yd.h, tau)
    assert rc_g == E.ELL_OK, E.ellpack_strerror(rc_g)
    rows = np.array([0, 1, 2, 1184, 1185, 1186, 9999, 16000, 16001, 23456, N - 1187, N - 2, N - 1])
    rc, nz, ix, vl, dd = oracle.x2_rows(H, tau, rows, M2=4096)
    assert rc == 0
    G = oracle_from_dev(Yd)
    gi = G.idx.reshape(N, G.M)
    gv = G.val.reshape(N, G.M)
    for q, i in enumerate(rows):
        assert G.nnz[i] == nz[q], (i, G.nnz[i], nz[q])
        assert np.array_equal(gi[i, :nz[q]], ix[q, :nz[q]]), i
        assert np.array_equal(gv[i, :nz[q]].view(np.uint64), vl[q, :nz[q]].view(np.uint64)), i
    assert w == int(G.nnz.max())


@pytest.mark.parametrize("N,per_row", [(3001, 200), (1000, 250)])
def test_gershgorin_bounds_of_rows_spanning_several_chunks(N, per_row):
    """Rows of several hundred entries (more than one pass of the bounds
    kernel's staged columns) and a last group of rows cut short by N: the
    solve's reported emin / emax equal the oracle's Gershgorin bounds, bit
    for bit (the solve is cut after one product)."""
    H = scattered_symmetric(N, per_row, seed=34)
    assert int(H.nnz.max()) > 272
    rc, lo, hi = oracle.gershgorin(H)
    assert rc == 0
    Hd = dev_from_oracle(H)
    Dd = E.DeviceEll(H.N, H.M + 1)
    rc, rep = E.sp2_solve(Hd.h, Dd.h, E.sp2_params(H.N // 4, 1e-6, 1e-6, max_iter=1))
    assert rc == E.ELL_ENOCONV, E.ellpack_strerror(rc)
    assert same_float(rep["emin"], lo) and same_float(rep["emax"], hi)
