"""Pins of the CPU oracle against things other than itself.

Each test ties one oracle function to exact rational arithmetic, a brute-force
dense computation, a closed form, a library routine or an invariant, so that a
dropped term, a wrong sign, a transposed operand or a wrong summation order in
the oracle fails here.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle
from paper_2102_08505_amd import synth
from tests import exact

RNG = np.random.default_rng(12345)


def random_sparse(N, density, rng, symmetric=False, dtype=np.float64, extra=None, M=None):
    """Random sparse matrix with assorted row shapes (empty, full, diagonal-only, single entry)."""
    D = rng.uniform(-1, 1, size=(N, N)) * (rng.random((N, N)) < density)
    if symmetric:
        D = np.triu(D) + np.triu(D, 1).T
    if extra:
        for kind, i in extra:
            if kind == "empty":
                D[i, :] = 0
                if symmetric:
                    D[:, i] = 0
            elif kind == "full":
                D[i, :] = rng.uniform(-1, 1, N)
                if symmetric:
                    D[:, i] = D[i, :]
            elif kind == "diag":
                D[i, :] = 0
                if symmetric:
                    D[:, i] = 0
                D[i, i] = rng.uniform(0.5, 1)
            elif kind == "single":
                D[i, :] = 0
                D[i, rng.integers(N)] = rng.uniform(-1, 1)
    D = D.astype(dtype)
    nnz, idx, val, Mx = synth.dense_to_ell(D, M=M, dtype=dtype)
    return D, oracle.Ell(N, Mx, nnz, idx, val)


# --------------------------------------------------------------------------- pairwise
def test_pairwise_matches_recursive_definition():
    for n in list(range(1, 40)) + [63, 64, 65, 127, 128, 129, 1000, 1023, 1025]:
        d = RNG.standard_normal(n) * np.exp2(RNG.integers(-30, 30, n))
        assert oracle.pairwise(d) == exact.pairwise_recursive(d)


def test_pairwise_is_a_tree_not_a_running_sum():
    d = [1.0, 2.0 ** -53, 2.0 ** -53, 0.0]
    # tree: (1 + 2^-53 -> 1, ties to even) + (2^-53 + 0) = 1 + 2^-53 -> 1
    assert oracle.pairwise(d) == 1.0
    d = [2.0 ** -53, 2.0 ** -53, 1.0, 0.0]
    # tree: (2^-53 + 2^-53) + (1 + 0) = 1 + 2^-52 exactly
    assert oracle.pairwise(d) == 1.0 + 2.0 ** -52
    d = [1.0, 0.0, 2.0 ** -53, 2.0 ** -53]
    # running sum: 1 + 0 + 2^-53 -> 1, + 2^-53 -> 1; tree: 1 + 2^-52
    assert oracle.pairwise(d) == 1.0 + 2.0 ** -52
    assert math.fsum(d) == 1.0 + 2.0 ** -52
    assert oracle.pairwise([]) == 0.0


# --------------------------------------------------------------------------- X^2
def brute_x2_exact(D, tau, f32=False):
    """Dense triple loop, k ascending over all of 0..N-1, correctly rounded fma."""
    N = D.shape[0]
    out = np.zeros((N, N), dtype=np.float32 if f32 else np.float64)
    for i in range(N):
        for j in range(N):
            acc = np.float32(0) if f32 else 0.0
            for k in range(N):
                a, b = D[i, k], D[k, j]
                if a == 0 or b == 0:
                    continue  # a zero product leaves a nonzero accumulator unchanged
                acc = exact.fma32(a, b, acc) if f32 else exact.fma64(a, b, acc)
            out[i, j] = acc
    return out


@pytest.mark.parametrize("sym", [False, True])
@pytest.mark.parametrize("f32", [False, True])
def test_x2_bit_exact_against_dense_brute_force(sym, f32):
    rng = np.random.default_rng(7 + sym + 2 * f32)
    N = 14
    extra = [("empty", 0), ("full", 3), ("diag", 5), ("single", 9)]
    dt = np.float32 if f32 else np.float64
    D, A = random_sparse(N, 0.35, rng, symmetric=sym, dtype=dt, extra=extra)
    tau = 0.05
    ref = brute_x2_exact(D.astype(np.float64) if not f32 else D, 0.0, f32=f32)
    rc, X2, d1, d2, w = oracle.x2(A, tau)
    assert rc == 0
    keep = np.abs(ref) > tau
    assert w == keep.sum(axis=1).max()
    for i, (c, v) in enumerate(X2.rows()):
        exp_c = np.nonzero(keep[i])[0]
        assert np.array_equal(c, exp_c), i
        assert np.array_equal(v, ref[i, exp_c]), i          # bit-exact values
    assert np.array_equal(d2, ref.diagonal().astype(np.float64))  # unpruned diagonal
    assert np.array_equal(d1, np.diag(D).astype(np.float64))


@pytest.mark.parametrize("f32", [False, True])
def test_row_loops_do_not_depend_on_thread_count(f32):
    """X^2 and the update share their rows out over OpenMP threads; every
    output (rows, traces, widths, status -- overflow included) is the same
    bits on one thread and on several."""
    rng = np.random.default_rng(31 + f32)
    dt = np.float32 if f32 else np.float64
    D, A = random_sparse(301, 0.04, rng, symmetric=True, dtype=dt, extra=[("full", 17), ("empty", 3)])
    before = oracle.threads()
    try:
        runs = []
        for th in (1, 5):
            oracle.threads(th)
            assert oracle.threads() == th
            out = []
            for M2 in (None, 40):  # 40: row 17 overflows
                rc, Y, d1, d2, w = oracle.x2(A, 0.01, M2=M2)
                rcu, Z, wu = oracle.update(A, Y, 0.01, Mo=M2)
                out.append((rc, Y, d1, d2, w, rcu, Z, wu))
            runs.append(out)
    finally:
        oracle.threads(before)
    assert runs[0][1][0] == oracle.EOVERFLOW and runs[0][1][5] == oracle.EOVERFLOW
    for (a, b) in zip(*runs):
        assert a[0] == b[0] and a[4] == b[4] and a[5] == b[5] and a[7] == b[7]
        for Ea, Eb in ((a[1], b[1]), (a[6], b[6])):
            assert np.array_equal(Ea.nnz, Eb.nnz) and np.array_equal(Ea.idx, Eb.idx)
            assert np.array_equal(Ea.val.view(np.uint8), Eb.val.view(np.uint8))
        assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])


def test_stream_triad_reports_a_bandwidth():
    assert oracle.stream_triad(1 << 20, 2) > 0


def test_x2_tau_zero_keeps_every_nonzero_and_drops_exact_zeros():
    # X with an exact cancellation: row 0 = [1, 1], row 1 = [1, -1] -> (X^2)[0,1] = 1 - 1 = 0
    D = np.array([[1.0, 1.0], [1.0, -1.0]])
    nnz, idx, val, M = synth.dense_to_ell(D)
    rc, X2, *_ = oracle.x2(oracle.Ell(2, M, nnz, idx, val), 0.0)
    rows = X2.rows()
    assert list(rows[0][0]) == [0] and rows[0][1][0] == 2.0
    assert list(rows[1][0]) == [1] and rows[1][1][0] == 2.0


def test_x2_threshold_edges_are_strict():
    tau = 1e-5
    vals = [tau, np.nextafter(tau, np.inf), np.nextafter(tau, 0), -tau, -np.nextafter(tau, np.inf),
            -np.nextafter(tau, 0), 0.5, 1e-300]
    n = len(vals)
    N = n + 2
    D = np.zeros((N, N))
    D[0, 1] = 1.0                      # row 0 of X^2 = 1 * row 1 of X, exactly
    D[1, 2:] = vals
    nnz, idx, val, M = synth.dense_to_ell(D)
    rc, X2, *_ = oracle.x2(oracle.Ell(N, M, nnz, idx, val), tau)
    c, v = X2.rows()[0]
    expect = [2 + q for q, x in enumerate(vals) if abs(x) > tau]
    assert list(c) == expect
    assert list(v) == [vals[q - 2] for q in expect]


def test_x2_of_symmetric_is_bitwise_symmetric():
    rng = np.random.default_rng(3)
    D, A = random_sparse(60, 0.15, rng, symmetric=True)
    rc, X2, *_ = oracle.x2(A, 1e-3)
    Y = X2.dense()
    assert np.array_equal(Y, Y.T)


def test_x2_overflow_reports_required_width():
    rng = np.random.default_rng(4)
    D, A = random_sparse(30, 0.3, rng)
    rc, X2full, _, _, w = oracle.x2(A, 0.0)
    rc2, _, _, _, w2 = oracle.x2(A, 0.0, M2=w - 1)
    assert rc2 == oracle.EOVERFLOW and w2 == w
    rc3, X2, _, _, w3 = oracle.x2(A, 0.0, M2=w)
    assert rc3 == 0 and w3 == w


def test_x2_against_numpy_matmul_on_banded_input():
    nnz, idx, val, M = synth.banded_hamiltonian(300, 9)
    H = oracle.Ell(300, M, nnz, idx, val)
    rc, X2, d1, d2, w = oracle.x2(H, 0.0)
    Hd = H.dense()
    ref = Hd @ Hd
    got = X2.dense()
    bound = 300 * 2.0 ** -53 * (np.abs(Hd) @ np.abs(Hd))
    assert np.all(np.abs(got - ref) <= bound + 1e-300)
    assert np.count_nonzero(got) == np.count_nonzero(ref)
    assert oracle.fma_count(H) == int(sum(nnz[idx.reshape(300, M)[i, :nnz[i]]].sum() for i in range(300)))


# --------------------------------------------------------------------------- traces, norm
def test_trace_and_norm_closed_form_on_diagonal():
    x = np.array([0.5, 0.25, 0.75, 1.0, 0.0, 0.125])
    N = x.size
    D = np.diag(x)
    nnz, idx, val, M = synth.dense_to_ell(D)
    A = oracle.Ell(N, M, nnz, idx, val)
    assert oracle.trace(A) == x.sum()
    rc, X2, d1, d2, w = oracle.x2(A, 0.0)
    assert np.array_equal(d2, x * x)
    eta2, e = oracle.norm2(A, X2)
    # (x^2 - x)^2 with dyadic x is exact
    assert np.array_equal(e, (x * x - x) ** 2)
    assert eta2 == ((x * x - x) ** 2).sum()


def test_norm_against_numpy_on_union_pattern():
    rng = np.random.default_rng(5)
    Dx, X = random_sparse(50, 0.2, rng)
    Dy, Y = random_sparse(50, 0.2, rng)
    eta2, e = oracle.norm2(X, Y)
    ref_rows = ((Dy - Dx) ** 2).sum(axis=1)
    assert np.allclose(e, ref_rows, rtol=1e-14, atol=0)
    assert abs(eta2 - np.linalg.norm(Dy - Dx) ** 2) <= 1e-13 * eta2
    assert eta2 == exact.pairwise_recursive(e)


def test_norm_f32_differences_in_double():
    # 0.3f - 1.0000001f and its square are exact in double (two binary32 values
    # differ by a 25-bit number) but not in float, so this separates a norm
    # formed in double from one formed in float: float gives 0.49000016.
    x = np.float32(1.0000001)
    y = np.float32(0.3)
    X = oracle.Ell(1, 1, [1], [0], np.array([x], np.float32))
    Y = oracle.Ell(1, 1, [1], [0], np.array([y], np.float32))
    eta2, e = oracle.norm2(X, Y)
    d = Fraction(float(y)) - Fraction(float(x))
    assert eta2 == float(d * d)                       # one rounding, of the exact square
    df = np.float32(y) - np.float32(x)
    assert eta2 != float(np.float32(df * df))          # what float arithmetic would give
    # a row of several such terms: each square rounded to double, then the tree
    xs = np.array([1.0000001, 0.7, -0.3000001, 2.5], np.float32)
    ys = np.array([0.3, 0.1, 0.9, 1.0000001], np.float32)
    pad = np.zeros(12, np.float32)
    X = oracle.Ell(4, 4, [4, 0, 0, 0], [0, 1, 2, 3] + [0] * 12, np.concatenate([xs, pad]))
    Y = oracle.Ell(4, 4, [4, 0, 0, 0], [0, 1, 2, 3] + [0] * 12, np.concatenate([ys, pad]))
    eta2, e = oracle.norm2(X, Y)
    q = [float((Fraction(float(b)) - Fraction(float(a))) ** 2) for a, b in zip(xs, ys)]
    assert eta2 == (q[0] + q[1]) + (q[2] + q[3])


# --------------------------------------------------------------------------- update
def test_update_exact_dyadic_and_threshold():
    tau = 0.1
    X = np.array([[0.5, 0.0, 0.25, 0.0], [0.0, 0.05, 0.0, 0.0], [0.25, 0.0, 0.0, 0.5], [0, 0, 0.5, 1.0]])
    Y = np.array([[0.75, 0.2, 0.5, 0.0], [0.0, 0.0, 0.0, -0.125], [0.5, 0.0, 0.0, 0.0], [0, 0, 0.5, 1.0]])
    nx = synth.dense_to_ell(X)
    ny = synth.dense_to_ell(Y)
    EX = oracle.Ell(4, nx[3], nx[0], nx[1], nx[2])
    EY = oracle.Ell(4, ny[3], ny[0], ny[1], ny[2])
    rc, Z, w = oracle.update(EX, EY, tau)
    ref = 2 * X - Y                     # exact on these dyadic values
    keep = np.abs(ref) > tau
    for i, (c, v) in enumerate(Z.rows()):
        assert list(c) == list(np.nonzero(keep[i])[0])
        assert np.array_equal(v, ref[i, keep[i]])
    # (1, 1): 2*0.05 - 0 = 0.1 is not > tau; (0, 2): 2*0.25 - 0.5 = 0 dropped
    assert 1 not in Z.rows()[1][0]
    assert 2 not in Z.rows()[0][0]


def test_update_single_rounding():
    # 2x - y rounded once: x = 1 + 2^-52, y = 2^-52 * 3 -> 2 + 2^-51 - 3*2^-52 = 2 - 2^-52 -> rounds to even
    x = 1.0 + 2.0 ** -52
    y = 3 * 2.0 ** -52
    X = oracle.Ell(1, 1, [1], [0], [x])
    Y = oracle.Ell(1, 1, [1], [0], [y])
    rc, Z, w = oracle.update(X, Y, 0.0)
    assert Z.rows()[0][1][0] == exact.fma64(2.0, x, -y)


def test_update_f32_rounds_and_thresholds_in_float():
    # FP32 mode: 2x - y is one binary32 rounding of the exact value, and the
    # threshold compares that float with the float tau.
    rng = np.random.default_rng(31)
    N = 24
    xs = (rng.uniform(-1, 1, N) * 2.0 ** rng.integers(-12, 2, N)).astype(np.float32)
    ys = (rng.uniform(-1, 1, N) * 2.0 ** rng.integers(-40, 2, N)).astype(np.float32)
    # row 0: 2 * 0.5 - (-2^-30) = 1 + 2^-30 exactly; binary32 rounds it to 1.0,
    # which is not > tau = 1.0 (in double it would be kept)
    xs[0], ys[0] = np.float32(0.5), np.float32(-(2.0 ** -30))
    # row 1: 2 * 1.0000001f - 2^-40 rounds back to 2 * 1.0000001f in float
    xs[1], ys[1] = np.float32(1.0000001), np.float32(2.0 ** -40)
    tau = np.float32(1.0)
    X = oracle.Ell(N, 1, [1] * N, list(range(N)), xs)
    Y = oracle.Ell(N, 1, [1] * N, list(range(N)), ys)
    rc, Z, w = oracle.update(X, Y, 0.0)
    assert Z.val.dtype == np.float32
    for i, (c, v) in enumerate(Z.rows()):
        ref = exact.to_f32(2 * Fraction(float(xs[i])) - Fraction(float(ys[i])))
        assert list(c) == ([i] if ref != 0 else [])
        if ref != 0:
            assert v[0].view(np.uint32) == np.float32(ref).view(np.uint32)
    assert Z.rows()[1][1][0] == np.float32(2) * xs[1]
    rc, Z, w = oracle.update(X, Y, float(tau))
    assert 0 not in Z.rows()[0][0]                      # 1 + 2^-30 -> 1.0f, not kept
    assert list(Z.rows()[1][0]) == [1]                  # 2.0000002f > 1


# --------------------------------------------------------------------------- Gershgorin, X0
def test_gershgorin_brute_force_dyadic():
    rng = np.random.default_rng(8)
    N = 40
    D = np.round(rng.uniform(-4, 4, (N, N)) * 64) / 64 * (rng.random((N, N)) < 0.2)
    D = np.triu(D) + np.triu(D, 1).T
    nnz, idx, val, M = synth.dense_to_ell(D)
    rc, lo, hi = oracle.gershgorin(oracle.Ell(N, M, nnz, idx, val))
    r = np.abs(D).sum(axis=1) - np.abs(np.diag(D))      # exact on 1/64-grid values
    assert lo == (np.diag(D) - r).min() and hi == (np.diag(D) + r).max()


def test_x0_uniform_chain_closed_form():
    N, t = 12, 1.0
    D = np.zeros((N, N))
    for i in range(N - 1):
        D[i, i + 1] = D[i + 1, i] = -t
    nnz, idx, val, M = synth.dense_to_ell(D)
    H = oracle.Ell(N, M, nnz, idx, val)
    rc, lo, hi = oracle.gershgorin(H)
    assert (lo, hi) == (-2 * t, 2 * t)
    rc, X0, w = oracle.x0(H, lo, hi, 0.0)
    ref = (2 * t * np.eye(N) - D) / (4 * t)
    assert np.array_equal(X0.dense(), ref)
    # threshold above 0.25 removes the couplings, keeps the diagonal 0.5
    rc, X0b, w = oracle.x0(H, lo, hi, 0.3)
    assert np.array_equal(X0b.dense(), 0.5 * np.eye(N))


def test_x0_inserts_missing_diagonal_and_f32_rounds_once():
    D = np.array([[0.0, 1.0, 0.0], [1.0, 0.0, 0.5], [0.0, 0.5, 2.0]])
    nnz, idx, val, M = synth.dense_to_ell(D)
    H = oracle.Ell(3, M, nnz, idx, val)
    rc, lo, hi = oracle.gershgorin(H)
    rc, X0, w = oracle.x0(H, lo, hi, 0.0)
    inv = 1.0 / (hi - lo)
    ref = np.array([[hi * inv, -1 * inv, 0], [-1 * inv, hi * inv, -0.5 * inv], [0, -0.5 * inv, (hi - 2.0) * inv]])
    assert np.array_equal(X0.dense(), ref)
    rc, X0f, w = oracle.x0(H, lo, hi, 0.0, fp32=True)
    for i, (c, v) in enumerate(X0f.rows()):
        assert np.array_equal(v, ref[i, c].astype(np.float32))


# --------------------------------------------------------------------------- SP2
def eig_projector(Hd, n_occ):
    w, V = np.linalg.eigh(Hd)
    assert w[n_occ] - w[n_occ - 1] > 1e-6, "test input must have a gap at the Fermi level"
    return V[:, :n_occ] @ V[:, :n_occ].T


def banded(N, b, seed=0):
    nnz, idx, val, M = synth.banded_hamiltonian(N, b, seed=seed)
    return oracle.Ell(N, M, nnz, idx, val)


def test_sp2_tau0_matches_eigendecomposition_projector():
    N, b = 96, 4
    H = banded(N, b, seed=1)
    P = eig_projector(H.dense(), N // 4)
    p = oracle.make_params(N // 4, 0.0, 1e-10, max_iter=200)
    rc, D, rep = oracle.sp2(H, p)
    assert rc == 0
    assert np.linalg.norm(D.dense() - P) <= 1e-9
    assert abs(rep["trace_x"] - N // 4) <= 1e-9


def test_sp2_tight_binding_chain_closed_form():
    N, t, n_occ = 40, 1.0, 13
    D = np.zeros((N, N))
    for i in range(N - 1):
        D[i, i + 1] = D[i + 1, i] = -t
    nnz, idx, val, M = synth.dense_to_ell(D)
    H = oracle.Ell(N, M, nnz, idx, val)
    # e_m = -2t cos(m pi/(N+1)), phi_m(i) = sqrt(2/(N+1)) sin(m i pi/(N+1)), m, i = 1..N
    i = np.arange(1, N + 1)
    phi = np.array([np.sqrt(2.0 / (N + 1)) * np.sin(m * i * np.pi / (N + 1)) for m in range(1, n_occ + 1)])
    P = phi.T @ phi
    p = oracle.make_params(n_occ, 0.0, 1e-11, max_iter=300)
    rc, Dm, rep = oracle.sp2(H, p)
    assert rc == 0
    assert np.linalg.norm(Dm.dense() - P) <= 1e-9


def test_sp2_diagonal_hamiltonian_becomes_exact_projector():
    h = np.array([0.3, -1.2, 2.5, 0.1, -0.7, 1.9, -2.2, 0.8])
    N = h.size
    nnz, idx, val, M = synth.dense_to_ell(np.diag(h))
    H = oracle.Ell(N, M, nnz, idx, val)
    n_occ = 3
    p = oracle.make_params(n_occ, 0.0, 0.0, max_iter=400, stall_stop=0)
    rc, D, rep = oracle.sp2(H, p)
    assert rc == oracle.ENOCONV  # the target 0 is never met strictly
    expect = np.zeros((N, N))
    for q in np.argsort(h)[:n_occ]:
        expect[q, q] = 1.0
    assert np.array_equal(D.dense(), expect)


def test_sp2_invariants_along_the_trajectory():
    N, b = 64, 3
    H = banded(N, b, seed=2)
    n_occ = 16
    eta = []
    for n in range(1, 60):
        p = oracle.make_params(n_occ, 0.0, 1e-12, max_iter=n, stall_stop=0)
        rc, D, rep = oracle.sp2(H, p)
        Xd = D.dense()
        ev = np.linalg.eigvalsh(Xd)
        assert ev.min() >= -1e-12 and ev.max() <= 1 + 1e-12, n
        assert np.array_equal(Xd, Xd.T)
        eta.append(rep["eta"])
        if rc == 0:
            break
    assert rc == 0
    assert abs(np.trace(Xd) - n_occ) < 1e-10
    # quadratic regime: the best of each pair of steps decreases
    pairs = [min(eta[q], eta[q + 1]) for q in range(len(eta) - 1)]
    tail = [v for v in pairs if v < 1e-2]
    assert all(tail[q + 2] < tail[q] for q in range(len(tail) - 2))


def test_sp2_branch_rule_and_history():
    H = banded(128, 6, seed=3)
    p = oracle.make_params(32, 1e-7, 1e-6, max_iter=200)
    rc, D, rep = oracle.sp2(H, p)
    n = rep["iterations"]
    for q in range(n - 1):
        up = abs(2 * rep["trx"][q] - rep["trx2"][q] - 32) < abs(rep["trx2"][q] - 32)
        assert rep["up"][q] == int(up)
    assert rep["up"][n - 1] == -1
    # traces are recomputed from the stored X: Tr X_{n+1} = Tr X_n^2 (pre-prune) when X <- X^2 and tau is tiny
    for q in range(n - 1):
        if rep["up"][q] == 0:
            assert abs(rep["trx"][q + 1] - rep["trx2"][q]) < 1e-9


def test_sp2_drop_tolerance_floor_and_stall_rule():
    N, b = 512, 16
    H = banded(N, b)
    p = oracle.make_params(N // 4, 1e-5, 1e-8, max_iter=100)
    rc, D, rep = oracle.sp2(H, p)
    assert rc == oracle.ENOCONV
    assert rep["iterations"] < 100          # the stall rule stopped it
    assert 1e-6 < rep["eta"] < 1e-2         # floor set by the tolerance
    ev = np.linalg.eigvalsh(D.dense())
    assert ev.min() > -1e-3 and ev.max() < 1 + 1e-3


def test_sp2_errors():
    H = banded(32, 2)
    p = oracle.make_params(0, 0.0, 1e-8)
    assert oracle.sp2(H, p)[0] == oracle.EDEGENERATE
    p = oracle.make_params(32, 0.0, 1e-8)
    assert oracle.sp2(H, p)[0] == oracle.EDEGENERATE
    I = oracle.Ell(4, 1, [1, 1, 1, 1], [0, 1, 2, 3], [2.0] * 4)
    assert oracle.sp2(I, oracle.make_params(2, 0.0, 1e-8))[0] == oracle.EDEGENERATE
    bad = oracle.Ell(3, 2, [2, 1, 1], [1, 0, 1, -1, 2, -1], [1.0, 1.0, 1, 0, 1, 0])
    assert oracle.sp2(bad, oracle.make_params(1, 0.0, 1e-8))[0] == oracle.EINVAL
    nan = oracle.Ell(2, 1, [1, 1], [0, 1], [np.nan, 1.0])
    assert oracle.sp2(nan, oracle.make_params(1, 0.0, 1e-8))[0] == oracle.ENONFINITE


def test_sp2_mixed_precision_accuracy_and_fp64_tail():
    N, b = 128, 4
    H = banded(N, b, seed=4)
    n_occ = N // 4
    P = eig_projector(H.dense(), n_occ)
    p = oracle.make_params(n_occ, 0.0, 1e-9, max_iter=200, precision=oracle.PREC_MIXED,
                           tau_fp32=0.0, switch_eta=1e-4)
    rc, D, rep = oracle.sp2(H, p)
    assert rc == 0
    prec = rep["prec"]
    assert prec[0] == 1 and prec[-1] == 0
    k = int(np.argmin(prec))                          # first FP64 product
    assert np.all(prec[:k] == 1) and np.all(prec[k:] == 0)
    assert len(prec) - k >= 3                          # >= 2 FP64 updates before the stop
    err = np.linalg.norm(D.dense() - P)
    assert err < 1e-4                                  # FP32-phase accuracy, restored idempotency
    assert rep["eta"] < 1e-9


def test_sp2_f32_x2_matches_brute_force_fmaf():
    rng = np.random.default_rng(11)
    D, A = random_sparse(12, 0.4, rng, symmetric=True, dtype=np.float32)
    ref = brute_x2_exact(D, 0.0, f32=True)
    rc, X2, d1, d2, w = oracle.x2(A, np.float32(1e-3))
    keep = np.abs(ref) > np.float32(1e-3)
    for i, (c, v) in enumerate(X2.rows()):
        assert list(c) == list(np.nonzero(keep[i])[0])
        assert np.array_equal(v, ref[i, keep[i]])


# --------------------------------------------------------------------------- dense variant
def test_bf16_rne_against_exact_and_torch():
    xs = np.concatenate([RNG.standard_normal(2000).astype(np.float32),
                         np.array([1.00390625, 1.01171875, -1.00390625, 3.0e-39, 65504.0], np.float32)])
    tt = torch.from_numpy(xs).to(torch.bfloat16).to(torch.float32).numpy()
    for x, t in zip(xs, tt):
        b = oracle.bf16_rne(x)
        assert b == exact.bf16(x) == t


def test_dense_x2_f64_matches_sparse_x2_and_exact_bound():
    N = 40
    Hd = synth.dense_hamiltonian(N, 5, seed=3)
    Cd = oracle.dense_x2_f64(Hd)
    nnz, idx, val, M = synth.dense_to_ell(Hd)
    rc, X2, *_ = oracle.x2(oracle.Ell(N, M, nnz, idx, val), 0.0)
    assert np.array_equal(Cd, X2.dense())
    assert np.all(np.abs(Cd - Hd @ Hd) <= N * 2.0 ** -53 * (np.abs(Hd) @ np.abs(Hd)))


def test_dense_bf16x3_error_bound():
    N = 48
    A = (synth.dense_hamiltonian(N, 8, seed=5) / 4).astype(np.float32)
    Cm = oracle.dense_x2_bf16x3(A).astype(np.float64)
    A64 = A.astype(np.float64)
    exact_prod = A64 @ A64              # error of this fp64 product is far below the bound
    bound = (2.0 ** -16 + N * 2.0 ** -24) * (np.abs(A64) @ np.abs(A64))
    assert np.all(np.abs(Cm - exact_prod) <= bound)
    # and the split is really more accurate than a single bf16 product
    hi = torch.from_numpy(A).to(torch.bfloat16).to(torch.float64).numpy()
    one = hi @ hi
    assert np.abs(Cm - exact_prod).max() < 0.1 * np.abs(one - exact_prod).max()


@pytest.mark.parametrize("mode", [oracle.DENSE_F64, oracle.DENSE_BF16X3])
def test_dense_sp2_against_projector(mode):
    N = 64
    Hd = synth.dense_hamiltonian(N, 4, seed=6)
    n_occ = 16
    P = eig_projector(Hd, n_occ)
    p = oracle.make_params(n_occ, 0.0, 1e-9, max_iter=200, switch_eta=1e-3)
    rc, D, rep = oracle.dense_sp2(Hd, mode, p)
    assert rc == 0
    tol = 1e-9 if mode == oracle.DENSE_F64 else 5e-3
    assert np.linalg.norm(D - P) <= tol
    assert rep["eta"] < 1e-9
    if mode == oracle.DENSE_BF16X3:
        assert rep["fp32_iterations"] > 0 and rep["prec"][-1] == 0


def test_norm_row_term_is_a_pairwise_tree():
    # d = [1, 0, 3*2^-28, 3*2^-28] at columns 0..3 -> squares [1, 0, 9*2^-56, 9*2^-56].
    # A running sum gives 1 + 2^-51; the pairwise tree (1 + 0) + (9*2^-56 + 9*2^-56)
    # = 1 + 1.125*2^-52 rounds to 1 + 2^-52.
    s = 3 * 2.0 ** -28
    Y = oracle.Ell(4, 4, [4, 0, 0, 0], [0, 1, 2, 3] + [-1] * 12, [1.0, 0.5, s, s] + [0.0] * 12)
    X = oracle.Ell(4, 1, [1, 0, 0, 0], [1, -1, -1, -1], [0.5, 0, 0, 0])
    eta2, e = oracle.norm2(X, Y)
    assert e[0] == 1.0 + 2.0 ** -52
    run = 0.0
    for d in (1.0, 0.0, s, s):
        run = run + d * d
    assert run == 1.0 + 2.0 ** -51


def test_norm_tree_runs_over_column_positions():
    # Stored columns 0, 2, 3 of a 4-column row (column 1 empty in both), squares
    # q = [1, -, 9*2^-56, 9*2^-56].  Over column positions the tree is
    # (1 + 0) + (q2 + q3) = 1 + 2^-52; a tree over the list of stored entries
    # would pair (1 + q2) + q3 = 1 + 2^-51.
    s = 3 * 2.0 ** -28
    Y = oracle.Ell(4, 4, [3, 0, 0, 0], [0, 2, 3, -1] + [-1] * 12, [1.0, s, s, 0.0] + [0.0] * 12)
    X = oracle.Ell(4, 1, [0, 0, 0, 0], [-1] * 4, [0.0] * 4)
    eta2, e = oracle.norm2(X, Y)
    assert e[0] == 1.0 + 2.0 ** -52
    listed = (1.0 + s * s) + s * s
    assert listed == 1.0 + 2.0 ** -51
    # and the same value as the dense row summed by the pairwise definition
    assert e[0] == exact.pairwise_recursive([1.0, 0.0, s * s, s * s])


def test_norm_equals_pairwise_over_dense_rows():
    rng = np.random.default_rng(21)
    for N in (5, 37, 64, 100):
        Dx, X = random_sparse(N, 0.2, rng)
        Dy, Y = random_sparse(N, 0.2, rng)
        eta2, e = oracle.norm2(X, Y)
        for i in range(N):
            assert e[i] == exact.pairwise_recursive((Dy[i] - Dx[i]) ** 2), (N, i)


# ---- Tr(AB) --------------------------------------------------------------------------

def _trace_product_exact(DA, DB):
    """Per row i, the exact-arithmetic fma chain over ascending j of A_ij B_ji
    (only where both are nonzero), each step rounded once; then the pairwise
    tree of the row terms by its recursive definition."""
    N = DA.shape[0]
    t = []
    for i in range(N):
        acc = 0.0
        for j in range(N):
            if DA[i, j] != 0 and DB[j, i] != 0:
                acc = exact.fma64(DA[i, j], DB[j, i], acc)
        t.append(acc)
    return exact.pairwise_recursive(t)


@pytest.mark.parametrize("f32", [False, True])
def test_trace_product_bit_exact_against_brute_force(f32):
    rng = np.random.default_rng(31 + f32)
    dt = np.float32 if f32 else np.float64
    DA, A = random_sparse(13, 0.4, rng, dtype=dt, extra=[("empty", 2), ("full", 4)])
    DB, B = random_sparse(13, 0.4, rng, dtype=dt, extra=[("single", 7), ("diag", 1)])
    got = oracle.trace_product(A, B)
    ref = _trace_product_exact(DA.astype(np.float64), DB.astype(np.float64))
    assert got == ref
    # Tr(AB) = Tr(BA) in exact arithmetic; numpy's product agrees to rounding
    assert abs(got - np.trace(DA.astype(np.float64) @ DB.astype(np.float64))) <= 1e-12 * np.abs(DA).sum() * np.abs(DB).max()
    assert abs(got - oracle.trace_product(B, A)) <= 1e-12 * np.abs(DA).sum() * np.abs(DB).max()


def test_trace_product_of_x_with_itself_is_the_unpruned_trace_of_x2():
    """Tr(XX) runs the chain of the diagonal of X^2: the same bits as the trace
    of the unpruned diagonal that the product reports."""
    nnz, idx, val, M = synth.banded_hamiltonian(200, 6, seed=11)
    X = oracle.Ell(200, M, nnz, idx, val)
    rc, _, _, d2, _ = oracle.x2(X, 1e-3)
    assert rc == 0
    assert oracle.trace_product(X, X) == oracle.pairwise(d2)


def test_trace_product_diagonal_closed_form():
    a = np.array([0.5, -0.25, 2.0, 0.0, 1.5])
    b = np.array([4.0, 8.0, -0.5, 3.0, 0.0])
    A = oracle.Ell(5, 1, (a != 0).astype(np.int32), np.where(a != 0, np.arange(5), -1).astype(np.int32), a.copy())
    B = oracle.Ell(5, 1, (b != 0).astype(np.int32), np.where(b != 0, np.arange(5), -1).astype(np.int32), b.copy())
    assert oracle.trace_product(A, B) == float((a * b).sum())  # dyadic: every sum is exact


def test_x2_rows_equal_the_rows_of_the_whole_product():
    """The sampled-row product (for checking products too large to form
    whole) gives exactly the rows, widths and unpruned diagonal of x2."""
    rng = np.random.default_rng(21)
    D, A = random_sparse(230, 0.08, rng, extra=[("full", 40), ("empty", 7)])
    rc, Y, d1, d2, w = oracle.x2(A, 0.05)
    assert rc == 0
    rows = np.array([0, 7, 40, 41, 117, 229])
    rc, nz, ix, vl, dd = oracle.x2_rows(A, 0.05, rows, M2=Y.M)
    assert rc == 0
    for q, i in enumerate(rows):
        c, v = Y.rows()[i]
        assert nz[q] == len(c)
        assert np.array_equal(ix[q, :nz[q]], c) and np.array_equal(vl[q, :nz[q]], v)
        assert dd[q] == d2[i]
    rc, nz, ix, vl, dd = oracle.x2_rows(A, 0.05, rows, M2=3)
    assert rc == oracle.EOVERFLOW
    rc, *_ = oracle.x2_rows(A, 0.05, np.array([230]), M2=4)
    assert rc == oracle.EINVAL
