"""Pins of the oracle's one-pruning SP2 mode (`prune_once`).

Two prunings (the default): X2 = prune(X.X) enters the norm and 2X - X2,
which is pruned again.  One pruning: the unpruned product Y = X.X enters the
norm and 2X - Y, and only the iterate taken is pruned.  The paper fuses its
"SP2 Loop X2", "Norm" and "Misc" steps without saying where the pruning falls
(section "Performance Evaluation using an ExaSP2 Application"), so both are
readings; these tests hold the one-pruning mode to a dense brute-force
evaluation of its definition (exact ascending fma chains), not to the
oracle's own sparse routines.
"""
import numpy as np
import pytest

import oracle
from tests import exact
from tests.test_oracle_pins import banded, brute_x2_exact, eig_projector, random_sparse


def pairwise(d):
    return exact.pairwise_recursive(list(d))


def dense_norm2(Y, X):
    """||Y - X||_F^2: per row the pairwise tree over all N column positions of
    the rounded squares of the double differences, then the tree over rows."""
    N = X.shape[0]
    rows = []
    for i in range(N):
        q = []
        for j in range(N):
            d = float(Y[i, j]) - float(X[i, j])
            q.append(d * d)
        rows.append(pairwise(q))
    return pairwise(rows)


def brute_sp2(Xd, tau, n_occ, steps, once, f32=False):
    """`steps` SP2 iterations from the dense X0, by the definition."""
    dt = np.float32 if f32 else np.float64
    tau = dt(tau)
    hist = []
    for _ in range(steps):
        Yd = brute_x2_exact(Xd, 0.0, f32=f32)  # the unpruned product, exact fma chains
        trx = pairwise(np.diag(Xd).astype(np.float64))
        trx2 = pairwise(np.diag(Yd).astype(np.float64))
        Yp = np.where(np.abs(Yd) > tau, Yd, dt(0))
        Ym = Yd if once else Yp
        eta2 = dense_norm2(Ym, Xd)
        up = abs(2 * trx - trx2 - n_occ) < abs(trx2 - n_occ)
        if up:
            V = (dt(2) * Xd - Ym).astype(dt)  # 2x exact, one rounding
            Xd = np.where(np.abs(V) > tau, V, dt(0)).astype(dt)
        else:
            Xd = Yp
        hist.append((trx, trx2, eta2, int(up)))
    return Xd, hist


def x0_dense(H, tau, f32):
    rc, lo, hi = oracle.gershgorin(H)
    rc, X0, w = oracle.x0(H, lo, hi, tau, fp32=f32)
    assert rc == 0
    return X0.dense().astype(np.float32 if f32 else np.float64)


@pytest.mark.parametrize("f32", [False, True])
def test_prune_once_trajectory_equals_its_definition(f32):
    rng = np.random.default_rng(44 + f32)
    N, n_occ, tau, steps = 12, 4, 0.004, 6
    _, H = random_sparse(N, 0.5, rng, symmetric=True)
    X0 = x0_dense(H, tau, f32)
    prec = oracle.PREC_MIXED if f32 else oracle.PREC_F64
    for once in (1, 0):
        # idem_target 0 never stops, switch_eta 0 never leaves FP32: the solve
        # ends at max_iter and returns X after `steps` updates
        p = oracle.make_params(n_occ, tau, 0.0, max_iter=steps + 1, precision=prec, stall_stop=0,
                               tau_fp32=tau, switch_eta=0.0, prune_once=once)
        rc, D, rep = oracle.sp2(H, p)
        assert rc == oracle.ENOCONV
        Xd, hist = brute_sp2(X0, tau, n_occ, steps, once, f32=f32)
        assert np.array_equal(D.dense(), Xd.astype(np.float64)), once
        for n, (trx, trx2, eta2, up) in enumerate(hist):
            assert rep["trx"][n] == trx and rep["trx2"][n] == trx2, (once, n)
            assert rep["eta2"][n] == eta2, (once, n)
            assert rep["up"][n] == up, (once, n)
        if once:
            D_once, eta_once = D.dense(), rep["eta2"][:steps].copy()
    # the two readings give different iterates and norms on this input
    assert not np.array_equal(D_once, D.dense())
    assert not np.array_equal(eta_once, rep["eta2"][:steps])


def test_prune_once_keeps_the_x2_branch_width_in_the_history():
    # hist_maxw is the widest row of prune(X.X) in both modes
    rng = np.random.default_rng(5)
    N, tau = 14, 0.004
    _, H = random_sparse(N, 0.45, rng, symmetric=True)
    p = oracle.make_params(5, tau, 0.0, max_iter=4, stall_stop=0, prune_once=1)
    rc, D, rep = oracle.sp2(H, p)
    Xd = x0_dense(H, tau, False)
    for n in range(3):
        Yd = brute_x2_exact(Xd, 0.0)
        assert rep["maxw"][n] == int((np.abs(Yd) > tau).sum(axis=1).max()), n
        trx, trx2 = pairwise(np.diag(Xd)), pairwise(np.diag(Yd))
        up = abs(2 * trx - trx2 - 5) < abs(trx2 - 5)
        V = 2 * Xd - Yd if up else Yd
        Xd = np.where(np.abs(V) > tau, V, 0.0)


def test_prune_once_converges_to_the_projector():
    N, b = 160, 5
    H = banded(N, b, seed=4)
    P = eig_projector(H.dense(), N // 4)
    for once in (0, 1):
        p = oracle.make_params(N // 4, 1e-9, 1e-7, max_iter=200, prune_once=once)
        rc, D, rep = oracle.sp2(H, p)
        assert rc == 0, once
        assert np.linalg.norm(D.dense() - P) <= 1e-6, once
        assert abs(rep["trace_x"] - N // 4) <= 1e-7


def test_prune_matches_selection():
    rng = np.random.default_rng(9)
    for dt in (np.float64, np.float32):
        D, A = random_sparse(40, 0.3, rng, dtype=dt)
        for tau in (0.0, 0.3, 2.0):
            rc, P, w = oracle.prune(A, tau)
            assert rc == 0
            keep = np.abs(D) > dt(tau)
            assert w == (keep.sum(axis=1).max() if keep.any() else 0)
            for i, (c, v) in enumerate(P.rows()):
                assert np.array_equal(c, np.nonzero(keep[i])[0])
                assert np.array_equal(v, D[i, keep[i]])
        rc, P, w = oracle.prune(A, 0.3, Mo=1)
        assert rc == oracle.EOVERFLOW and w == (np.abs(D) > dt(0.3)).sum(axis=1).max()
