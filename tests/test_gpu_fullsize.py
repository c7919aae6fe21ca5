"""Full-size parity of the benchmark's SP2 solves, by induction over steps.

A whole SP2 trajectory at N = 32768 or 131072 is too long for the oracle, so
each test cuts the GPU solve at k and at k + 1 products (max_iter = k and
k + 1: the solve returns the matrix whose product was its last, X_{k-1} and
X_k) and applies one oracle step to the GPU's X_{k-1}: X^2 with its traces,
the norm, the branch, and 2X - X^2.  The GPU's X_k and the history entries of
product k - 1 (Tr X, Tr X^2, eta^2, branch) must equal it bit for bit, and the
entries of product k must equal the oracle's traces and norm of X_k.  With X0
checked against the oracle elsewhere, every step being exact makes the whole
trajectory exact.

Workloads: the banded generator (H_ij = exp(-0.5|i-j|) U(-1, 1) for
0 < |i-j| <= 64, H_ii ~ N(0, 1), seed 0), N_occ = N/4, target 1e-6:
  * N = 32768, FP64, tau = 1e-8 (the benchmark's headline solve);
  * N = 131072, FP64, tau = 1e-9;
  * N = 131072, mixed: FP32 phase at tau 1e-7 switching at eta < 1e-2, FP64
    steps at tau 1e-9 -- cut inside the FP32 phase and at the first FP64 step.
"""
import numpy as np
import pytest

import oracle
from paper_2102_08505_amd import ellsp2 as E
from paper_2102_08505_amd import synth
from tests.gpu_helpers import assert_same_rows, oracle_from_dev, same_float

pytestmark = pytest.mark.gpu

WIDTH = 512  # oracle output capacity (the iterates here stay below 300 entries per row)


def _as_f32(A):
    v = A.val.astype(np.float32)
    assert np.array_equal(v.astype(np.float64), A.val)  # a widened FP32 iterate
    return oracle.Ell(A.N, A.M, A.nnz, A.idx, v)


def oracle_step(X, tau, n_occ, width=WIDTH):
    """One SP2 step of the oracle on X (FP32 mode when X holds float values)."""
    tau = np.float32(tau) if X.val.dtype == np.float32 else tau
    rc, Y, d1, d2, wy = oracle.x2(X, tau, M2=width)
    assert rc == 0
    trx, trx2 = oracle.pairwise(d1), oracle.pairwise(d2)
    eta2, _ = oracle.norm2(X, Y)
    up = abs(2.0 * trx - trx2 - n_occ) < abs(trx2 - n_occ)
    nxt = Y
    if up:
        rc, nxt, _ = oracle.update(X, Y, tau, Mo=width)
        assert rc == 0
    return trx, trx2, eta2, up, nxt


def _hist_entry(rep, q, trx, trx2, eta2):
    assert same_float(rep["trx"][q], trx), ("Tr X", q)
    assert same_float(rep["trx2"][q], trx2), ("Tr X^2", q)
    assert same_float(rep["eta2"][q], eta2), ("eta^2", q)


def _cut(Hd, N, params, it):
    params.max_iter = it
    D = E.DeviceEll(N, 256)
    rc, rep = E.sp2_solve(Hd.h, D.h, params)
    assert rc == E.ELL_ENOCONV and rep["iterations"] == it, (rc, rep["iterations"], it)
    return oracle_from_dev(D), rep


def induction(N, params, k, n_occ, phase_f32, tau, ham=None, width=WIDTH):
    """`ham` = (nnz, idx, val, M) of H, else the banded generator's."""
    nnz, idx, val, M = ham if ham is not None else synth.banded_hamiltonian(N, 64)
    Hd = E.DeviceEll.from_host(N, M, nnz, idx, val)
    Xa, rep_a = _cut(Hd, N, params, k)
    Xb, rep_b = _cut(Hd, N, params, k + 1)
    assert rep_b["prec"][k - 1] == (1 if phase_f32 else 0)
    if phase_f32:
        Xa, Xb = _as_f32(Xa), _as_f32(Xb)
    trx, trx2, eta2, up, want = oracle_step(Xa, tau, n_occ, width)
    for rep in (rep_a, rep_b):
        _hist_entry(rep, k - 1, trx, trx2, eta2)
    assert rep_b["up"][k - 1] == (1 if up else 0)
    assert_same_rows(Xb, want, f"X after product {k - 1} ({'2X - X^2' if up else 'X^2'})")
    # the product of X_k itself: its history entry in the longer solve
    tau_b = tau if rep_b["prec"][k] == rep_b["prec"][k - 1] else None
    if tau_b is not None:
        trx, trx2, eta2, _, _ = oracle_step(Xb, tau_b, n_occ, width)
        _hist_entry(rep_b, k, trx, trx2, eta2)


@pytest.mark.parametrize("k", [30, 60])
def test_fp64_n32768_tau1e8(k):
    N, tau = 32768, 1e-8
    p = E.sp2_params(N // 4, tau, 1e-6, max_iter=200)
    induction(N, p, k, N // 4, False, tau)


@pytest.mark.parametrize("k", [30, 60])
def test_fp64_n131072_tau1e9(k):
    N, tau = 131072, 1e-9
    p = E.sp2_params(N // 4, tau, 1e-6, max_iter=200)
    induction(N, p, k, N // 4, False, tau)


def _mixed_params(N):
    return E.sp2_params(N // 4, 1e-9, 1e-6, max_iter=200, precision=E.SP2_MIXED, tau_fp32=1e-7, switch_eta=1e-2)


def test_mixed_n131072_fp32_phase():
    N = 131072
    induction(N, _mixed_params(N), 35, N // 4, True, 1e-7)


def test_mixed_n131072_first_fp64_step():
    """The mixed solve's first FP64 product squares the widened last FP32
    iterate; cut there and one step later."""
    N = 131072
    nnz, idx, val, M = synth.banded_hamiltonian(N, 64)
    Hd = E.DeviceEll.from_host(N, M, nnz, idx, val)
    D = E.DeviceEll(N, 256)
    rc, rep = E.sp2_solve(Hd.h, D.h, _mixed_params(N))
    assert rc == E.ELL_OK
    s = rep["fp32_iterations"]
    assert 0 < s < rep["iterations"] - 1 and rep["prec"][s] == 0 and rep["prec"][s - 1] == 1
    induction(N, _mixed_params(N), s + 1, N // 4, False, 1e-9)
