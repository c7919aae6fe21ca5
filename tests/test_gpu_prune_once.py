"""The one-pruning SP2 mode (`prune_once`) and the two-output iteration for a
Hamiltonian that is not bitwise symmetric, on the GPU, against the oracle:
whole trajectories (traces, norms, branches, widths, the result) bit for bit,
on each kernel path a solve can take -- the symmetric one-output iteration,
the two-output iteration, the ELLPACK fallback and the batched stack -- and
the benchmark's size by induction."""
import numpy as np
import pytest

import oracle
from paper_2102_08505_amd import ellsp2 as E
from paper_2102_08505_amd import synth
from tests.gpu_helpers import assert_same_rows, oracle_from_dev
from tests.test_gpu_batched import _check, _instances, _run
from tests.test_gpu_parity import assert_same_trajectory

pytestmark = pytest.mark.gpu


def both(N, M, nnz, idx, val, tau, target, once, mixed=False, max_iter=120, Mg=64, tau32=1e-7,
         switch_eta=1e-3):
    H = oracle.Ell(N, M, nnz, idx, val)
    po = oracle.make_params(N // 4, tau, target, max_iter=max_iter,
                            precision=oracle.PREC_MIXED if mixed else oracle.PREC_F64,
                            tau_fp32=tau32, switch_eta=switch_eta, prune_once=once)
    o = oracle.sp2(H, po, Mo=N)
    Hd = E.DeviceEll.from_host(N, M, nnz, idx, val)
    Dd = E.DeviceEll(N, Mg, E.ELL_F64)
    pg = E.sp2_params(N // 4, tau, target, max_iter=max_iter, precision=E.SP2_MIXED if mixed else E.SP2_F64,
                      tau_fp32=tau32, switch_eta=switch_eta, prune_once=once)
    rc, rep = E.sp2_solve(Hd.h, Dd.h, pg)
    return o, (rc, Dd, rep)


def asymmetric(N, b, seed):
    """A banded Hamiltonian with one coupling's two sides one ulp apart: not
    bitwise symmetric, so the solve takes the two-output iteration."""
    nnz, idx, val, M = synth.banded_hamiltonian(N, b, seed=seed)
    D = synth.ell_to_dense(N, M, nnz, idx, val)
    D[5, 9] = np.nextafter(D[5, 9], np.inf)
    assert D[5, 9] != D[9, 5]
    return (N, *_ell(D))


def pattern_asymmetric(N, b, seed, below):
    """A banded Hamiltonian plus one entry outside the band with no partner:
    below the diagonal (found only by counting the entries on each side) or
    above it (found by looking up its mirror)."""
    nnz, idx, val, M = synth.banded_hamiltonian(N, b, seed=seed)
    D = synth.ell_to_dense(N, M, nnz, idx, val)
    i, j = (300, 10) if below else (10, 300)
    assert D[i, j] == 0.0 and D[j, i] == 0.0
    D[i, j] = 0.02
    return (N, *_ell(D))


def _ell(D):
    nnz, idx, val, M = synth.dense_to_ell(D)
    return M, nnz, idx, val


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("once", [0, 1])
def test_symmetric_iteration_both_prunings(once, mixed):
    N, b = 512, 16
    nnz, idx, val, M = synth.banded_hamiltonian(N, b)
    o, g = both(N, M, nnz, idx, val, 1e-9, 1e-6 if mixed else 1e-7, once, mixed=mixed)
    assert_same_trajectory(o, g)
    assert g[0] == E.ELL_OK


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("once", [0, 1])
def test_two_output_iteration_for_a_hamiltonian_not_bitwise_symmetric(once, mixed):
    N, M, nnz, idx, val = asymmetric(512, 16, seed=3)
    o, g = both(N, M, nnz, idx, val, 1e-9, 1e-6 if mixed else 1e-7, once, mixed=mixed)
    assert_same_trajectory(o, g)
    assert g[0] == E.ELL_OK


@pytest.mark.parametrize("below", [True, False])
def test_two_output_iteration_for_a_hamiltonian_with_an_unpaired_entry(below):
    N, M, nnz, idx, val = pattern_asymmetric(512, 16, seed=3, below=below)
    o, g = both(N, M, nnz, idx, val, 1e-9, 1e-7, 0)
    assert_same_trajectory(o, g)
    assert g[0] == o[0]


def test_prune_once_changes_the_trajectory():
    N, b = 512, 16
    nnz, idx, val, M = synth.banded_hamiltonian(N, b)
    _, (_, _, r1) = both(N, M, nnz, idx, val, 1e-5, 1e-8, 1, max_iter=30)
    _, (_, _, r0) = both(N, M, nnz, idx, val, 1e-5, 1e-8, 0, max_iter=30)
    assert not np.array_equal(r1["eta2"], r0["eta2"])


def test_prune_once_on_the_ellpack_fallback():
    """A long-range coupling (rows 10 and 900) that the span kernels cannot
    hold: the solve continues on the ELLPACK kernel."""
    N = 1024
    nnz, idx, val, M = synth.banded_hamiltonian(N, 4, seed=7)
    D = synth.ell_to_dense(N, M, nnz, idx, val)
    D[10, 900] = D[900, 10] = 0.3
    M, nnz, idx, val = _ell(D)
    o, g = both(N, M, nnz, idx, val, 1e-7, 1e-6, 1)
    assert_same_trajectory(o, g)


@pytest.mark.parametrize("k", [30])
def test_prune_once_full_size_step(k):
    """The benchmark's Hamiltonian (N = 32768, half-bandwidth 64, FP64,
    tau = 1e-8) in the one-pruning mode, by induction: the GPU's X_k and
    X_{k+1} against one oracle step of that mode applied to X_k -- the
    unpruned X_k^2, the traces, the branch, then prune(2X - X^2) or
    prune(X^2)."""
    N, b, tau = 32768, 64, 1e-8
    nnz, idx, val, M = synth.banded_hamiltonian(N, b)
    Hd = E.DeviceEll.from_host(N, M, nnz, idx, val)
    outs = []
    for it in (k, k + 1):
        D = E.DeviceEll(N, 256, E.ELL_F64)
        rc, rep = E.sp2_solve(Hd.h, D.h, E.sp2_params(N // 4, tau, 1e-6, max_iter=it, prune_once=1),
                              history=False)
        assert rc == E.ELL_ENOCONV and rep["iterations"] == it
        outs.append(oracle_from_dev(D))
    Xk, Xk1 = outs
    rc, Y, d1, d2, wy = oracle.x2(Xk, 0.0, M2=1024)
    assert rc == 0
    trx, trx2 = oracle.pairwise(d1), oracle.pairwise(d2)
    up = abs(2.0 * trx - trx2 - N // 4) < abs(trx2 - N // 4)
    if up:
        rc, want, _ = oracle.update(Xk, Y, tau, Mo=512)
    else:
        rc, want, _ = oracle.prune(Y, tau, Mo=512)
    assert rc == 0
    assert_same_rows(Xk1, want, f"X_{k + 1} ({'2X - X^2' if up else 'X^2'})")


def test_batched_prune_once_instances_equal_single_solves_and_the_oracle():
    specs = [(64, 4, 1), (257, 8, 3), (300, 9, 4), (513, 16, 5), (130, 4, 10), (77, 4, 7)]
    inst = _instances(specs)
    params = []
    for q, (N, *_r) in enumerate(inst):
        params.append(E.sp2_params(N // 4, 1e-9, 1e-6, max_iter=100,
                                   precision=E.SP2_MIXED if q % 3 == 1 else E.SP2_F64, tau_fp32=1e-7,
                                   switch_eta=1e-3, poll_every=4, prune_once=0 if q == 2 else 1))
    rc_b, reps_b, Db, singles, Hs = _run(inst, params)
    _check(rc_b, reps_b, Db, singles)
    for q in (0, 1, 4):
        N, Mh, nnz, idx, val = inst[q]
        po = oracle.make_params(N // 4, 1e-9, 1e-6, max_iter=100,
                                precision=oracle.PREC_MIXED if q % 3 == 1 else oracle.PREC_F64,
                                tau_fp32=1e-7, switch_eta=1e-3, prune_once=1)
        o = oracle.sp2(oracle.Ell(N, Mh, nnz, idx, val), po, Mo=N)
        assert_same_trajectory(o, (reps_b[q]["status"], Db[q], reps_b[q]))
