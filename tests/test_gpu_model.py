"""The GPU path on the paper's model Hamiltonians (section "On the Generation of
Model Hamiltonian System Matrices"), against the oracle, bit for bit: the X^2
product on all three systems, SP2 on the two the paper solves (semiconductors
and soft matter, gapped at the 0 eV Fermi level); and a non-banded pattern, a
3D lattice, through both the span form and the ELLPACK kernels."""
import numpy as np
import pytest

import oracle
from paper_2102_08505_amd import ellsp2 as E
from paper_2102_08505_amd import synth
from tests.gpu_helpers import assert_same_rows, oracle_from_dev, same_float
from tests.test_gpu_parity import assert_same_trajectory

pytestmark = pytest.mark.gpu


def model(kind, N):
    nnz, idx, val, M = synth.model_hamiltonian(kind, N)
    return oracle.Ell(N, M, nnz, idx, val), (nnz, idx, val, M)


def x2_both(kind, N, tau=1e-5):
    H, (nnz, idx, val, M) = model(kind, N)
    rc, Y, d1, d2, wy = oracle.x2(H, tau)
    assert rc == 0
    X = E.DeviceEll.from_host(N, M, nnz, idx, val)
    Yd = E.DeviceEll(N, wy, E.ELL_F64)
    rc_g, tr, w = E.ellpack_x2_threshold(X.h, Yd.h, tau)
    assert rc_g == E.ELL_OK and w == wy
    assert_same_rows(oracle_from_dev(Yd), Y, f"{kind} N={N} X^2")
    assert same_float(tr[0], oracle.pairwise(d1)) and same_float(tr[1], oracle.pairwise(d2))


@pytest.mark.parametrize("kind", ["metal", "semiconductor", "soft_matter"])
@pytest.mark.parametrize("N", [300, 1000])
def test_x2_of_model_hamiltonians_bitwise(kind, N):
    x2_both(kind, N)


def test_x2_of_a_metal_with_output_windows_of_73_blocks():
    """N = 4608: a wavefront's output window spans up to 4605 columns (73
    aligned blocks of 64), so the norm's per-row tree climbs past 64 blocks
    and starts from blocks at odd positions."""
    x2_both("metal", 4608)


def sp2_both(kind, N, mixed=False, tau=1e-8, target=1e-6, M=64):
    H, (nnz, idx, val, Mh) = model(kind, N)
    n_occ, w = synth.fermi_occupation(nnz, idx, val, Mh)
    assert w[n_occ] - w[n_occ - 1] > 1e-3
    po = oracle.make_params(n_occ, tau, target, max_iter=200,
                            precision=oracle.PREC_MIXED if mixed else oracle.PREC_F64,
                            tau_fp32=1e-7, switch_eta=1e-2)
    rc_o, Do, ro = oracle.sp2(H, po, Mo=N)
    Hd = E.DeviceEll.from_host(N, Mh, nnz, idx, val)
    Dd = E.DeviceEll(N, M, E.ELL_F64)
    pg = E.sp2_params(n_occ, tau, target, max_iter=200, precision=E.SP2_MIXED if mixed else E.SP2_F64,
                      tau_fp32=1e-7, switch_eta=1e-2)
    rc_g, rg = E.sp2_solve(Hd.h, Dd.h, pg)
    return (rc_o, Do, ro), (rc_g, Dd, rg)


@pytest.mark.parametrize("kind", ["semiconductor", "soft_matter"])
def test_sp2_on_model_hamiltonians_bitwise(kind):
    o, g = sp2_both(kind, 256)
    assert o[0] == 0
    assert_same_trajectory(o, g)


def test_sp2_mixed_on_soft_matter_bitwise():
    o, g = sp2_both("soft_matter", 256, mixed=True, tau=1e-9)
    assert o[0] == 0
    assert_same_trajectory(o, g)
    assert 0 < g[2]["fp32_iterations"] < g[2]["iterations"]


# ------------------------------------------ a non-banded pattern: the 3D lattice
def grid(n):
    nnz, idx, val, M = synth.grid3d_hamiltonian(n)
    return oracle.Ell(n ** 3, M, nnz, idx, val), (nnz, idx, val, M)


@pytest.mark.parametrize("n", [10, 16])
def test_x2_of_the_3d_lattice_bitwise(n):
    """n = 10: rows fill 7 of 201 interval positions (span form); n = 16: 7 of
    513, below 1/64 (ELLPACK kernels)."""
    H, (nnz, idx, val, M) = grid(n)
    N = n ** 3
    rc, Y, d1, d2, wy = oracle.x2(H, 1e-5)
    X = E.DeviceEll.from_host(N, M, nnz, idx, val)
    Yd = E.DeviceEll(N, wy, E.ELL_F64)
    rc_g, tr, w = E.ellpack_x2_threshold(X.h, Yd.h, 1e-5)
    assert rc_g == E.ELL_OK and w == wy
    assert_same_rows(oracle_from_dev(Yd), Y, f"3D lattice n={n} X^2")
    assert same_float(tr[0], oracle.pairwise(d1)) and same_float(tr[1], oracle.pairwise(d2))


def test_sp2_on_the_3d_lattice_bitwise():
    n = 6
    H, (nnz, idx, val, M) = grid(n)
    N = n ** 3
    po = oracle.make_params(N // 2, 1e-8, 1e-6, max_iter=200)
    rc_o, Do, ro = oracle.sp2(H, po, Mo=N)
    Hd = E.DeviceEll.from_host(N, M, nnz, idx, val)
    Dd = E.DeviceEll(N, 32, E.ELL_F64)
    rc_g, rg = E.sp2_solve(Hd.h, Dd.h, E.sp2_params(N // 2, 1e-8, 1e-6, max_iter=200))
    assert rc_o == 0
    assert_same_trajectory((rc_o, Do, ro), (rc_g, Dd, rg))


# ------------------------------------------------ the paper's ExaSP2 size: 32000 orbitals
#
# SP2 at 32000 orbitals with the benchmark's settings there (FP64 tau 1e-10,
# target 1e-6; N_occ the inertia count below the Fermi level), by induction
# over steps as for the banded solves: cut the solve at q and q + 1 products and
# apply one oracle step to the GPU's X_{q-1}.  The cut points are taken from the
# solve's own branch history so that both branches are stepped.

N_EXA, TAU_EXA = 32000, 1e-10


def _branch_points(Hd, n_occ, lo, hi, **kw):
    """(q with branch 2X - X^2 at product q - 1, q with branch X^2), lo <= q < hi."""
    D = E.DeviceEll(N_EXA, 256)
    rc, rep = E.sp2_solve(Hd.h, D.h, E.sp2_params(n_occ, TAU_EXA, 1e-6, max_iter=hi, **kw))
    assert rc == E.ELL_ENOCONV and rep["iterations"] == hi
    up = [int(u) for u in rep["up"][:hi]]
    q_up = next(q for q in range(lo, hi) if up[q - 1] == 1)
    q_sq = next(q for q in range(lo, hi) if up[q - 1] == 0)
    return q_up, q_sq


@pytest.mark.parametrize("mixed", [False, True])
def test_sp2_on_soft_matter_at_32000_orbitals_by_induction(mixed):
    """Soft matter, whole matrices: FP64, and the mixed solve inside its FP32
    phase (tau_fp32 1e-7), at products 20 .. 24 (rows of 500 - 900 entries)."""
    from tests.test_gpu_fullsize import induction
    nnz, idx, val, M = synth.model_hamiltonian("soft_matter", N_EXA)
    n_occ, _ = synth.fermi_occupation_banded(nnz, idx, val, M)
    kw = dict(precision=E.SP2_MIXED, tau_fp32=1e-7, switch_eta=1e-2) if mixed else {}
    Hd = E.DeviceEll.from_host(N_EXA, M, nnz, idx, val)
    for q in _branch_points(Hd, n_occ, 20, 25, **kw):
        p = E.sp2_params(n_occ, TAU_EXA, 1e-6, max_iter=200, **kw)
        induction(N_EXA, p, q, n_occ, mixed, 1e-7 if mixed else TAU_EXA, ham=(nnz, idx, val, M), width=2048)


def test_sp2_on_semiconductor_at_32000_orbitals_sampled_rows():
    """Semiconductor (rows of 3000 - 3500 entries: whole oracle products are
    too slow here): at an X^2 step between products 15 and 25, sampled rows of
    the GPU's X_q against the oracle's rows of prune(X_{q-1}^2), and Tr X_{q-1}
    against the pairwise tree of the GPU's X_{q-1} diagonal."""
    from tests.test_gpu_fullsize import _cut
    nnz, idx, val, M = synth.model_hamiltonian("semiconductor", N_EXA)
    n_occ = N_EXA // 2  # the inertia count below 0.05, inside the gap (0, 0.93)
    Hd = E.DeviceEll.from_host(N_EXA, M, nnz, idx, val)
    _, q = _branch_points(Hd, n_occ, 15, 25)
    # cut after q and q + 1 products: X_{q-1} (squared by product q - 1) and X_q
    Xa, _ = _cut(Hd, N_EXA, E.sp2_params(n_occ, TAU_EXA, 1e-6, max_iter=200), q)
    Xb, rep_b = _cut(Hd, N_EXA, E.sp2_params(n_occ, TAU_EXA, 1e-6, max_iter=200), q + 1)
    assert rep_b["up"][q - 1] == 0
    ia = Xa.idx.reshape(N_EXA, Xa.M)
    va = Xa.val.reshape(N_EXA, Xa.M)
    diag = np.array([va[i, :Xa.nnz[i]][ia[i, :Xa.nnz[i]] == i].sum() for i in range(N_EXA)])
    assert same_float(rep_b["trx"][q - 1], oracle.pairwise(diag))
    rows = np.array([0, 1, 2, 3, 1220, 1221, 5000, 9999, 16000, 16001, 23457, N_EXA - 1221, N_EXA - 2, N_EXA - 1])
    rc, nz, ix, vl, _ = oracle.x2_rows(Xa, TAU_EXA, rows, M2=8192)
    assert rc == 0
    ib = Xb.idx.reshape(N_EXA, Xb.M)
    vb = Xb.val.reshape(N_EXA, Xb.M)
    for r, i in enumerate(rows):
        assert Xb.nnz[i] == nz[r], (i, Xb.nnz[i], nz[r])
        assert np.array_equal(ib[i, :nz[r]], ix[r, :nz[r]]), i
        assert np.array_equal(vb[i, :nz[r]].view(np.uint64), vl[r, :nz[r]].view(np.uint64)), i
