"""The GPU path on the paper's model Hamiltonians (section "On the Generation of
Model Hamiltonian System Matrices"), against the oracle, bit for bit: the X^2
product on all three systems, SP2 on the two the paper solves (semiconductors
and soft matter, gapped at the 0 eV Fermi level); and a non-banded pattern, a
3D lattice, through both the span form and the ELLPACK kernels."""
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
