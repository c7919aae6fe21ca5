"""Dense-block variant on the matrix cores against the oracle, through the C ABI.

  * FP64: the FP64 MFMA updates each output with a chain of fused multiply-adds
    in ascending k, and the kernel walks k in ascending order, so the product,
    and with it the whole FP64 dense SP2 trajectory, equals the oracle's bit for
    bit.  The product is also held to the order-independent dot-product bound
    |C - A.A| <= gamma_N (|A|.|A|), gamma_N = N u / (1 - N u), u = 2^-53
    (Higham, Accuracy and Stability of Numerical Algorithms, Sec. 3.1).
  * BF16x3: the three bf16 products are exact in FP32 but the MFMA adds them in
    its own order, so against the same split summed in FP64 the only error is
    the FP32 accumulation of 3N terms:
    |C - S| <= gamma_3N(2^-24) (|hi|.|hi| + |hi|.|lo| + |lo|.|hi|).
Non-symmetric inputs are used so a transposed operand cannot pass."""
import numpy as np
import pytest

import oracle
from paper_2102_08505_amd import ellsp2 as E
from paper_2102_08505_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def gamma(n, u):
    return n * u / (1 - n * u)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _split(A32):
    """bf16 hi / lo split by the oracle's rounding (round to nearest even)."""
    bits = A32.view(np.uint32).astype(np.uint64)
    def rne(b):
        exp_all = (b & 0x7F800000) == 0x7F800000
        r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
        return np.where(exp_all, b & 0xFFFF0000, r).astype(np.uint32).view(np.float32)
    hi = rne(bits)
    lo = rne((A32 - hi).view(np.uint32).astype(np.uint64))
    return hi, lo


DENSE_SIZES = [1, 7, 64, 129, 256, 300, 513]


@pytest.mark.parametrize("N", DENSE_SIZES)
def test_dense_x2_f64_bound(N):
    rng = np.random.default_rng(500 + N)
    A = rng.uniform(-1, 1, (N, N))
    dA, dC = _dev(A), torch.zeros((N, N), dtype=torch.float64, device="cuda")
    rc = E.dense_x2(dA.data_ptr(), dC.data_ptr(), N, E.DENSE_F64, torch.cuda.current_stream())
    assert rc == E.ELL_OK, E.ellpack_strerror(rc)
    torch.cuda.synchronize()
    C = dC.cpu().numpy()
    ref = oracle.dense_x2_f64(A)
    assert np.array_equal(C.view(np.uint64), ref.view(np.uint64)), np.max(np.abs(C - ref))
    bound = gamma(N, 2.0 ** -53) * (np.abs(A) @ np.abs(A))
    assert np.all(np.abs(C - A @ A) <= 2 * bound + 1e-300)


@pytest.mark.parametrize("N", DENSE_SIZES)
def test_dense_x2_bf16x3_bound(N):
    rng = np.random.default_rng(600 + N)
    A = rng.uniform(-1, 1, (N, N)).astype(np.float32)
    A[0, 0] = 0.0
    dA, dC = _dev(A), torch.zeros((N, N), dtype=torch.float32, device="cuda")
    rc = E.dense_x2(dA.data_ptr(), dC.data_ptr(), N, E.DENSE_BF16X3, torch.cuda.current_stream())
    assert rc == E.ELL_OK, E.ellpack_strerror(rc)
    torch.cuda.synchronize()
    C = dC.cpu().numpy().astype(np.float64)
    hi, lo = _split(A)
    assert np.array_equal(hi + lo, hi.astype(np.float64) + lo.astype(np.float64))
    h, l = hi.astype(np.float64), lo.astype(np.float64)
    S = h @ h + h @ l + l @ h
    mag = np.abs(h) @ np.abs(h) + np.abs(h) @ np.abs(l) + np.abs(l) @ np.abs(h)
    bound = gamma(3 * N, 2.0 ** -24) * mag
    assert np.all(np.abs(C - S) <= bound + 1e-30), np.max(np.abs(C - S) / (bound + 1e-30))
    # the oracle's own BF16x3 product obeys the same bound, so the two differ by at most twice it
    ref = oracle.dense_x2_bf16x3(A).astype(np.float64)
    assert np.all(np.abs(C - ref) <= 2 * bound + 1e-30)
    # and the split product is within a few bf16^2 units of the FP64 product
    A64 = A.astype(np.float64)
    assert np.all(np.abs(C - A64 @ A64) <= (4 * 2.0 ** -16) * (np.abs(A64) @ np.abs(A64)) + bound + 1e-30)


def test_dense_x2_errors():
    d = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    p = d.data_ptr()
    assert E.dense_x2(p, p, 4, E.DENSE_F64) == E.ELL_EINVAL           # aliasing
    assert E.dense_x2(p, 0, 4, E.DENSE_F64) == E.ELL_EINVAL
    assert E.dense_x2(p, p + 8, 0, E.DENSE_F64) == E.ELL_EINVAL
    assert E.dense_x2(p, p + 8, 4, 7) == E.ELL_EINVAL


def _oracle_params(n_occ, target, max_iter=100, tail=2, switch=1e-3):
    return oracle.make_params(n_occ, 0.0, target, max_iter=max_iter, fp64_tail_steps=tail, switch_eta=switch)


def _solve(H, mode, target, n_occ, max_iter=100, tail=2, switch=1e-3, poll=4):
    N = H.shape[0]
    dH, dD = _dev(H), torch.zeros((N, N), dtype=torch.float64, device="cuda")
    p = E.sp2_params(n_occ, 0.0, target, max_iter=max_iter, fp64_tail_steps=tail, switch_eta=switch,
                     poll_every=poll)
    rc, rep = E.dense_sp2_solve(dH.data_ptr(), N, dD.data_ptr(), mode, p, torch.cuda.current_stream())
    torch.cuda.synchronize()
    return rc, dD.cpu().numpy(), rep


def _projector(H, n_occ):
    w, V = np.linalg.eigh(H)
    k = int(round(n_occ))
    return V[:, :k] @ V[:, :k].T


@pytest.mark.parametrize("N,b", [(64, 4), (200, 6), (257, 8)])
def test_dense_sp2_f64_matches_oracle(N, b):
    H = synth.dense_hamiltonian(N, b, seed=7)
    n_occ = N // 4
    rc, D, rep = _solve(H, E.DENSE_F64, 1e-8, n_occ)
    orc, Do, ro = oracle.dense_sp2(H, oracle.DENSE_F64, _oracle_params(n_occ, 1e-8))
    assert rc == orc == E.ELL_OK
    assert rep["iterations"] == ro["iterations"]
    assert np.array_equal(rep["up"], ro["up"])
    assert rep["fp32_iterations"] == 0
    for k in ("trx", "trx2", "eta2"):
        assert np.array_equal(rep[k].view(np.uint64), ro[k].view(np.uint64)), k
    assert np.array_equal(D.view(np.uint64), Do.view(np.uint64))
    assert rep["emin"] == ro["emin"] and rep["emax"] == ro["emax"]
    P = _projector(H, n_occ)
    assert np.linalg.norm(D - P) < 1e-6


def test_dense_sp2_f64_several_tile_groups():
    """N = 1100: 9 x 9 output tiles of 128, so the symmetric products' tile
    order spans two groups of tile rows (8 and 1) and the XCD stretches cut
    through them; three products against the oracle, bit for bit."""
    N = 1100
    H = synth.dense_hamiltonian(N, 12, seed=11)
    n_occ = N // 4
    rc, D, rep = _solve(H, E.DENSE_F64, 1e-10, n_occ, max_iter=3)
    orc, Do, ro = oracle.dense_sp2(H, oracle.DENSE_F64, _oracle_params(n_occ, 1e-10, max_iter=3))
    assert rc == orc == E.ELL_ENOCONV
    assert rep["iterations"] == ro["iterations"] == 3
    assert np.array_equal(rep["up"], ro["up"])
    for k in ("trx", "trx2", "eta2"):
        assert np.array_equal(rep[k].view(np.uint64), ro[k].view(np.uint64)), k
    assert np.array_equal(D.view(np.uint64), Do.view(np.uint64))


def test_dense_sp2_f64_hamiltonian_not_bitwise_symmetric():
    """One coupling's two sides one ulp apart: the solve takes the full
    product (a transposed copy, every tile) instead of the mirrored upper
    triangle, with the oracle's bits all the same."""
    N = 257
    H = synth.dense_hamiltonian(N, 8, seed=7)
    H[3, 7] = np.nextafter(H[3, 7], np.inf)
    assert H[3, 7] != H[7, 3]
    rc, D, rep = _solve(H, E.DENSE_F64, 1e-8, N // 4)
    orc, Do, ro = oracle.dense_sp2(H, oracle.DENSE_F64, _oracle_params(N // 4, 1e-8))
    assert rc == orc == E.ELL_OK
    for k in ("trx", "trx2", "eta2"):
        assert np.array_equal(rep[k].view(np.uint64), ro[k].view(np.uint64)), k
    assert np.array_equal(D.view(np.uint64), Do.view(np.uint64))


@pytest.mark.parametrize("N,b", [(128, 4), (300, 6)])
def test_dense_sp2_bf16x3_reaches_fp64_accuracy(N, b):
    H = synth.dense_hamiltonian(N, b, seed=11)
    n_occ = N // 4
    rc, D, rep = _solve(H, E.DENSE_BF16X3, 1e-8, n_occ, tail=2, switch=1e-3)
    orc, Do, ro = oracle.dense_sp2(H, oracle.DENSE_BF16X3, _oracle_params(n_occ, 1e-8, tail=2, switch=1e-3))
    assert rc == E.ELL_OK and orc == E.ELL_OK
    assert rep["fp32_iterations"] > 0
    prec = rep["prec"]
    k = rep["fp32_iterations"]
    assert np.all(prec[:k] == 1) and np.all(prec[k:] == 0)
    assert rep["eta"] < 1e-8
    # The FP32 phase leaves X a projector onto a subspace rotated by rounding
    # (the FP64 steps restore idempotency, not the subspace), so the distance to
    # the exact projector is at the FP32 level for both implementations.
    P = _projector(H, n_occ)
    eg, eo = np.linalg.norm(D - P), np.linalg.norm(Do - P)
    assert eg < 1e-3 and eo < 1e-3
    assert eg <= 10 * eo + 1e-9, (eg, eo)
    assert abs(np.trace(D) - n_occ) < 1e-6


def test_dense_sp2_poll_independent():
    H = synth.dense_hamiltonian(96, 5, seed=3)
    a = _solve(H, E.DENSE_F64, 1e-8, 24, poll=1)
    b = _solve(H, E.DENSE_F64, 1e-8, 24, poll=7)
    assert a[0] == b[0] == E.ELL_OK
    assert np.array_equal(a[1], b[1])
    assert a[2]["iterations"] == b[2]["iterations"]


def test_dense_sp2_max_iter_and_errors():
    H = synth.dense_hamiltonian(64, 4, seed=5)
    rc, D, rep = _solve(H, E.DENSE_F64, 1e-12, 16, max_iter=3)
    orc, Do, ro = oracle.dense_sp2(H, oracle.DENSE_F64, _oracle_params(16, 1e-12, max_iter=3))
    assert rc == orc == E.ELL_ENOCONV
    assert rep["iterations"] == ro["iterations"] == 3
    assert np.array_equal(D, Do)
    # degenerate spectrum bounds (N = 1) and occupation outside (0, N)
    assert _solve(np.ones((1, 1)), E.DENSE_F64, 1e-8, 0.5)[0] == E.ELL_EDEGENERATE
    assert _solve(H, E.DENSE_F64, 1e-8, 64)[0] == E.ELL_EDEGENERATE
    Hn = H.copy()
    Hn[3, 5] = np.nan
    assert _solve(Hn, E.DENSE_F64, 1e-8, 16)[0] == E.ELL_ENONFINITE
    d = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    p = E.sp2_params(1, 0.0, 1e-8)
    assert E.dense_sp2_solve(d.data_ptr(), 4, d.data_ptr(), E.DENSE_F64, p)[0] == E.ELL_EINVAL
    assert E.dense_sp2_solve(d.data_ptr(), 4, d.data_ptr() + 128, 5, p)[0] == E.ELL_EINVAL


def test_dense_sp2_reports_each_product_when_profiling():
    N, b, n_occ = 200, 6, 50
    H = synth.dense_hamiltonian(N, b, seed=3)
    dH = torch.from_numpy(H).cuda()
    dD = torch.empty_like(dH)
    p = E.sp2_params(n_occ, 0.0, 1e-8, max_iter=100, poll_every=3, profile=1, tau_fp32=1e-7, switch_eta=1e-3)
    rc, rep = E.dense_sp2_solve(dH.data_ptr(), N, dD.data_ptr(), E.DENSE_BF16X3, p, torch.cuda.current_stream())
    assert rc == E.ELL_OK
    n = rep["iterations"]
    assert rep["x2_launches"] == n and len(rep["x2_seconds_each"]) == n
    assert np.all(rep["x2_seconds_each"] > 0)
    assert abs(rep["x2_seconds_each"].sum() - rep["x2_seconds"]) <= 1e-9 * n
    per = np.where(rep["prec"] == 1, N * N * 8, N * N * 16)  # X read and X^2 written, FP32 or FP64
    assert np.array_equal(rep["x2_bytes_each"], per) and rep["x2_bytes"] == per.sum()
