"""The paper's model Hamiltonians (section "On the Generation of Model
Hamiltonian System Matrices"): the generator's structure against the section's
definition, the one sparsity figure it prints that the reading reproduces, and
oracle pins on these inputs (X^2 against a dense product, SP2 against the
spectral projector at the 0 eV Fermi level); and the same for a non-banded
pattern, a 3D lattice in lexicographic order.  CPU only."""
import numpy as np
import pytest

import oracle
from paper_2102_08505_amd import synth

KINDS = ("metal", "semiconductor", "soft_matter")


def dense(kind, N, **kw):
    nnz, idx, val, M = synth.model_hamiltonian(kind, N, **kw)
    return synth.ell_to_dense(N, M, nnz, idx, val), (nnz, idx, val, M)


def test_parameter_sets_are_the_sections():
    # metals: d_AA = d_BB = -1, k = -0.01; semiconductors: d_BB = -1, d_AB = -2,
    # k = -0.01; soft matter: d_BB = -1, d_AB = -1, eps_A = -10, k = -0.1, r = 1;
    # every other parameter 0
    P = synth.MODEL_PARAMS
    assert P["metal"] == dict(eps_a=0.0, eps_b=0.0, d_aa=-1.0, d_bb=-1.0, d_ab=0.0, k=-0.01, r=0.0)
    assert P["semiconductor"] == dict(eps_a=0.0, eps_b=0.0, d_aa=0.0, d_bb=-1.0, d_ab=-2.0, k=-0.01, r=0.0)
    assert P["soft_matter"] == dict(eps_a=-10.0, eps_b=0.0, d_aa=0.0, d_bb=-1.0, d_ab=-1.0, k=-0.1, r=1.0)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("N", [1, 2, 301])
def test_symmetric_sorted_and_above_threshold(kind, N):
    D, (nnz, idx, val, M) = dense(kind, N)
    assert np.array_equal(D, D.T)
    rows = synth.ell_rows(N, M, nnz, idx, val)
    for c, v in rows:
        assert np.all(np.diff(c) > 0)
        assert np.all(np.abs(v) > 1e-5)


@pytest.mark.parametrize("kind", KINDS)
def test_orbital_types_and_couplings(kind):
    N = 300
    D, _ = dense(kind, N)
    p = synth.MODEL_PARAMS[kind]
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    off = i != j
    aa = off & (i % 2 == 0) & (j % 2 == 0)
    bb = off & (i % 2 == 1) & (j % 2 == 1)
    ab = off & (i % 2 != j % 2)
    damp = np.exp(p["k"] * np.abs(i - j))
    for mask, d in ((aa, p["d_aa"]), (bb, p["d_bb"]), (ab, p["d_ab"])):
        if d == 0.0:
            assert np.all(D[mask] == 0.0)
            continue
        lo, hi = sorted((d * (1 - p["r"]), d * (1 + p["r"])))
        stored = mask & (D != 0)
        ratio = D[stored] / damp[stored]  # param (1 + r RAND)
        assert np.all(ratio >= lo - 1e-12) and np.all(ratio <= hi + 1e-12)
        if p["r"] == 0.0:  # no noise: exactly d exp(k |j - i|) wherever that exceeds the threshold
            want = np.where(np.abs(d * damp) > 1e-5, d * damp, 0.0)
            assert np.array_equal(D[mask], want[mask])
        else:  # the noise spreads the factor over the whole range, centred on 1
            f = ratio / d
            assert f.min() < 0.1 and f.max() > 1.9 and abs(f.mean() - 1.0) < 0.05


@pytest.mark.parametrize("kind", KINDS)
def test_onsite_energies(kind):
    N = 400
    D, _ = dense(kind, N)
    p = synth.MODEL_PARAMS[kind]
    diag = np.diag(D)
    for parity, e in ((0, p["eps_a"]), (1, p["eps_b"])):
        d = diag[parity::2]
        lo, hi = sorted((e * (1 - p["r"]), e * (1 + p["r"])))
        assert np.all(d >= lo) and np.all(d <= hi)
        if e == 0.0:
            assert np.all(d == 0.0)  # an onsite energy of 0 is not stored
    if kind == "soft_matter":
        assert diag[0::2].min() < -19.0 and diag[0::2].max() > -1.0


@pytest.mark.parametrize("kind", KINDS)
def test_reach_is_the_last_offset_above_threshold(kind):
    r = synth.model_reach(kind)
    p = synth.MODEL_PARAMS[kind]
    top = max(abs(p["d_aa"]), abs(p["d_bb"]), abs(p["d_ab"])) * (1 + p["r"])
    assert top * np.exp(p["k"] * r) > 1e-5 >= top * np.exp(p["k"] * (r + 1))
    N = 3 * r + 5
    nnz, idx, val, M = synth.model_hamiltonian(kind, N)
    far = max(int(np.abs(c - i).max()) for i, (c, v) in enumerate(synth.ell_rows(N, M, nnz, idx, val)) if len(c))
    assert far <= r


def test_seed_and_stream_change_only_the_noise():
    a, _ = dense("soft_matter", 200, seed=0)
    b, _ = dense("soft_matter", 200, seed=1)
    c, _ = dense("semiconductor", 200, seed=0)
    d, _ = dense("semiconductor", 200, seed=7)
    assert not np.array_equal(a, b)
    assert np.array_equal(c, d)  # no noise (r = 0): the seed has nothing to change


def test_semiconductor_sparsity_is_the_printed_94_percent():
    # the section prints 94 % sparse for its semiconductor matrices, the size its
    # SP2 runs use being 32000 orbitals
    N = 32000
    nnz, idx, val, M = synth.model_hamiltonian("semiconductor", N)
    sparsity = 1.0 - nnz.sum(dtype=np.int64) / (N * N)
    assert abs(sparsity - 0.94) < 0.01


def test_fermi_occupation_counts_eigenvalues_below_zero():
    D = np.diag([-2.0, -0.5, 0.25, 3.0])
    nnz, idx, val, M = synth.dense_to_ell(D)
    n, w = synth.fermi_occupation(nnz, idx, val, M)
    assert n == 2 and np.allclose(w, [-2.0, -0.5, 0.25, 3.0])


@pytest.mark.parametrize("kind,N,mus", [("banded", 700, (-1.0, 0.0, 0.37)),
                                         ("soft_matter", 1500, (0.0, -0.5)),
                                         ("semiconductor", 1500, (0.05, -0.3, 1.0)),
                                         ("metal", 1200, (0.0, 0.02))])
def test_banded_occupation_is_the_eigenvalue_count(kind, N, mus):
    """Sylvester's inertia over block Schur complements gives the number of
    eigenvalues below mu that the dense spectrum gives."""
    if kind == "banded":
        nnz, idx, val, M = synth.banded_hamiltonian(N, 9, seed=3)
    else:
        nnz, idx, val, M = synth.model_hamiltonian(kind, N)
    _, w = synth.fermi_occupation(nnz, idx, val, M)
    for mu in mus:
        n, smallest = synth.fermi_occupation_banded(nnz, idx, val, M, mu=mu)
        assert n == int((w < mu).sum()), (kind, mu)
        assert smallest > 0


def test_semiconductor_occupation_counts_its_zero_energy_band():
    """The semiconductor's A orbitals carry no onsite energy and no A-A
    coupling: the upper half of its occupied states crowds against 0 from
    below (the highest round to negatives of order 1e-10), and nothing lies in
    (0, 0.93).  The count below 0 (dense spectrum) is the well-conditioned
    count below 0.05 (banded inertia): N / 2."""
    N = 2000
    nnz, idx, val, M = synth.model_hamiltonian("semiconductor", N)
    n0, w = synth.fermi_occupation(nnz, idx, val, M)
    assert n0 == N // 2 and w[n0] > 0.9 and abs(w[n0 - 1]) < 1e-6
    assert synth.fermi_occupation_banded(nnz, idx, val, M, mu=0.05)[0] == N // 2


# ------------------------------------------------------- oracle pins on these inputs
def test_oracle_x2_of_a_model_hamiltonian_is_the_dense_product():
    N = 200
    D, (nnz, idx, val, M) = dense("metal", N)
    H = oracle.Ell(N, M, nnz, idx, val)
    rc, Y, d1, d2, w = oracle.x2(H, 0.0)
    assert rc == 0
    ref = D @ D
    # fma chains of at most N terms of magnitude <= 1: the sum's rounding bound
    bound = N * np.finfo(np.float64).eps * (np.abs(D) @ np.abs(D))
    assert np.all(np.abs(Y.dense() - ref) <= bound + 1e-300)
    assert np.array_equal(d1, np.diag(D))


@pytest.mark.parametrize("kind", ["semiconductor", "soft_matter"])
def test_oracle_sp2_reaches_the_projector_below_the_fermi_level(kind):
    N = 96
    D, (nnz, idx, val, M) = dense(kind, N)
    n_occ, w = synth.fermi_occupation(nnz, idx, val, M)
    assert w[n_occ] - w[n_occ - 1] > 1e-3  # gapped at 0 eV
    vals, V = np.linalg.eigh(D)
    P = V[:, :n_occ] @ V[:, :n_occ].T
    H = oracle.Ell(N, M, nnz, idx, val)
    p = oracle.make_params(n_occ, 0.0, 1e-10, max_iter=300)
    rc, X, rep = oracle.sp2(H, p)
    assert rc == 0
    assert np.linalg.norm(X.dense() - P) <= 1e-8
    assert abs(rep["trace_x"] - n_occ) <= 1e-8


# ------------------------------------------ a non-banded pattern: the 3D lattice
@pytest.mark.parametrize("n", [1, 3, 6])
def test_grid3d_structure(n):
    nnz, idx, val, M = synth.grid3d_hamiltonian(n, delta=1.5, t=1.0, r=0.1)
    N = n ** 3
    D = synth.ell_to_dense(N, M, nnz, idx, val)
    assert np.array_equal(D, D.T)
    for i, (c, v) in enumerate(synth.ell_rows(N, M, nnz, idx, val)):
        x, y, z = i % n, (i // n) % n, i // (n * n)
        want = sorted([i] + [i + s * d for d, co in ((1, x), (n, y), (n * n, z)) for s in (-1, 1)
                             if 0 <= co + s < n])
        assert list(c) == want
        assert D[i, i] == (1.5 if (x + y + z) % 2 == 0 else -1.5)
        off = v[c != i]
        assert np.all(off <= -0.9 + 1e-15) and np.all(off >= -1.1 - 1e-15)


def test_grid3d_gap_and_occupation():
    nnz, idx, val, M = synth.grid3d_hamiltonian(6)
    n_occ, w = synth.fermi_occupation(nnz, idx, val, M)
    assert n_occ == 6 ** 3 // 2
    assert w[n_occ - 1] <= -1.0 + 1e-12 and w[n_occ] >= 1.0 - 1e-12  # nothing inside (-delta, delta)


def test_oracle_sp2_on_the_3d_lattice_reaches_the_projector():
    n = 4
    nnz, idx, val, M = synth.grid3d_hamiltonian(n)
    N = n ** 3
    D = synth.ell_to_dense(N, M, nnz, idx, val)
    w, V = np.linalg.eigh(D)
    P = V[:, : N // 2] @ V[:, : N // 2].T
    p = oracle.make_params(N // 2, 0.0, 1e-10, max_iter=200)
    rc, X, rep = oracle.sp2(oracle.Ell(N, M, nnz, idx, val), p)
    assert rc == 0
    assert np.linalg.norm(X.dense() - P) <= 1e-8
