"""Pins of the oracle's sector matrix (paper eq. (1)/(2), Sec. 2.1).

The strongest pin is an independent construction of eq. (2): the full 2^L x 2^L
matrix assembled from Kronecker products of Pauli matrices, then restricted to
the sector.  It fixes the sign and size of the flip-flop element, the site/bit
convention, Delta and the field term element by element.
"""

import math

import numpy as np
import pytest

from oracle import basis, hamiltonian, freefermion
from paper_2012_00217_amd import workloads

SX = np.array([[0, 1], [1, 0]], dtype=complex) / 2
SY = np.array([[0, 1j], [-1j, 0]], dtype=complex) / 2  # basis (down, up) = (bit 0, bit 1)
SZ = np.array([[-1, 0], [0, 1]], dtype=complex) / 2
I2 = np.eye(2, dtype=complex)


def _site(op, i, L):
    """Operator on site i of L (site i = bit i: factor for site L-1 leftmost)."""
    return np.kron(np.kron(np.eye(1 << (L - 1 - i)), op), np.eye(1 << i))


def kron_hamiltonian(L, J, Delta, h):
    """Eq. (2) literally: bond terms J(XX + YY + Delta ZZ) plus fields h_i Z_i."""
    H = np.zeros((1 << L, 1 << L), dtype=complex)
    for i in range(L - 1):
        for op, c in ((SX, 1.0), (SY, 1.0), (SZ, Delta)):
            H += J * c * _site(op, i, L) @ _site(op, i + 1, L)
    for i in range(L):
        H += h[i] * _site(SZ, i, L)
    return H


@pytest.mark.parametrize("L", [2, 3, 5, 8])
def test_sector_matrix_equals_tensor_product_construction(L):
    rng = np.random.default_rng(100 + L)
    J, Delta = rng.uniform(0.5, 2), rng.uniform(-1.5, 1.5)
    h = rng.uniform(-3, 3, L)
    Hf = kron_hamiltonian(L, J, Delta, h)
    assert np.max(np.abs(Hf.imag)) < 1e-14
    Hf = Hf.real
    allstates = np.arange(1 << L, dtype=np.uint64)
    for k in range(L + 1):
        st, H = hamiltonian.sector_matrix(L, k, J, Delta, h)
        idx = st.astype(np.int64)
        np.testing.assert_allclose(H.toarray(), Hf[np.ix_(idx, idx)], rtol=0, atol=1e-14)
        other = allstates[np.bitwise_count(allstates) != k].astype(np.int64)
        assert np.max(np.abs(Hf[np.ix_(idx, other)]), initial=0.0) == 0.0  # S^z conservation


def test_union_of_sector_spectra_is_full_spectrum():
    L = 7
    h = np.random.default_rng(5).uniform(-2, 2, L)
    full = np.linalg.eigvalsh(kron_hamiltonian(L, 1.0, 1.0, h).real)
    parts = []
    for k in range(L + 1):
        _, H = hamiltonian.sector_matrix(L, k, 1.0, 1.0, h)
        parts.append(np.linalg.eigvalsh(H.toarray()))
    np.testing.assert_allclose(np.sort(np.concatenate(parts)), full, atol=1e-12)


@pytest.mark.parametrize("L", [10, 12])
def test_trace_closed_form_at_zero_magnetisation(L):
    """sum_s E(s) = -J Delta n / 4 at S^z = 0, whatever the fields."""
    for seed in range(3):
        rng = np.random.default_rng(seed)
        J, Delta = rng.uniform(0.5, 2), rng.uniform(-1, 2)
        h = rng.uniform(-8, 8, L)
        st, H = hamiltonian.sector_matrix(L, L // 2, J, Delta, h)
        assert abs(H.diagonal().sum() - (-J * Delta * len(st) / 4)) < 1e-9


@pytest.mark.parametrize("L,k", [(10, 5), (11, 4), (9, 2)])
def test_offdiagonal_count_and_ones_form(L, k):
    """nnz_off = n 2k(L-k)/L;  1^T H 1 = trace + (J/2) nnz_off."""
    h = np.random.default_rng(1).uniform(-1, 1, L)
    J = 1.3
    st, H = hamiltonian.sector_matrix(L, k, J, 0.7, h)
    n = len(st)
    r, c, _ = hamiltonian.offdiagonal_triplets(L, st, J)
    assert len(r) * L == n * 2 * k * (L - k)
    one = np.ones(n)
    assert abs(one @ (H @ one) - (H.diagonal().sum() + 0.5 * J * len(r))) < 1e-9


def test_two_site_singlet_triplet():
    """L = 2, S^z = 0: -J Delta/4 +- sqrt((J/2)^2 + ((h0 - h1)/2)^2)."""
    for J, Delta, h in [(1.0, 1.0, [0.0, 0.0]), (0.7, 1.9, [0.3, -1.1])]:
        _, H = hamiltonian.sector_matrix(2, 1, J, Delta, np.array(h))
        w = np.linalg.eigvalsh(H.toarray())
        rad = math.sqrt((J / 2) ** 2 + ((h[0] - h[1]) / 2) ** 2)
        np.testing.assert_allclose(w, [-J * Delta / 4 - rad, -J * Delta / 4 + rad], atol=1e-15)
    _, H = hamiltonian.sector_matrix(2, 1, 1.0, 1.0, np.zeros(2))
    np.testing.assert_allclose(np.linalg.eigvalsh(H.toarray()), [-0.75, 0.25], atol=1e-15)


@pytest.mark.parametrize("L,k", [(8, 4), (10, 5), (11, 3)])
def test_free_fermion_spectrum_at_delta_zero(L, k):
    """Delta = 0: every sector eigenvalue is a subset sum of single-particle levels."""
    h = np.random.default_rng(L).uniform(-4, 4, L)
    J = 1.0
    st, H = hamiltonian.sector_matrix(L, k, J, 0.0, h)
    w = np.linalg.eigvalsh(H.toarray())
    e = np.sort(freefermion.energies(L, k, J, h, st))
    np.testing.assert_allclose(w, e, atol=1e-12)


@pytest.mark.parametrize("L", [8, 10])
def test_su2_multiplets_at_zero_field(L):
    """h = 0, J = Delta = 1: the S^z = 1 spectrum is contained in the S^z = 0 one."""
    _, H0 = hamiltonian.sector_matrix(L, L // 2, 1.0, 1.0, np.zeros(L))
    _, H1 = hamiltonian.sector_matrix(L, L // 2 + 1, 1.0, 1.0, np.zeros(L))
    w0 = np.linalg.eigvalsh(H0.toarray())
    w1 = np.linalg.eigvalsh(H1.toarray())
    assert np.all(np.min(np.abs(w1[:, None] - w0[None, :]), axis=1) < 1e-10)
    # the inclusion fails for an anisotropic chain: Delta is pinned against J
    _, H0b = hamiltonian.sector_matrix(L, L // 2, 1.0, 1.1, np.zeros(L))
    _, H1b = hamiltonian.sector_matrix(L, L // 2 + 1, 1.0, 1.1, np.zeros(L))
    w0b = np.linalg.eigvalsh(H0b.toarray())
    w1b = np.linalg.eigvalsh(H1b.toarray())
    assert np.max(np.min(np.abs(w1b[:, None] - w0b[None, :]), axis=1)) > 1e-6


def test_flip_and_reflection_symmetries():
    L = 9
    h = np.random.default_rng(2).uniform(-3, 3, L)
    spec = lambda k, hh: np.linalg.eigvalsh(hamiltonian.sector_matrix(L, k, 1.0, 1.0, hh)[1].toarray())
    np.testing.assert_allclose(spec(4, h), spec(5, -h), atol=1e-12)  # global spin flip
    np.testing.assert_allclose(spec(4, h), spec(4, h[::-1].copy()), atol=1e-12)  # reflection


def test_frobenius_norm_closed_form():
    """sum lambda^2 = sum_s E(s)^2 + (J/2)^2 n 2k(L-k)/L."""
    L, k, J = 10, 5, 0.9
    h = np.random.default_rng(3).uniform(-5, 5, L)
    st, H = hamiltonian.sector_matrix(L, k, J, 1.2, h)
    w = np.linalg.eigvalsh(H.toarray())
    d = H.diagonal()
    n = len(st)
    assert abs(np.sum(w ** 2) - (np.sum(d ** 2) + (J / 2) ** 2 * n * 2 * k * (L - k) / L)) < 1e-8


def test_apply_paths_agree_with_dense():
    L, k = 12, 6
    h = np.random.default_rng(4).uniform(-8, 8, L)
    st, H = hamiltonian.sector_matrix(L, k, 1.0, 1.0, h)
    X = np.random.default_rng(5).standard_normal((len(st), 7))
    sigma = 0.37
    Hd = H.toarray()
    Y0 = Hd @ X - sigma * X
    np.testing.assert_allclose(hamiltonian.apply_shifted(H, X, sigma), Y0, atol=1e-12)
    np.testing.assert_allclose(hamiltonian.matrix_free_apply(L, st, 1.0, 1.0, h, X, sigma), Y0, atol=1e-12)
    A = (Hd - sigma * np.eye(len(st))) @ (Hd - sigma * np.eye(len(st)))
    np.testing.assert_allclose(hamiltonian.apply_fold(H, X, sigma), A @ X, atol=1e-10)


def test_row_wise_apply_matches_dense_rows_and_bound():
    """apply_rows on scattered rows (fetching X through a callback) equals the
    dense rows of H X - sigma X, and its bound is |H - sigma I| |X| row by row."""
    L, k = 12, 5
    h = np.random.default_rng(8).uniform(-3, 3, L)
    J, Delta, sigma = 0.7, 1.3, -0.4
    st, H = hamiltonian.sector_matrix(L, k, J, Delta, h)
    X = np.random.default_rng(9).standard_normal((len(st), 5))
    rows = np.array([0, 3, 17, 400, len(st) - 1])
    Y, B = hamiltonian.apply_rows(L, st, J, Delta, h, rows, sigma, lambda idx: X[idx])
    Hd = H.toarray() - sigma * np.eye(len(st))
    np.testing.assert_allclose(Y, (Hd @ X)[rows], atol=1e-12)
    np.testing.assert_allclose(B, (np.abs(Hd) @ np.abs(X))[rows], atol=1e-12)


def test_fold_diagonal_matches_dense_square_and_closed_form():
    """diag((H - sigma)^2) = (E - sigma)^2 + (J/2)^2 * (number of active bonds)."""
    L, k, J, sigma = 10, 5, 1.0, -0.8
    h = np.random.default_rng(6).uniform(-4, 4, L)
    st, H = hamiltonian.sector_matrix(L, k, J, 1.0, h)
    Hd = H.toarray() - sigma * np.eye(len(st))
    d = hamiltonian.fold_diagonal(H, sigma)
    np.testing.assert_allclose(d, np.diag(Hd @ Hd), rtol=1e-14)
    nd = np.bitwise_count((st ^ (st >> np.uint64(1))) & np.uint64((1 << (L - 1)) - 1)).astype(float)
    np.testing.assert_allclose(d, (H.diagonal() - sigma) ** 2 + (J / 2) ** 2 * nd, rtol=1e-13)


def test_trace_closed_form_in_every_sector():
    """trace(H) over the sector with k up spins, from counting k-subsets: each of
    the L-1 bonds gives n [k(k-1)/(L(L-1)) - k/L + 1/4] J Delta, each field gives
    n (k/L - 1/2) h_i.  Pins the diagonal and the assembled matrix at any k."""
    for L in (5, 8, 11):
        for k in range(L + 1):
            h = workloads.disorder(L, 2.5, 31 * L + k)
            J, D = 0.7, 1.3
            st, Hs = hamiltonian.sector_matrix(L, k, J, D, h)
            n = len(st)
            pair = k * (k - 1) / (L * (L - 1)) - k / L + 0.25
            want = J * D * (L - 1) * n * pair + n * (k / L - 0.5) * h.sum()
            assert hamiltonian.diagonal(L, st, J, D, h).sum() == pytest.approx(want, abs=1e-9)
            assert Hs.diagonal().sum() == pytest.approx(want, abs=1e-9)
