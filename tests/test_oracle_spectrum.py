"""Pins of the oracle's nearest-eigenpair solver, free-fermion closed form, PCG
and dense block tools."""

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import basis, hamiltonian, spectrum, freefermion, pcg, linalg


def test_dense_and_shift_invert_agree(monkeypatch):
    L, k = 14, 7
    h = np.random.default_rng(0).uniform(-4, 4, L)
    _, H = hamiltonian.sector_matrix(L, k, 1.0, 1.0, h)
    emin, emax = spectrum.bounds(H)
    sigma = spectrum.shift_from_density(emin, emax, 0.5)
    w_d, V_d = spectrum.nearest(H, sigma, 10)
    monkeypatch.setattr(spectrum, "DENSE_MAX", 100)
    w_s, V_s = spectrum.nearest(H, sigma, 10)
    np.testing.assert_allclose(w_s, w_d, atol=1e-11)
    assert linalg.max_cluster_angle(w_d, V_d, V_s, 1e-8) < 1e-7
    assert np.all(linalg.residual_norms(H, w_s, V_s) < 1e-11)


def test_nearest_picks_by_distance_and_sorts_ascending():
    L, k = 10, 5
    h = np.random.default_rng(1).uniform(-2, 2, L)
    _, H = hamiltonian.sector_matrix(L, k, 1.0, 1.0, h)
    w_all = np.linalg.eigvalsh(H.toarray())
    sigma = 0.1
    w, V = spectrum.nearest(H, sigma, 6)
    assert np.all(np.diff(w) > 0)
    far = np.max(np.abs(w - sigma))
    outside = np.setdiff1d(np.round(w_all, 12), np.round(w, 12))
    assert np.all(np.abs(outside - sigma) >= far - 1e-12)
    np.testing.assert_allclose(np.linalg.norm(V, axis=0), 1.0, atol=1e-14)
    np.testing.assert_allclose(np.sum(w_all), H.diagonal().sum(), atol=1e-10)  # trace


@pytest.mark.parametrize("L", [12, 16])
def test_nearest_matches_free_fermions(L):
    """Delta = 0 at energy density 0.5: oracle eigenvalues equal subset sums."""
    k = L // 2
    h = np.random.default_rng(L).uniform(-3, 3, L)
    st, H = hamiltonian.sector_matrix(L, k, 1.0, 0.0, h)
    e_all = freefermion.energies(L, k, 1.0, h, st)
    sigma = spectrum.shift_from_density(e_all.min(), e_all.max(), 0.5)
    nev = 12
    w, V = spectrum.nearest(H, sigma, nev)
    e, _ = freefermion.nearest(L, k, 1.0, h, st, sigma, nev)
    np.testing.assert_allclose(w, e, atol=1e-10)
    lo, hi = spectrum.bounds(H)
    np.testing.assert_allclose([lo, hi], [e_all.min(), e_all.max()], atol=1e-10)


def test_slater_determinants_are_the_eigenvectors():
    L, k = 10, 5
    h = np.random.default_rng(7).uniform(-3, 3, L)
    st, H = hamiltonian.sector_matrix(L, k, 1.0, 0.0, h)
    e, masks = freefermion.nearest(L, k, 1.0, h, st, 0.2, 6)
    w, V = spectrum.nearest(H, 0.2, 6)
    np.testing.assert_allclose(w, e, atol=1e-12)
    for j, m in enumerate(masks):
        v = freefermion.slater_vector(L, 1.0, h, m, st)
        assert np.linalg.norm(H @ v - e[j] * v) < 1e-12
        if (j == 0 or w[j] - w[j - 1] > 1e-6) and (j == len(w) - 1 or w[j + 1] - w[j] > 1e-6):
            assert abs(abs(v @ V[:, j]) - 1.0) < 1e-10


def _fold_problem(L=8, k=4, seed=0, sigma=None):
    h = np.random.default_rng(seed).uniform(-2, 2, L)
    st, H = hamiltonian.sector_matrix(L, k, 1.0, 1.0, h)
    if sigma is None:
        sigma = spectrum.bounds(H)[0] - 0.5
    d = hamiltonian.fold_diagonal(H, sigma)
    return H, sigma, d


@pytest.mark.parametrize("m", [1, 2, 4, 6])
def test_pcg_iterate_is_krylov_optimal(m):
    """CG's m-th iterate minimises the A-norm error over the preconditioned
    Krylov space span{z, (M^-1 A) z, ..., (M^-1 A)^{m-1} z}, z = M^-1 b."""
    H, sigma, d = _fold_problem(sigma=0.05)
    n = H.shape[0]
    B = np.random.default_rng(1).standard_normal((n, 3))
    X = pcg.pcg_fold(H, sigma, d, B, m)
    Hd = H.toarray() - sigma * np.eye(n)
    A = Hd @ Hd
    for j in range(B.shape[1]):
        K = [B[:, j] / d]
        for _ in range(m - 1):
            K.append((A @ K[-1]) / d)
        Q, _ = np.linalg.qr(np.array(K).T)
        y = np.linalg.solve(Q.T @ A @ Q, Q.T @ B[:, j])
        xs = Q @ y
        assert np.linalg.norm(X[:, j] - xs) <= 1e-8 * np.linalg.norm(xs)


def test_pcg_one_step_closed_form():
    H, sigma, d = _fold_problem(seed=3)
    b = np.random.default_rng(2).standard_normal((H.shape[0], 1))
    z = b[:, 0] / d
    Az = hamiltonian.apply_fold(H, z[:, None], sigma)[:, 0]
    x1 = (b[:, 0] @ z) / (z @ Az) * z
    np.testing.assert_allclose(pcg.pcg_fold(H, sigma, d, b, 1)[:, 0], x1, rtol=1e-13)


def test_pcg_solves_small_system():
    H, sigma, d = _fold_problem(L=6, k=3, seed=4)
    n = H.shape[0]
    B = np.random.default_rng(3).standard_normal((n, 2))
    X = pcg.pcg_fold(H, sigma, d, B, 3 * n)
    Hd = H.toarray() - sigma * np.eye(n)
    np.testing.assert_allclose(X, np.linalg.solve(Hd @ Hd, B), rtol=1e-8, atol=1e-10)


def test_cholqr_and_angles():
    S = np.random.default_rng(9).standard_normal((200, 12))
    Q, R = linalg.cholqr(S)
    np.testing.assert_allclose(Q.T @ Q, np.eye(12), atol=1e-13)
    np.testing.assert_allclose(Q @ R, S, atol=1e-12)
    assert np.allclose(R, np.triu(R)) and np.all(np.diag(R) > 0)
    Qn, Rn = np.linalg.qr(S)
    sgn = np.sign(np.diag(Rn))
    np.testing.assert_allclose(R, sgn[:, None] * Rn, atol=1e-12)
    G = linalg.gram(S)
    np.testing.assert_allclose(G, S.T @ S)
    ev = np.array([0.0, 1.0, 1.0 + 1e-12, 2.0])
    U = np.linalg.qr(np.random.default_rng(1).standard_normal((30, 4)))[0]
    rot = np.eye(4)
    c, s = np.cos(0.7), np.sin(0.7)
    rot[1:3, 1:3] = [[c, -s], [s, c]]
    assert linalg.max_cluster_angle(ev, U, U @ rot, 1e-8) < 1e-7
    V = U.copy()
    V[:, 3] = sla.null_space(U.T)[:, 0]
    assert abs(linalg.max_cluster_angle(ev, U, V, 1e-8) - np.pi / 2) < 1e-7


def test_clusters_group_near_degenerate_levels():
    """Neighbouring eigenvalues closer than tol share a cluster; others do not."""
    ev = np.array([0.0, 1e-12, 1.0, 2.0, 2.0 + 5e-10, 2.0 + 1e-9, 3.0])
    assert linalg.clusters(ev, 1e-9) == [[0, 1], [2], [3, 4, 5], [6]]
    assert linalg.clusters(ev, 1e-13) == [[0], [1], [2], [3], [4], [5], [6]]


def test_residual_norms_known_answers():
    """The checker behind every 'residual <= tol' claim, against residuals
    fixed by construction: an exact eigenpair with lambda shifted by delta
    scores |delta|; a rescaled column scores as its unit vector; a vector
    tilted by angle t off an eigenvector u towards another w scores
    sin t |lambda_w - lambda_u| at lambda_u and sin t cos t |lambda_w - lambda_u|
    at its Rayleigh quotient; nev < n and nev = n shapes; a random vector is
    far from any eigenvector."""
    L, k = 10, 5
    h = np.random.default_rng(5).uniform(-3, 3, L)
    _, H = hamiltonian.sector_matrix(L, k, 1.0, 1.0, h)
    w, V = np.linalg.eigh(H.toarray())
    n = len(w)
    # exact pairs: residual at rounding level, for nev = n and nev = 3
    assert linalg.residual_norms(H, w, V).max() < 1e-12
    assert linalg.residual_norms(H, w[[0, 7, n - 1]], V[:, [0, 7, n - 1]]).shape == (3,)
    # shifted eigenvalues score exactly the shift
    deltas = np.array([1e-3, -2.5e-6, 0.75])
    cols = [3, 40, 200]
    r = linalg.residual_norms(H, w[cols] + deltas, V[:, cols])
    np.testing.assert_allclose(r, np.abs(deltas), rtol=1e-9)
    # non-unit columns are normalised first
    r2 = linalg.residual_norms(H, w[cols] + deltas, V[:, cols] * np.array([3.0, 1e-4, -7.0]))
    np.testing.assert_allclose(r2, r, rtol=1e-9)
    # a vector tilted between two eigenvectors
    u, v2 = 10, 11
    t = 0.2
    x = np.cos(t) * V[:, u] + np.sin(t) * V[:, v2]
    gap = abs(w[v2] - w[u])
    want = np.sin(t) * gap  # at lambda_u only the w-part leaves a residual
    np.testing.assert_allclose(linalg.residual_norms(H, [w[u]], x[:, None]), [want], rtol=1e-9)
    rq = np.cos(t) ** 2 * w[u] + np.sin(t) ** 2 * w[v2]
    np.testing.assert_allclose(linalg.residual_norms(H, [rq], x[:, None]),
                               [np.sin(t) * np.cos(t) * gap], rtol=1e-9)
    # a random vector is not an eigenvector
    rnd = np.random.default_rng(0).standard_normal(n)
    assert linalg.residual_norms(H, [0.0], rnd[:, None])[0] > 0.1
