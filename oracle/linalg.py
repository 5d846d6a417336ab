"""Dense block tools: Gram products, Cholesky-QR, residuals, subspace angles.

LOBPCG is a block method whose dense work is tall-skinny products and small
dense factorisations (paper Sec. 3.2, property (ii)).  The oracle's versions are
plain numpy/scipy calls so that a reader can check them by eye.
"""

import numpy as np
import scipy.linalg as sla


def gram(S, T=None):
    """S^T T (S^T S when T is None), FP64."""
    S = np.asarray(S, dtype=np.float64)
    T = S if T is None else np.asarray(T, dtype=np.float64)
    return S.T @ T


def cholqr(S):
    """(Q, R) with S = Q R, R upper triangular from Cholesky of S^T S."""
    G = gram(S)
    R = np.linalg.cholesky(G).T
    Q = sla.solve_triangular(R, np.asarray(S, dtype=np.float64).T, trans="T", lower=False).T
    return Q, R


def residual_norms(H, evals, V):
    """||H v_j - lambda_j v_j||_2 for unit-normalised columns of V."""
    V = np.asarray(V, dtype=np.float64)
    V = V / np.linalg.norm(V, axis=0)
    R = H @ V - V * np.asarray(evals)[None, :]
    return np.linalg.norm(R, axis=0)


def clusters(evals, tol):
    """Group ascending eigenvalues whose neighbouring gaps are below tol."""
    groups, cur = [], [0]
    for j in range(1, len(evals)):
        if evals[j] - evals[j - 1] < tol:
            cur.append(j)
        else:
            groups.append(cur)
            cur = [j]
    groups.append(cur)
    return groups


def max_cluster_angle(evals, U, V, tol):
    """Largest principal angle between span(U[:, c]) and span(V[:, c]) over
    clusters c of ``evals`` (eigenvectors are defined only up to rotations
    inside a cluster of nearly equal eigenvalues)."""
    worst = 0.0
    for c in clusters(np.asarray(evals), tol):
        ang = sla.subspace_angles(np.asarray(U)[:, c], np.asarray(V)[:, c])
        worst = max(worst, float(np.max(ang)))
    return worst
