"""MBL observables of eigenpairs (paper Sec. 2.2): adjacent gap ratio and
bipartite entanglement entropy.

* Adjacent gap ratio of an ascending list of eigenvalues:
  r_n = min(d_n, d_{n+1}) / max(d_n, d_{n+1}),  d_n = E_{n+1} - E_n.
* Entanglement entropy of a sector eigenvector across the cut between sites
  l-1 and l: write the state in the full 2^L space, reshape to the
  (right part) x (left part) matrix, take its singular values s_i and
  S = -sum_i s_i^2 ln s_i^2 (natural log).  Sites 0..l-1 are the left part
  (bits 0..l-1 of the state).
"""

import numpy as np


def gap_ratios(evals):
    e = np.sort(np.asarray(evals, dtype=np.float64))
    d = np.diff(e)
    a, b = d[:-1], d[1:]
    with np.errstate(invalid="ignore", divide="ignore"):
        r = np.minimum(a, b) / np.maximum(a, b)
    return r


def entanglement_entropy(psi, states, L, cut):
    """Von Neumann entropy (natural log) of a unit vector on the sector basis."""
    full = np.zeros(1 << L)
    full[np.asarray(states, dtype=np.int64)] = np.asarray(psi, dtype=np.float64)
    M = full.reshape(1 << (L - cut), 1 << cut)  # [high bits][low bits]
    s = np.linalg.svd(M, compute_uv=False)
    p = s ** 2
    p = p[p > 1e-300]
    return float(-np.sum(p * np.log(p)))
