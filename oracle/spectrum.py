"""Eigenpairs of the sector matrix nearest a shift (paper Sec. 3.2).

LOBPCG on the spectral fold (H - sigma I)^2 converges to the eigenvectors of
the fold's smallest eigenvalues, i.e. the eigenpairs of H whose eigenvalues are
nearest sigma.  The oracle computes that definition directly:

* dense ``numpy.linalg.eigh`` (LAPACK) for small sectors;
* shift-invert Lanczos (``scipy.sparse.linalg.eigsh`` with ``sigma``, SuperLU),
  the traditional method the paper contrasts with (Sec. 1), for larger ones.

Result convention: the nev pairs with smallest |lambda - sigma|, returned in
ascending lambda, unit 2-norm vectors.
"""

import numpy as np
import scipy.sparse.linalg as sla

DENSE_MAX = 5000


def _select_nearest(w, V, sigma, nev):
    idx = np.argsort(np.abs(w - sigma), kind="stable")[:nev]
    idx = idx[np.argsort(w[idx], kind="stable")]
    V = V[:, idx]
    V = V / np.linalg.norm(V, axis=0)
    return w[idx], V


def dense_eigh(H):
    """All eigenpairs of the (small) sector matrix, ascending."""
    A = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    return np.linalg.eigh(A)


def nearest(H, sigma, nev, extra=8):
    """(evals, evecs) of the nev eigenpairs nearest sigma."""
    n = H.shape[0]
    if n <= DENSE_MAX:
        w, V = dense_eigh(H)
        return _select_nearest(w, V, sigma, nev)
    k = min(n - 2, nev + extra)
    w, V = sla.eigsh(H.tocsc(), k=k, sigma=sigma, which="LM", tol=1e-14)
    return _select_nearest(w, V, sigma, nev)


def bounds(H):
    """(Emin, Emax) of the sector matrix."""
    n = H.shape[0]
    if n <= DENSE_MAX:
        w = np.linalg.eigvalsh(H.toarray())
        return float(w[0]), float(w[-1])
    lo = sla.eigsh(H, k=1, which="SA", tol=1e-14, ncv=64)[0][0]
    hi = sla.eigsh(H, k=1, which="LA", tol=1e-14, ncv=64)[0][0]
    return float(lo), float(hi)


def shift_from_density(emin, emax, eps):
    """sigma at energy density eps: Emin + eps (Emax - Emin)."""
    return emin + eps * (emax - emin)
