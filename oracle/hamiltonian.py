"""Sector matrix of the random-field spin chain (paper eq. (1)/(2), Sec. 2.1).

H = J sum_{i=0}^{L-2} [S^x_i S^x_{i+1} + S^y_i S^y_{i+1} + Delta S^z_i S^z_{i+1}]
    + sum_{i=0}^{L-1} h_i S^z_i,        S = sigma/2, open boundaries.

With J = Delta = 1 this is eq. (1).  In the S^z basis:

* the ZZ and field terms are diagonal: S^z_i = b_i - 1/2;
* S^x S^x + S^y S^y = (S^+ S^- + S^- S^+)/2 flips an anti-aligned pair
  (bits i and i+1 differ) and has matrix element 1/2, so J/2 in H.

The oracle writes these out literally, site by site and bond by bond, and
stores the sector matrix as scipy CSR in FP64.
"""

import numpy as np
import scipy.sparse as sp

from . import basis


def diagonal(L, states, J, Delta, h):
    """<s|H|s> for every state, literal site sums of eq. (1)."""
    b = basis.bits(states, L).astype(np.float64)
    sz = b - 0.5
    h = np.asarray(h, dtype=np.float64)
    e = np.zeros(len(states))
    for i in range(L - 1):
        e += J * Delta * sz[:, i] * sz[:, i + 1]
    for i in range(L):
        e += h[i] * sz[:, i]
    return e


def offdiagonal_triplets(L, states, J):
    """(row, col, value) of every flip-flop element, bond by bond."""
    rows, cols = [], []
    for i in range(L - 1):
        bi = (states >> np.uint64(i)) & np.uint64(1)
        bj = (states >> np.uint64(i + 1)) & np.uint64(1)
        r = np.nonzero(bi != bj)[0]
        flipped = states[r] ^ np.uint64(3 << i)
        c = basis.rank(states, flipped)
        assert np.all(c >= 0), "flip left the sector"
        rows.append(r)
        cols.append(c)
    rows = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    cols = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    vals = np.full(len(rows), 0.5 * J)
    return rows, cols, vals


def sector_matrix(L, nup, J, Delta, h, states=None):
    """(states, H) with H the n x n sector matrix as FP64 CSR."""
    if states is None:
        states = basis.enumerate_sector(L, nup)
    n = len(states)
    d = diagonal(L, states, J, Delta, h)
    r, c, v = offdiagonal_triplets(L, states, J)
    rr = np.concatenate([np.arange(n), r])
    cc = np.concatenate([np.arange(n), c])
    vv = np.concatenate([d, v])
    H = sp.csr_matrix((vv, (rr, cc)), shape=(n, n))
    H.sum_duplicates()
    return states, H


def apply_shifted(H, X, sigma):
    """Y = H X - sigma X, the shifted block apply (paper Sec. 3.2, 4.1)."""
    X = np.asarray(X, dtype=np.float64)
    return H @ X - sigma * X


def apply_fold(H, X, sigma):
    """(H - sigma I)^2 X as two shifted applies; the fold is never formed."""
    return apply_shifted(H, apply_shifted(H, X, sigma), sigma)


def fold_diagonal(H, sigma):
    """diag((H - sigma I)^2): squared 2-norm of each row of H - sigma I.

    This is the Jacobi preconditioner of the PCG inner solve (Sec. 3.2),
    computed from its definition (row norms of the shifted sector matrix).
    """
    n = H.shape[0]
    Hs = (H - sigma * sp.identity(n, format="csr")).tocsr()
    return np.asarray(Hs.multiply(Hs).sum(axis=1)).ravel()


def matrix_free_apply(L, states, J, Delta, h, X, sigma):
    """H X - sigma X without storing H: diagonal plus one gather per bond.

    Used where a CSR of the sector would not fit the host (about 600 M
    nonzeros at L = 28).  Same arithmetic as the CSR path in a different order.
    """
    X = np.asarray(X, dtype=np.float64)
    d = diagonal(L, states, J, Delta, h) - sigma
    Y = d[:, None] * X if X.ndim == 2 else d * X
    for i in range(L - 1):
        bi = (states >> np.uint64(i)) & np.uint64(1)
        bj = (states >> np.uint64(i + 1)) & np.uint64(1)
        r = np.nonzero(bi != bj)[0]
        c = basis.rank(states, states[r] ^ np.uint64(3 << i))
        Y[r] += 0.5 * J * X[c]
    return Y


def apply_rows(L, states, J, Delta, h, rows, sigma, fetch):
    """Rows ``rows`` of H X - sigma X, each from its own definition.

    For a row with state s the result is (E(s) - sigma) X[s] plus J/2 times
    X at every state reached by one flip-flop of an anti-aligned bond (eq. (1),
    Sec. 2.1).  ``fetch(idx)`` returns the rows ``idx`` of X as a 2-D array, so
    X itself may live elsewhere (a device block too large for the host).
    Returns (Y_rows, bound_rows) with bound = the same sum taken over absolute
    values, for componentwise rounding tolerances.
    """
    rows = np.asarray(rows, dtype=np.int64)
    s = states[rows]
    d = diagonal(L, s, J, Delta, h) - sigma
    Xr = np.asarray(fetch(rows), dtype=np.float64)
    Y = d[:, None] * Xr
    B = np.abs(d)[:, None] * np.abs(Xr)
    for i in range(L - 1):
        bi = (s >> np.uint64(i)) & np.uint64(1)
        bj = (s >> np.uint64(i + 1)) & np.uint64(1)
        k = np.nonzero(bi != bj)[0]
        if len(k) == 0:
            continue
        c = basis.rank(states, s[k] ^ np.uint64(3 << i))
        assert np.all(c >= 0), "flip left the sector"
        Xc = np.asarray(fetch(c), dtype=np.float64)
        Y[k] += 0.5 * J * Xc
        B[k] += 0.5 * abs(J) * np.abs(Xc)
    return Y, B
