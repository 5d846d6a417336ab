"""Jacobi-preconditioned conjugate gradient on the spectral fold (paper Sec. 3.2).

The fold A = (H - sigma I)^2 is symmetric positive (semi)definite, so LOBPCG
is preconditioned by approximately solving A w = r with diagonal (Jacobi)
preconditioned CG.  The paper fixes the iteration count per LOBPCG step (5,000
at L = 24, 20,000 at L = 26, Sec. 6) and gives no stopping rule; here the
count m is an argument.  Each column of the block is an independent CG run
(its own alpha and beta); one iteration advances every column by one step.

This is Hestenes-Stiefel preconditioned CG written out step by step, with
x_0 = 0 and M = diag(A):

    r = b, z = M^-1 r, p = z, rho = r.z
    repeat m times:
        q = A p                     (two shifted applies)
        alpha = rho / (p.q)
        x += alpha p ; r -= alpha q
        z = M^-1 r ; rho' = r.z
        p = z + (rho'/rho) p ; rho = rho'

A column stops changing (is frozen) once p.q <= 0 or rho = 0, which happens
only when it has converged exactly.
"""

import numpy as np

from . import hamiltonian


def pcg_fold(H, sigma, d, B, m):
    """Approximate A^-1 B column by column with m Jacobi-PCG steps.

    H: CSR sector matrix; d: diag(A) (``hamiltonian.fold_diagonal``);
    B: (n, b) right-hand sides.  Returns X (n, b).
    """
    B = np.asarray(B, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    n, b = B.shape
    X = np.zeros((n, b))
    R = B.copy()
    Z = R / d[:, None]
    P = Z.copy()
    rho = np.einsum("ij,ij->j", R, Z)
    live = rho > 0
    for _ in range(m):
        Q = hamiltonian.apply_fold(H, P, sigma)
        pq = np.einsum("ij,ij->j", P, Q)
        live = live & (pq > 0)
        alpha = np.where(live, rho / np.where(live, pq, 1.0), 0.0)
        X += alpha[None, :] * P
        R -= alpha[None, :] * Q
        Z = R / d[:, None]
        rho_new = np.einsum("ij,ij->j", R, Z)
        live = live & (rho_new > 0)
        beta = np.where(live, rho_new / np.where(rho > 0, rho, 1.0), 0.0)
        P = np.where(live[None, :], Z + beta[None, :] * P, P)
        rho = np.where(live, rho_new, rho)
    return X
