"""Closed form of the chain at Delta = 0 (XX chain in random fields).

Jordan-Wigner maps S^z_i = n_i - 1/2 and, on an open chain, the nearest
neighbour flip-flop (S^+_i S^-_{i+1} + h.c.)/2 to the hop
(c^+_i c_{i+1} + h.c.)/2 with no string sign.  With Delta = 0 the model of
eq. (1) becomes free fermions with the L x L tridiagonal single-particle matrix

    T_ii = h_i,    T_{i,i+1} = T_{i+1,i} = J/2,

so every many-body eigenvalue in the sector with nup particles is a subset sum

    E(Q) = sum_{q in Q} eps_q - (1/2) sum_i h_i,     |Q| = nup,

and the eigenvector is the Slater determinant of the occupied orbitals:
psi(x_1 < ... < x_nup) = det[phi_q(x_a)].  Exact at any L and any disorder.
"""

import numpy as np


def single_particle(L, J, h):
    """(eps, phi) of the tridiagonal single-particle matrix, ascending."""
    h = np.asarray(h, dtype=np.float64)
    T = np.diag(h) + np.diag(np.full(L - 1, 0.5 * J), 1) + np.diag(np.full(L - 1, 0.5 * J), -1)
    return np.linalg.eigh(T)


def energies(L, nup, J, h, subsets):
    """Many-body energies for each occupation bitmask in ``subsets``.

    ``subsets`` are L-bit integers with nup set bits; bit q set means orbital q
    (ascending single-particle energy) is occupied.
    """
    eps, _ = single_particle(L, J, h)
    s = np.asarray(subsets, dtype=np.uint64)
    e = np.full(len(s), -0.5 * float(np.sum(h)))
    for q in range(L):
        e += eps[q] * ((s >> np.uint64(q)) & np.uint64(1)).astype(np.float64)
    return e


def nearest(L, nup, J, h, subsets, sigma, nev):
    """(evals ascending, occupation masks) of the nev energies nearest sigma."""
    e = energies(L, nup, J, h, subsets)
    idx = np.argsort(np.abs(e - sigma), kind="stable")[:nev]
    idx = idx[np.argsort(e[idx], kind="stable")]
    return e[idx], np.asarray(subsets, dtype=np.uint64)[idx]


def slater_vector(L, J, h, occ_mask, states):
    """Eigenvector (unit norm) for one occupation mask, on the given basis."""
    _, phi = single_particle(L, J, h)
    occ = [q for q in range(L) if (int(occ_mask) >> q) & 1]
    s = np.asarray(states, dtype=np.uint64)
    pos = np.zeros((len(s), len(occ)), dtype=np.int64)
    col = np.zeros(len(s), dtype=np.int64)
    for x in range(L):
        on = ((s >> np.uint64(x)) & np.uint64(1)).astype(bool)
        pos[on, col[on]] = x
        col[on] += 1
    M = phi[pos][:, :, occ]  # (n, nup, nup): rows = particle positions, cols = orbitals
    v = np.linalg.det(M)
    return v / np.linalg.norm(v)
