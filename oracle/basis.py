"""Fixed-S^z sector of the L-site spin-1/2 chain (paper Sec. 2.1, sector paragraph).

H commutes with total S^z, so it is block diagonal; the block with ``nup`` up
spins has dimension C(L, nup) (Table 1 prints these for nup = L/2).  The oracle
enumerates the block by brute force over all 2^L bit strings -- no
combinatorial formula is used, so it can pin one.
"""

import numpy as np

_CHUNK = 1 << 24


def nup_from_sz(L, Sz):
    """Number of up spins for magnetisation Sz (Sz = nup - L/2)."""
    two = 2.0 * Sz
    if two != round(two) or (round(two) + L) % 2 != 0 or abs(Sz) > L / 2:
        raise ValueError(f"no sector with Sz={Sz} for L={L}")
    return (round(two) + L) // 2


def enumerate_sector(L, nup):
    """All L-bit integers with exactly ``nup`` set bits, ascending (uint64).

    Brute force: scan 0 .. 2^L - 1 in chunks and keep those whose popcount is
    ``nup``.
    """
    if not (1 <= L <= 32) or not (0 <= nup <= L):
        raise ValueError("bad (L, nup)")
    out = []
    total = 1 << L
    for start in range(0, total, _CHUNK):
        s = np.arange(start, min(total, start + _CHUNK), dtype=np.uint64)
        out.append(s[np.bitwise_count(s) == nup])
    return np.concatenate(out)


def rank(states, query):
    """Row index of each query state in the ascending list, -1 if absent."""
    q = np.asarray(query, dtype=np.uint64)
    pos = np.searchsorted(states, q)
    pos_c = np.minimum(pos, len(states) - 1)
    hit = (pos < len(states)) & (states[pos_c] == q)
    return np.where(hit, pos_c.astype(np.int64), np.int64(-1))


def bits(states, L):
    """(n, L) array of site occupations b_i in {0, 1} (site i = bit i)."""
    s = np.asarray(states, dtype=np.uint64)
    return ((s[:, None] >> np.arange(L, dtype=np.uint64)[None, :]) & np.uint64(1)).astype(np.int8)
