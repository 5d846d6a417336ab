"""Pins of the oracle's sector enumeration and rank lookup (paper Sec. 2.1, Table 1)."""

import math
import os

import numpy as np
import pytest

from oracle import basis

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_sector_dims.txt")


def _table1():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                L, n = line.split()
                rows.append((int(L), int(n)))
    return rows


@pytest.mark.parametrize("L,n", _table1())
def test_table1_sector_dimension(L, n):
    """Brute-force enumeration reproduces the dimensions printed in Table 1."""
    assert len(basis.enumerate_sector(L, L // 2)) == n


@pytest.mark.parametrize("L", range(1, 15))
def test_counts_are_binomial(L):
    for k in range(L + 1):
        s = basis.enumerate_sector(L, k)
        assert len(s) == math.comb(L, k)
        assert np.all(np.diff(s.astype(np.int64)) > 0)  # strictly ascending
        assert np.all(np.bitwise_count(s) == k)
        assert s.size == 0 or int(s.max()) < (1 << L)


def _colex_rank(s, L):
    """Independent closed form: rank = sum_t C(p_t, t+1), p_t = t-th set bit."""
    r, t = 0, 0
    for p in range(L):
        if (s >> p) & 1:
            t += 1
            r += math.comb(p, t)
    return r


@pytest.mark.parametrize("L", [4, 7, 10, 13])
def test_rank_matches_colex_closed_form(L):
    for k in range(L + 1):
        s = basis.enumerate_sector(L, k)
        got = basis.rank(s, s)
        want = np.array([_colex_rank(int(x), L) for x in s], dtype=np.int64)
        assert np.array_equal(got, want)
        assert np.array_equal(got, np.arange(len(s)))


def test_rank_of_non_members_is_minus_one():
    s = basis.enumerate_sector(10, 5)
    q = np.array([0, 1, 0b11111, 0b111111, (1 << 10) - 1, 1 << 11], dtype=np.uint64)
    r = basis.rank(s, q)
    assert r[2] >= 0
    assert np.all(r[[0, 1, 3, 4, 5]] == -1)


def test_flip_rank_offsets_are_binomials():
    """A flip-flop on bond (i, i+1) moves the rank by +-C(i, t), t = ups below i.

    Checked exhaustively on L = 12 from the brute-force list (the GPU kernel
    relies on this identity; here it is derived from the oracle's enumeration).
    """
    L = 12
    for k in range(1, L):
        s = basis.enumerate_sector(L, k)
        r = np.arange(len(s))
        for i in range(L - 1):
            bi = (s >> np.uint64(i)) & np.uint64(1)
            bj = (s >> np.uint64(i + 1)) & np.uint64(1)
            act = np.nonzero(bi != bj)[0]
            t = np.bitwise_count(s[act] & np.uint64((1 << i) - 1)).astype(int)
            target = basis.rank(s, s[act] ^ np.uint64(3 << i))
            sign = np.where(bi[act] == 1, 1, -1)
            comb = np.array([math.comb(i, int(x)) for x in t])
            assert np.array_equal(target - r[act], sign * comb)


def test_sz_to_nup():
    assert basis.nup_from_sz(12, 0) == 6
    assert basis.nup_from_sz(13, 0.5) == 7
    for bad in [(13, 0), (12, 0.5), (4, 3)]:
        with pytest.raises(ValueError):
            basis.nup_from_sz(*bad)


def test_bits_are_site_occupations():
    """Site i is bit i (U2): hand-written occupations of three 4-site states."""
    b = basis.bits([0b0101, 0b0011, 0b1000], 4)
    assert b.tolist() == [[1, 0, 1, 0], [1, 1, 0, 0], [0, 0, 0, 1]]
