"""Pins of the oracle's MBL observables (paper Sec. 2.2)."""

import math

import numpy as np
import pytest

from oracle import basis, hamiltonian, spectrum, freefermion, observables


def test_gap_ratio_definition_and_limits():
    r = observables.gap_ratios([0.0, 1.0, 3.0, 3.5])
    np.testing.assert_allclose(r, [0.5, 0.25])
    # equally spaced levels: r = 1
    assert np.all(observables.gap_ratios(np.arange(10.0)) == 1.0)
    # Poisson levels: <r> = 2 ln 2 - 1
    rng = np.random.default_rng(0)
    e = np.cumsum(rng.exponential(1.0, 200000))
    assert abs(np.mean(observables.gap_ratios(e)) - (2 * math.log(2) - 1)) < 3e-3


def test_entropy_of_product_state_and_singlet():
    L, k = 6, 3
    st = basis.enumerate_sector(L, k)
    psi = np.zeros(len(st))
    psi[3] = 1.0  # a basis state is a product state
    assert observables.entanglement_entropy(psi, st, L, 3) == pytest.approx(0.0, abs=1e-14)
    # (|up down> - |down up>)/sqrt2 on sites 2,3 (across the cut at 3), others fixed
    a = (1 << 0) | (1 << 2) | (1 << 4)   # sites 0,2,4 up
    b = (1 << 0) | (1 << 3) | (1 << 4)   # sites 0,3,4 up
    psi = np.zeros(len(st))
    psi[basis.rank(st, [a])[0]] = 1 / math.sqrt(2)
    psi[basis.rank(st, [b])[0]] = -1 / math.sqrt(2)
    assert observables.entanglement_entropy(psi, st, L, 3) == pytest.approx(math.log(2), abs=1e-14)


@pytest.mark.parametrize("L,cut", [(10, 5), (10, 3), (12, 6)])
def test_entropy_matches_free_fermion_correlation_matrix(L, cut):
    """Delta = 0 eigenstates are Slater determinants: S = -sum c ln c + (1-c) ln(1-c)
    over the eigenvalues c of the single-particle correlation matrix restricted
    to the left part (Peschel's formula)."""
    k = L // 2
    h = np.random.default_rng(L + cut).uniform(-2, 2, L)
    st = basis.enumerate_sector(L, k)
    eps, phi = freefermion.single_particle(L, 1.0, h)
    _, masks = freefermion.nearest(L, k, 1.0, h, st, 0.1, 3)
    for m in masks:
        psi = freefermion.slater_vector(L, 1.0, h, m, st)
        occ = [q for q in range(L) if (int(m) >> q) & 1]
        Cm = phi[:cut, occ] @ phi[:cut, occ].T
        c = np.clip(np.linalg.eigvalsh(Cm), 1e-300, 1 - 1e-16)
        want = -np.sum(c * np.log(c) + (1 - c) * np.log1p(-c))
        assert observables.entanglement_entropy(psi, st, L, cut) == pytest.approx(want, abs=1e-10)
