"""End-to-end parity of the interior eigensolver against the FP64 oracle.

Bars (per the target): eigenvalues within 1e-10 of the oracle, residual
||H x - lambda x||_2 <= 1e-10 recomputed on the CPU in FP64, and per-cluster
subspace angle <= max(1e-8, 2 (r_gpu + r_oracle) / gap).
"""

import numpy as np
import pytest
import torch

from oracle import basis, hamiltonian, spectrum, freefermion, linalg
from paper_2012_00217_amd import workloads

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_2012_00217_amd.api")


def _angle_bound(w, r_gpu, r_ora):
    """Davis-Kahan style allowance per pair: 2 (r_gpu + r_oracle) / gap."""
    gaps = np.diff(w)
    left = np.concatenate([[np.inf], gaps])
    right = np.concatenate([gaps, [np.inf]])
    gap = np.minimum(left, right)
    return np.maximum(1e-8, 2 * (r_gpu + r_ora) / gap)


def _check(Ho, sigma, nev, ev, V, rs, w_ref, V_ref, tol=1e-10):
    Vn = V.cpu().numpy()
    r_cpu = linalg.residual_norms(Ho, ev, Vn)
    assert np.all(r_cpu <= tol), r_cpu
    assert np.all(np.abs(ev - w_ref) <= 1e-10), np.abs(ev - w_ref).max()
    if V_ref is not None:
        r_ref = linalg.residual_norms(Ho, w_ref, V_ref)
        bound = _angle_bound(w_ref, r_cpu, r_ref)
        for j in range(nev):
            ang = linalg.max_cluster_angle(w_ref[[j]], Vn[:, [j]], V_ref[:, [j]], 0.0)
            assert ang <= bound[j], (j, ang, bound[j])


@pytest.mark.parametrize("precision", ["f64", "pcg32", "mixed"])
def test_cfg1_l12_dense_parity(precision):
    """L=12, S^z=0, W=8, seed 0, sigma at energy density 0.5, nev 8, block 16."""
    L, W, nev, b = 12, 8.0, 8, 16
    h = workloads.disorder(L, W, 0)
    st, Ho = hamiltonian.sector_matrix(L, L // 2, 1.0, 1.0, h)
    emin, emax = spectrum.bounds(Ho)
    sigma = spectrum.shift_from_density(emin, emax, 0.5)
    w_ref, V_ref = spectrum.nearest(Ho, sigma, nev)
    H = api.Hamiltonian(L, h)
    ev, V, rs, info = H.solve(sigma, nev, b, tol=1e-10, precision=precision)
    assert info["status"] == "MBL_OK"
    assert np.all(rs <= 1e-10)
    _check(Ho, sigma, nev, ev, V, rs, w_ref, V_ref)


@pytest.mark.parametrize("precision", ["f64", "mixed"])
@pytest.mark.parametrize("L,Sz,J,Delta,eps", [(13, 0.5, 0.8, 1.7, 0.3), (14, -1.0, 1.2, 0.5, 0.7)])
def test_other_sectors_and_couplings_dense_parity(L, Sz, J, Delta, eps, precision):
    """Odd L, S^z != 0, J != 1 and Delta != 1 through the whole solver."""
    nev, b = 6, 12
    h = workloads.disorder(L, 5.0, 3)
    k = basis.nup_from_sz(L, Sz)
    st, Ho = hamiltonian.sector_matrix(L, k, J, Delta, h)
    emin, emax = spectrum.bounds(Ho)
    sigma = spectrum.shift_from_density(emin, emax, eps)
    w_ref, V_ref = spectrum.nearest(Ho, sigma, nev)
    H = api.Hamiltonian(L, h, Sz=Sz, J=J, Delta=Delta)
    assert H.n == len(st)
    glo, ghi = H.spectrum_bounds(1e-12)
    assert abs(glo - emin) < 1e-10 and abs(ghi - emax) < 1e-10
    ev, V, rs, info = H.solve(sigma, nev, b, tol=1e-10, precision=precision)
    assert info["status"] == "MBL_OK"
    _check(Ho, sigma, nev, ev, V, rs, w_ref, V_ref)


def test_spectrum_bounds_give_same_sigma():
    L = 12
    h = workloads.disorder(L, 8.0, 0)
    st, Ho = hamiltonian.sector_matrix(L, L // 2, 1.0, 1.0, h)
    lo, hi = spectrum.bounds(Ho)
    H = api.Hamiltonian(L, h)
    glo, ghi = H.spectrum_bounds(1e-12)
    assert abs(glo - lo) < 1e-10 and abs(ghi - hi) < 1e-10


@pytest.mark.parametrize("L", [14, 16])
def test_delta_zero_free_fermions(L):
    """Delta = 0: exact eigenvalues from single-particle subset sums."""
    nev, b = 12, 24
    h = workloads.disorder(L, 3.0, 1)
    st = basis.enumerate_sector(L, L // 2)
    e_all = freefermion.energies(L, L // 2, 1.0, h, st)
    sigma = spectrum.shift_from_density(e_all.min(), e_all.max(), 0.5)
    e_ref, _ = freefermion.nearest(L, L // 2, 1.0, h, st, sigma, nev)
    H = api.Hamiltonian(L, h, Delta=0.0)
    ev, V, rs, info = H.solve(sigma, nev, b, tol=1e-10)
    _, Ho = hamiltonian.sector_matrix(L, L // 2, 1.0, 0.0, h, states=st)
    assert np.all(linalg.residual_norms(Ho, ev, V.cpu().numpy()) <= 1e-10)
    np.testing.assert_allclose(ev, e_ref, atol=1e-10)


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_delta_zero_twin_of_the_l20_workload(precision):
    """The L = 20 workload (n = 184756, 32 pairs, block 64, tol 1e-10) at Delta = 0,
    where the exact eigenvalues are single-particle subset sums at full size."""
    L, nev, b = 20, 32, 64
    h = workloads.disorder(L, 4.0, 0)
    st = basis.enumerate_sector(L, L // 2)
    e_all = freefermion.energies(L, L // 2, 1.0, h, st)
    sigma = spectrum.shift_from_density(e_all.min(), e_all.max(), 0.5)
    e_ref, _ = freefermion.nearest(L, L // 2, 1.0, h, st, sigma, nev)
    H = api.Hamiltonian(L, h, Delta=0.0)
    ev, V, rs, info = H.solve(sigma, nev, b, tol=1e-10, precision=precision)
    _, Ho = hamiltonian.sector_matrix(L, L // 2, 1.0, 0.0, h, states=st)
    assert np.all(linalg.residual_norms(Ho, ev, V.cpu().numpy()) <= 1e-10)
    np.testing.assert_allclose(ev, e_ref, atol=1e-10)


def test_solve_is_deterministic():
    L = 12
    h = workloads.disorder(L, 4.0, 2)
    H = api.Hamiltonian(L, h)
    a = H.solve(0.1, 4, 8, tol=1e-10)
    b = H.solve(0.1, 4, 8, tol=1e-10)
    assert np.array_equal(a[0], b[0]) and torch.equal(a[1], b[1])


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_soft_locking_dense_parity(precision):
    """Soft locking (opts.lock): the same pairs as dense diagonalisation, and the
    inner CG ran on fewer columns than block x steps once pairs locked; without
    the option every CG step covers the whole block."""
    L, nev, b = 14, 32, 48
    h = workloads.disorder(L, 4.0, 0)
    st, Ho = hamiltonian.sector_matrix(L, L // 2, 1.0, 1.0, h)
    emin, emax = spectrum.bounds(Ho)
    sigma = spectrum.shift_from_density(emin, emax, 0.5)
    w_ref, V_ref = spectrum.nearest(Ho, sigma, nev)
    H = api.Hamiltonian(L, h)
    ev, V, rs, info = H.solve(sigma, nev, b, tol=1e-10, precision=precision, lock=True)
    assert info["status"] == "MBL_OK"
    _check(Ho, sigma, nev, ev, V, rs, w_ref, V_ref)
    assert info["pcg_columns"] < info["pcg_steps"] * b, info
    ev0, V0, rs0, info0 = H.solve(sigma, nev, b, tol=1e-10, precision=precision)
    assert info0["pcg_columns"] == info0["pcg_steps"] * b
    _check(Ho, sigma, nev, ev0, V0, rs0, w_ref, V_ref)


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_soft_locking_with_guard_columns(precision):
    """Soft locking together with guard columns that run a quarter of the CG
    steps: the locked path puts the unlocked wanted pairs first so that only
    the rest stop early.  The same pairs as dense diagonalisation, and fewer
    CG column-steps than with locking alone."""
    L, nev, b = 14, 32, 96
    h = workloads.disorder(L, 4.0, 0)
    st, Ho = hamiltonian.sector_matrix(L, L // 2, 1.0, 1.0, h)
    emin, emax = spectrum.bounds(Ho)
    sigma = spectrum.shift_from_density(emin, emax, 0.5)
    w_ref, V_ref = spectrum.nearest(Ho, sigma, nev)
    H = api.Hamiltonian(L, h)
    ev, V, rs, info = H.solve(sigma, nev, b, tol=1e-10, precision=precision, lock=True,
                              guard_cg=0.25)
    assert info["status"] == "MBL_OK"
    _check(Ho, sigma, nev, ev, V, rs, w_ref, V_ref)
    ev1, V1, rs1, info1 = H.solve(sigma, nev, b, tol=1e-10, precision=precision, lock=True,
                                  guard_cg=1.0)
    _check(Ho, sigma, nev, ev1, V1, rs1, w_ref, V_ref)
    per_step = info["pcg_columns"] / info["pcg_steps"]
    assert per_step < info1["pcg_columns"] / info1["pcg_steps"], (info, info1)


def test_soft_locking_delta_zero_l18():
    """Soft locking on a larger sector (L = 18, n = 48620, 32 pairs, block 48) at
    Delta = 0, against the exact single-particle subset sums.  Short inner
    solves (60 CG steps) spread the pairs' convergence over many outer
    iterations, so pairs lock well before the last one converges."""
    L, nev, b = 18, 32, 48
    h = workloads.disorder(L, 4.0, 0)
    st = basis.enumerate_sector(L, L // 2)
    e_all = freefermion.energies(L, L // 2, 1.0, h, st)
    sigma = spectrum.shift_from_density(e_all.min(), e_all.max(), 0.5)
    e_ref, _ = freefermion.nearest(L, L // 2, 1.0, h, st, sigma, nev)
    H = api.Hamiltonian(L, h, Delta=0.0)
    ev, V, rs, info = H.solve(sigma, nev, b, tol=1e-10, lock=True, pcg_iters=60)
    assert info["status"] == "MBL_OK"
    _, Ho = hamiltonian.sector_matrix(L, L // 2, 1.0, 0.0, h, states=st)
    assert np.all(linalg.residual_norms(Ho, ev, V.cpu().numpy()) <= 1e-10)
    np.testing.assert_allclose(ev, e_ref, atol=1e-10)
    assert info["pcg_columns"] < info["pcg_steps"] * b, info
