"""GPU parity at the shapes of the benchmark configurations.

* L=20 workload (Delta=1, W in {1,2,4,8}, seed 0, sigma at energy density
  0.5, 32 pairs, block 64, FP64): every pair's residual recomputed by the
  oracle's FP64 CSR apply <= 1e-10.  Completeness of "the 32 nearest" cannot
  be checked by dense or shift-invert diagonalisation at this size here
  (shift-invert at L = 18 already takes minutes), so it is pinned indirectly:
  a solve with block 128 must return the same 32 eigenvalues (parity
  unpinned beyond that).
* Batched workload: a stratified sample of its problems, one per (L, W) of
  the recipe (L = 14, 16, 18; W = 2, 4, 6, 8), 16 pairs, block 32, FP64,
  solved through the batch entry point: dense-oracle eigenvalues for L <= 16,
  CPU residuals and the block-64 agreement for L = 18, bitwise equality with
  the single-solve path.
* L=24 workload's FP32 block Jacobi-PCG (128 columns): every entry against the
  oracle's FP64 PCG on the same FP32 right-hand side.
"""

import numpy as np
import pytest
import torch

from oracle import hamiltonian, linalg, pcg as opcg, spectrum
from paper_2012_00217_amd import workloads

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_2012_00217_amd.api")


@pytest.mark.parametrize("W", [1.0, 2.0, 4.0, 8.0])
def test_l20_workload_residuals_and_block_agreement(W):
    L, nev, b = 20, 32, 64
    h = workloads.disorder(L, W, 0)
    st, Ho = hamiltonian.sector_matrix(L, L // 2, 1.0, 1.0, h)
    lo, hi = spectrum.bounds(Ho)
    sigma = spectrum.shift_from_density(lo, hi, 0.5)
    H = api.Hamiltonian(L, h)
    ev, V, rs, info = H.solve(sigma, nev, b, tol=1e-10)
    assert info["status"] == "MBL_OK"
    r_cpu = linalg.residual_norms(Ho, ev, V.cpu().numpy())
    assert np.all(r_cpu <= 1e-10), r_cpu.max()
    assert np.all(np.abs(rs - r_cpu) <= 1e-12)
    assert np.all(np.diff(ev) > 0)  # ascending, distinct
    # completeness, indirectly: a block twice as wide finds the same 32
    ev2, V2, rs2, info2 = H.solve(sigma, nev, 2 * b, tol=1e-10, want_vectors=False)
    assert np.abs(ev2 - ev).max() <= 1e-10


def _stratified():
    probs, seen = [], set()
    for p in workloads.batch_problems(64):
        key = (p["L"], p["W"])
        if key in seen:
            continue
        seen.add(key)
        probs.append({"L": p["L"], "h": p["h"], "eps": 0.5, "nev": 16, "block": 32,
                      "tol": 1e-10, "precision": "f64", "seed": 7})
    assert len(probs) == 12
    return probs


def test_batched_workload_stratified_sample():
    probs = _stratified()
    res = api.batch_solve(probs, concurrency=4, vectors=True)
    for d, r in zip(probs, res):
        assert r["status"] == "MBL_OK", (d["L"], r)
        L = d["L"]
        st, Ho = hamiltonian.sector_matrix(L, L // 2, 1.0, 1.0, d["h"])
        Vn = r["evecs"].cpu().numpy()
        assert np.max(linalg.residual_norms(Ho, r["evals"], Vn)) <= 1e-10
        H = api.Hamiltonian(L, d["h"])
        ev, V, rs, info = H.solve(r["sigma"], d["nev"], d["block"], tol=d["tol"], seed=d["seed"])
        assert np.array_equal(ev, r["evals"])  # alone = in the batch, bitwise
        if L <= 16:
            w_ref, _ = spectrum.nearest(Ho, r["sigma"], d["nev"])
            assert np.max(np.abs(r["evals"] - w_ref)) <= 1e-10
        else:
            ev2, _, _, _ = H.solve(r["sigma"], d["nev"], 2 * d["block"], tol=d["tol"],
                                   want_vectors=False)
            assert np.max(np.abs(ev2 - r["evals"])) <= 1e-10
        H.close()


def test_l24_fp32_pcg_elementwise():
    """Two CG steps of the L=24 workload's preconditioner (FP32, 128 columns,
    the solver's launch configuration): every entry within 1e-4 of its
    column's largest against the oracle's FP64 step-by-step PCG."""
    L, b, m = 24, 128, 2
    h = workloads.disorder(L, 4.0, 0)
    st, Ho = hamiltonian.sector_matrix(L, L // 2, 1.0, 1.0, h)
    H = api.Hamiltonian(L, h)
    sigma = -0.37
    R = torch.from_numpy(workloads.random_block(H.n, b, seed=L)).to("cuda", torch.float32)
    Ro = R.double().cpu().numpy()
    W = H.pcg(R, sigma, m).double().cpu().numpy()
    del R
    torch.cuda.empty_cache()
    Wr = opcg.pcg_fold(Ho, sigma, hamiltonian.fold_diagonal(Ho, sigma), Ro, m)
    err = np.abs(W - Wr) / np.abs(Wr).max(axis=0)[None, :]
    assert err.max() <= 1e-4, err.max()
