"""GPU parity of the two-pass (split) apply and the CG steps built on it.

The split path normally runs only on blocks that leave the caches; here
MBL_APPLY_SPLIT=1 forces it on small sectors (every chain length from 2, odd
L, S^z != 0, J and Delta != 1, ragged column panels) so that the oracle's CSR
apply and step-by-step PCG can check it element by element.  Bars as in
test_gpu_kernels.py: componentwise |dY| <= tol (|H - sigma I| |X|) with tol
1e-13 (FP64) / 2e-6 (FP32); PCG to 1e-9 of its largest entry (FP64).
"""

import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle import basis, hamiltonian, pcg as opcg
from paper_2012_00217_amd import workloads

pytestmark = pytest.mark.gpu

api = pytest.importorskip("paper_2012_00217_amd.api")
DEV = "cuda"


def _case(L, Sz=0.0, J=1.0, Delta=1.0, W=3.0, seed=0):
    h = workloads.disorder(L, W, seed)
    H = api.Hamiltonian(L, h, Sz=Sz, J=J, Delta=Delta)
    k = basis.nup_from_sz(L, Sz)
    st, Ho = hamiltonian.sector_matrix(L, k, J, Delta, h)
    return H, Ho


def _bound(Ho, X, sigma):
    return abs(Ho - sigma * sp.identity(Ho.shape[0], format="csr")) @ np.abs(X)


@pytest.fixture
def split_on(monkeypatch):
    monkeypatch.setenv("MBL_APPLY_SPLIT", "1")
    return monkeypatch


@pytest.mark.parametrize("L,Sz,J,Delta", [(2, 0.0, 1.0, 1.0), (3, 0.5, 0.7, 1.3), (5, -0.5, 1.0, 0.0),
                                          (8, 0.0, 1.3, -0.6), (11, 0.5, 0.7, -1.3),
                                          (12, 0.0, 1.0, 1.0), (13, -1.5, 2.0, 0.4),
                                          (14, 1.0, 1.0, 1.0)])
@pytest.mark.parametrize("dtype,b", [(torch.float64, 2), (torch.float64, 24), (torch.float64, 100),
                                     (torch.float32, 4), (torch.float32, 40), (torch.float32, 128)])
def test_split_apply_parity(L, Sz, J, Delta, dtype, b, split_on):
    H, Ho = _case(L, Sz, J, Delta)
    X = workloads.random_block(H.n, b, seed=L + b)
    Xo = X.astype(np.float32).astype(np.float64) if dtype == torch.float32 else X
    sigma = -0.41
    Y = H.apply(torch.from_numpy(X).to(DEV, dtype), sigma).double().cpu().numpy()
    tol = 1e-13 if dtype == torch.float64 else 2e-6
    err = np.abs(Y - hamiltonian.apply_shifted(Ho, Xo, sigma))
    assert np.all(err <= tol * _bound(Ho, Xo, sigma) + 1e-30)


@pytest.mark.parametrize("pb", [16, 32, 64, 128, 256])
@pytest.mark.parametrize("slots", [1, 3, 8])
def test_split_apply_same_under_every_panel_and_slot_count(pb, slots, split_on):
    """The per-row arithmetic of the split apply does not depend on the panel
    width or the number of workgroups, so every launch shape gives the same bits."""
    H, Ho = _case(14, W=4.0)
    X = torch.from_numpy(workloads.random_block(H.n, 72, seed=3)).to(DEV, torch.float32)
    ref = H.apply(X, 0.21)
    split_on.setenv("MBL_SPLIT_PANEL_BYTES", str(pb))
    split_on.setenv("MBL_SPLIT_SLOTS", str(slots))
    Y = H.apply(X, 0.21)
    assert torch.equal(Y, ref)


def test_split_and_one_pass_apply_agree(monkeypatch):
    """The split and one-pass kernels sum the same terms in different orders."""
    H, Ho = _case(16, W=4.0)
    X = torch.from_numpy(workloads.random_block(H.n, 64, seed=4)).to(DEV)
    monkeypatch.setenv("MBL_APPLY_SPLIT", "1")
    Ys = H.apply(X, 0.3).cpu().numpy()
    monkeypatch.setenv("MBL_APPLY_SPLIT", "0")
    Y1 = H.apply(X, 0.3).cpu().numpy()
    Xo = X.cpu().numpy()
    assert np.all(np.abs(Ys - Y1) <= 2e-13 * _bound(Ho, Xo, 0.3) + 1e-300)
    assert not np.array_equal(Ys, np.zeros_like(Ys))


def test_split_apply_strided_views(split_on):
    """ld > b (16-byte aligned: split path; odd offsets: one-pass fallback), and
    nothing is written outside the view."""
    H, Ho = _case(12, W=2.0)
    n = H.n
    X = workloads.random_block(n, 32, seed=9)
    want = hamiltonian.apply_shifted(Ho, X, 0.1)
    for off_in, off_out in [(4, 8), (3, 5)]:
        big = torch.zeros((n, 48), dtype=torch.float64, device=DEV)
        big[:, off_in:off_in + 32] = torch.from_numpy(X).to(DEV)
        out = torch.full((n, 56), 7.0, dtype=torch.float64, device=DEV)
        Y = H.apply(big[:, off_in:off_in + 32], 0.1, out=out[:, off_out:off_out + 32])
        assert np.all(np.abs(Y.cpu().numpy() - want) <= 1e-13 * _bound(Ho, X, 0.1) + 1e-300)
        o = out.cpu().numpy()
        assert np.all(o[:, :off_out] == 7.0) and np.all(o[:, off_out + 32:] == 7.0)


@pytest.mark.parametrize("L,Sz", [(12, 0.0), (11, 0.5), (14, -1.0)])
@pytest.mark.parametrize("m", [1, 2, 5])
@pytest.mark.parametrize("b", [8, 24, 40])
def test_split_pcg_parity(L, Sz, m, b, split_on):
    H, Ho = _case(L, Sz=Sz, W=4.0)
    sigma = 0.05
    R = workloads.random_block(H.n, b, seed=7 + m)
    W = H.pcg(torch.from_numpy(R).to(DEV), sigma, m).cpu().numpy()
    Wr = opcg.pcg_fold(Ho, sigma, hamiltonian.fold_diagonal(Ho, sigma), R, m)
    np.testing.assert_allclose(W, Wr, rtol=0, atol=1e-9 * np.abs(Wr).max())


def test_split_pcg_fp32_elementwise(split_on):
    """FP32 CG (the paper's precision for the preconditioner, Sec. 6) against the
    oracle's FP64 CG on the same FP32 right-hand side: every entry within 1e-4
    of its column's largest."""
    H, Ho = _case(14, W=4.0)
    sigma = 0.1
    Rd = torch.from_numpy(workloads.random_block(H.n, 32, seed=9)).to(DEV, torch.float32)
    Ro = Rd.double().cpu().numpy()
    W = H.pcg(Rd, sigma, 3).double().cpu().numpy()
    Wr = opcg.pcg_fold(Ho, sigma, hamiltonian.fold_diagonal(Ho, sigma), Ro, 3)
    assert np.all(np.abs(W - Wr) <= 1e-4 * np.abs(Wr).max(axis=0)[None, :])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_split_pcg_graph_replay_is_bitwise_identical(dtype, split_on):
    H, Ho = _case(14, W=4.0)
    R = torch.from_numpy(workloads.random_block(H.n, 32, seed=11)).to(DEV, dtype)
    split_on.setenv("MBL_PCG_GRAPH", "0")
    W_direct = H.pcg(R, 0.07, 40)
    split_on.setenv("MBL_PCG_GRAPH", "1")
    for _ in range(3):
        W_graph = H.pcg(R, 0.07, 40)
        assert torch.equal(W_direct, W_graph)
        _ = (R * 2).sum().item()  # eager work and a synchronisation between replays


def test_split_solve_dense_parity(split_on):
    """A whole interior solve with every apply and CG step on the split path."""
    L = 12
    H, Ho = _case(L, W=8.0)
    w = np.linalg.eigvalsh(Ho.toarray())
    sigma = w[0] + 0.5 * (w[-1] - w[0])
    ev, V, rs, info = H.solve(sigma, 8, 16, tol=1e-10)
    want = np.sort(w[np.argsort(np.abs(w - sigma), kind="stable")[:8]])
    assert np.abs(ev - want).max() < 1e-10
    from oracle import linalg
    assert linalg.residual_norms(Ho, ev, V.cpu().numpy()).max() <= 1e-10
