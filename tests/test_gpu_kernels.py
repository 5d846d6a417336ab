"""GPU parity of the hot-path kernels against the FP64 CPU oracle.

Bars: bit-exact for enumeration and rank; componentwise
|dY| <= tol * (|H - sigma I| |X|) for the applies (FP64 tol 1e-13, FP32 2e-6);
PCG, Gram, combine and the small eigensolver against the oracle's step-by-step
or numpy definitions.
"""

import math

import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle import basis, hamiltonian, pcg as opcg
from paper_2012_00217_amd import workloads

pytestmark = pytest.mark.gpu

api = pytest.importorskip("paper_2012_00217_amd.api")
DEV = "cuda"


def _ham(L, W=8.0, seed=0, Sz=0.0, J=1.0, Delta=1.0):
    h = workloads.disorder(L, W, seed)
    return h, api.Hamiltonian(L, h, Sz=Sz, J=J, Delta=Delta)


def _oracle(L, h, Sz=0.0, J=1.0, Delta=1.0):
    k = basis.nup_from_sz(L, Sz)
    return hamiltonian.sector_matrix(L, k, J, Delta, h)


def _abs_bound(H, X, sigma):
    Habs = abs(H - sigma * sp.identity(H.shape[0], format="csr"))
    return Habs @ np.abs(X)


@pytest.mark.parametrize("L,Sz", [(L, 0.0) for L in range(2, 21, 2)] + [(5, 0.5), (9, -1.5),
                                                                      (12, 2.0), (15, 0.5)])
def test_sector_states_bit_exact(L, Sz):
    h, H = _ham(L, Sz=Sz)
    want = basis.enumerate_sector(L, basis.nup_from_sz(L, Sz))
    got = H.states()
    assert got.dtype == np.uint64 and np.array_equal(got, want)


@pytest.mark.parametrize("L", [24, 28])
def test_sector_states_large(L):
    h, H = _ham(L, W=4.0)
    want = basis.enumerate_sector(L, L // 2)
    assert H.n == len(want)
    assert np.array_equal(H.states(), want)


@pytest.mark.parametrize("L,Sz", [(12, 0.0), (13, 0.5), (20, 1.0)])
def test_rank_bit_exact(L, Sz):
    h, H = _ham(L, Sz=Sz)
    st = basis.enumerate_sector(L, basis.nup_from_sz(L, Sz))
    rng = np.random.default_rng(3)
    q = np.concatenate([st, rng.integers(0, 1 << L, 5000, dtype=np.uint64),
                        np.array([0, (1 << L) - 1, 1 << L, (1 << 40) + 3], dtype=np.uint64)])
    assert np.array_equal(H.rank(q), basis.rank(st, q))


@pytest.mark.parametrize("L,Sz,J,Delta", [(12, 0.0, 1.0, 1.0), (11, 0.5, 0.7, -1.3), (16, 1.0, 1.3, 0.0)])
def test_diagonal_and_jacobi(L, Sz, J, Delta):
    h, H = _ham(L, W=3.0, Sz=Sz, J=J, Delta=Delta)
    st, Ho = _oracle(L, h, Sz, J, Delta)
    sigma = 0.3
    d, jac = H.diagonal(sigma)
    np.testing.assert_allclose(d.cpu().numpy(), Ho.diagonal(), rtol=0, atol=1e-13 * (1 + np.abs(Ho.diagonal()).max()))
    jd = hamiltonian.fold_diagonal(Ho, sigma)
    np.testing.assert_allclose(jac.cpu().numpy(), jd, rtol=1e-13)


@pytest.mark.parametrize("L,Sz,J,Delta", [(11, 0.5, 0.7, -1.3), (16, 1.0, 1.3, 0.0), (13, -2.5, 2.0, 0.4)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_apply_parity_other_sectors_and_couplings(L, Sz, J, Delta, dtype):
    h, H = _ham(L, W=3.0, Sz=Sz, J=J, Delta=Delta)
    st, Ho = _oracle(L, h, Sz, J, Delta)
    X = workloads.random_block(H.n, 24, seed=L)
    Xo = X.astype(np.float32).astype(np.float64) if dtype == torch.float32 else X
    sigma = -0.41
    Y = H.apply(torch.from_numpy(X).to(DEV, dtype), sigma).double().cpu().numpy()
    tol = 1e-13 if dtype == torch.float64 else 2e-6
    assert np.all(np.abs(Y - hamiltonian.apply_shifted(Ho, Xo, sigma)) <= tol * _abs_bound(Ho, Xo, sigma) + 1e-30)


@pytest.mark.parametrize("b", [1, 3, 8, 16, 17, 64, 100])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_apply_parity_small(b, dtype):
    L = 12
    h, H = _ham(L)
    st, Ho = _oracle(L, h)
    X = workloads.random_block(H.n, b, seed=b)
    sigma = -0.37
    Y = H.apply(torch.from_numpy(X).to(DEV, dtype), sigma).double().cpu().numpy()
    Yr = hamiltonian.apply_shifted(Ho, X.astype(np.float32).astype(np.float64) if dtype == torch.float32 else X, sigma)
    tol = 1e-13 if dtype == torch.float64 else 2e-6
    bound = tol * _abs_bound(Ho, X, sigma) + (1e-300 if dtype == torch.float64 else 1e-30)
    assert np.all(np.abs(Y - Yr) <= bound)


def test_apply_strided_and_basis_vectors():
    """ld > b views, and H e_r equals column r of the oracle matrix."""
    L = 10
    h, H = _ham(L, W=2.0)
    st, Ho = _oracle(L, h)
    n = H.n
    big = torch.zeros((n, 40), dtype=torch.float64, device=DEV)
    E = torch.eye(n, dtype=torch.float64, device=DEV)[:, :24]
    big[:, 5:29] = E
    X = big[:, 5:29]
    out = torch.full((n, 50), 7.0, dtype=torch.float64, device=DEV)
    Y = H.apply(X, 0.0, out=out[:, 10:34])
    want = Ho.toarray()[:, :24]
    np.testing.assert_allclose(Y.cpu().numpy(), want, rtol=0, atol=1e-14)
    o = out.cpu().numpy()
    assert np.all(o[:, :10] == 7.0) and np.all(o[:, 34:] == 7.0)  # nothing written outside


@pytest.mark.parametrize("L,b", [(20, 64), (16, 32), (14, 48)])
def test_apply_parity_full_size(L, b):
    h, H = _ham(L, W=4.0)
    st, Ho = _oracle(L, h)
    X = workloads.random_block(H.n, b, seed=L)
    sigma = 0.11
    Y = H.apply(torch.from_numpy(X).to(DEV), sigma).cpu().numpy()
    Yr = hamiltonian.apply_shifted(Ho, X, sigma)
    assert np.all(np.abs(Y - Yr) <= 1e-13 * _abs_bound(Ho, X, sigma) + 1e-300)


@pytest.mark.parametrize("L,b,dtype", [(24, 128, torch.float32), (24, 128, torch.float64),
                                         (28, 32, torch.float64)])
def test_apply_sampled_rows_at_full_size(L, b, dtype):
    """The applies of the L = 24 (block 128, FP32 and FP64) and L = 28 (block 32,
    FP64) workloads in the launch configuration the solver uses: 600 sampled
    rows (first, last, tile edges, random) against the oracle's row-wise apply."""
    h, H = _ham(L, W=4.0)
    g = torch.Generator(device=DEV)
    g.manual_seed(L * 1000 + b)
    X = torch.randn(H.n, b, dtype=dtype, device=DEV, generator=g)
    sigma = -0.29
    Y = H.apply(X, sigma)
    rng = np.random.default_rng(L)
    edges = np.array([0, 1, 15, 16, 31, 32, 63, 64, 127, 128, H.n - 2, H.n - 1])
    rows = np.unique(np.concatenate([edges, rng.integers(0, H.n, 588)]))
    st = basis.enumerate_sector(L, L // 2)
    assert len(st) == H.n
    fetch = lambda idx: X[torch.from_numpy(np.asarray(idx)).to(DEV)].double().cpu().numpy()
    Yr, B = hamiltonian.apply_rows(L, st, 1.0, 1.0, h, rows, sigma, fetch)
    got = Y[torch.from_numpy(rows).to(DEV)].double().cpu().numpy()
    tol = 1e-13 if dtype == torch.float64 else 2e-6
    assert np.all(np.abs(got - Yr) <= tol * B + 1e-300)
    del X, Y
    torch.cuda.empty_cache()


def test_apply_symmetry_at_l24():
    """<X, H Y> = <H X, Y> at L = 24 (catches rank/index bugs at any size)."""
    L = 24
    h, H = _ham(L, W=4.0)
    X = torch.from_numpy(workloads.random_block(H.n, 4, seed=1)).to(DEV)
    Y = torch.from_numpy(workloads.random_block(H.n, 4, seed=2)).to(DEV)
    a = (X * H.apply(Y, 0.3)).sum(0)
    c = (H.apply(X, 0.3) * Y).sum(0)
    assert torch.allclose(a, c, rtol=1e-11, atol=0)
    # sampled rows against the oracle's matrix-free apply on those rows
    st = H.states()
    e = torch.zeros((H.n, 1), dtype=torch.float64, device=DEV)
    ones = torch.ones((H.n, 1), dtype=torch.float64, device=DEV)
    tr = H.apply(ones, 0.0).sum().item()
    # 1^T H 1 = trace + (J/2) * n * 2k(L-k)/L with trace = -J Delta n / 4 at S^z = 0
    n, k = H.n, L // 2
    assert abs(tr - (-n / 4 + 0.5 * n * 2 * k * (L - k) / L)) < 1e-8 * n
    del e, st


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_fold_apply(dtype):
    L = 12
    h, H = _ham(L)
    st, Ho = _oracle(L, h)
    X = workloads.random_block(H.n, 16, seed=5)
    sigma = 0.2
    Y, T = H.fold_apply(torch.from_numpy(X).to(DEV, dtype), sigma)
    Xr = X.astype(np.float32).astype(np.float64) if dtype == torch.float32 else X
    Yr = hamiltonian.apply_fold(Ho, Xr, sigma)
    Habs = abs(Ho - sigma * sp.identity(H.n, format="csr"))
    bound = Habs @ (Habs @ np.abs(X))
    tol = 3e-13 if dtype == torch.float64 else 5e-6
    assert np.all(np.abs(Y.double().cpu().numpy() - Yr) <= tol * bound + 1e-30)


@pytest.mark.parametrize("m", [0, 1, 2, 5])
@pytest.mark.parametrize("b", [1, 16, 24])
def test_pcg_parity(m, b):
    L = 12
    h, H = _ham(L)
    st, Ho = _oracle(L, h)
    sigma = 0.05
    R = workloads.random_block(H.n, b, seed=7)
    W = H.pcg(torch.from_numpy(R).to(DEV), sigma, m).cpu().numpy()
    d = hamiltonian.fold_diagonal(Ho, sigma)
    Wr = opcg.pcg_fold(Ho, sigma, d, R, m)
    if m == 0:
        assert np.all(W == 0)
    else:
        np.testing.assert_allclose(W, Wr, rtol=0, atol=1e-9 * np.abs(Wr).max())


# Launch schedules the autotuner may choose: (chunk bytes, lane bytes, tiles per
# XCD group, workgroups per XCD).  Each must give the same applies (the per-row
# arithmetic does not depend on the schedule) and oracle-exact CG.
SCHEDULES = [(128, 16, 4, 128), (256, 32, 16, 256), (256, 64, 64, 64), (512, 64, 1, 3),
             (128, 32, 0, 256)]


def _set_schedule(monkeypatch, sc):
    for k, v in zip(("MBL_APPLY_CHUNK_BYTES", "MBL_APPLY_LANE_BYTES", "MBL_APPLY_XCD_GROUP",
                     "MBL_APPLY_SLOTS_PER_XCD"), sc):
        monkeypatch.setenv(k, str(v))


@pytest.mark.parametrize("sc", SCHEDULES)
@pytest.mark.parametrize("dtype,b", [(torch.float64, 40), (torch.float32, 72)])
def test_apply_and_pcg_under_every_schedule(sc, dtype, b, monkeypatch):
    L = 14  # 3432 rows: many tiles and a ragged last tile for every row width
    h, H = _ham(L, W=4.0)
    st, Ho = _oracle(L, h)
    X = workloads.random_block(H.n, b, seed=3)
    Xd = torch.from_numpy(X).to(DEV, dtype)
    Xo = X.astype(np.float32).astype(np.float64) if dtype == torch.float32 else X
    sigma = 0.21
    ref = H.apply(Xd, sigma)  # default schedule
    _set_schedule(monkeypatch, sc)
    Y = H.apply(Xd, sigma)
    assert torch.equal(Y, ref)
    tol = 1e-13 if dtype == torch.float64 else 2e-6
    Yr = hamiltonian.apply_shifted(Ho, Xo, sigma)
    assert np.all(np.abs(Y.double().cpu().numpy() - Yr) <= tol * _abs_bound(Ho, Xo, sigma) + 1e-30)
    if dtype == torch.float64:
        m = 4
        W = H.pcg(Xd, sigma, m).cpu().numpy()
        Wr = opcg.pcg_fold(Ho, sigma, hamiltonian.fold_diagonal(Ho, sigma), X, m)
        np.testing.assert_allclose(W, Wr, rtol=0, atol=1e-9 * np.abs(Wr).max())


@pytest.mark.parametrize("L,b,dtype,m", [(20, 64, torch.float64, 8), (24, 128, torch.float32, 2)])
def test_pcg_at_full_size(L, b, dtype, m):
    """The block Jacobi-PCG of the L=20 (FP64, 64 columns, 8 steps: the captured
    graph path) and L=24 (FP32 CG, 128 columns) workloads in the launch
    configuration the solver uses, against the oracle's step-by-step PCG."""
    h, H = _ham(L, W=4.0)
    st, Ho = _oracle(L, h)
    sigma = -0.37
    R = workloads.random_block(H.n, b, seed=L)
    Rd = torch.from_numpy(R).to(DEV, dtype)
    Ro = Rd.double().cpu().numpy()
    W = H.pcg(Rd, sigma, m).double().cpu().numpy()
    del Rd
    torch.cuda.empty_cache()
    Wr = opcg.pcg_fold(Ho, sigma, hamiltonian.fold_diagonal(Ho, sigma), Ro, m)
    if dtype == torch.float64:
        np.testing.assert_allclose(W, Wr, rtol=0, atol=1e-9 * np.abs(Wr).max())
    else:
        rel = np.linalg.norm(W - Wr, axis=0) / np.linalg.norm(Wr, axis=0)
        assert rel.max() <= 1e-3, rel.max()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_pcg_column_chunks_agree(dtype, monkeypatch):
    """Solving the block CG in cache-sized column chunks (ragged last chunk)
    changes only the rounding order of the dot products."""
    L = 12
    h, H = _ham(L)
    R = torch.from_numpy(workloads.random_block(H.n, 40, seed=8)).to(DEV, dtype)
    monkeypatch.setenv("MBL_PCG_CACHE_MB", "0")
    W_full = H.pcg(R, 0.05, 6)
    monkeypatch.setenv("MBL_PCG_CACHE_MB", "0.3")
    W_chunk = H.pcg(R, 0.05, 6)
    tol = 1e-11 if dtype == torch.float64 else 1e-4
    assert torch.allclose(W_full, W_chunk, rtol=tol, atol=tol * W_full.abs().max().item())
    assert not torch.equal(W_full, torch.zeros_like(W_full))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_pcg_graph_replay_is_bitwise_identical(dtype, monkeypatch):
    """The captured CG step replayed many times equals direct launches, and the
    solve's eager work between replays does not disturb it."""
    L = 14
    h, H = _ham(L, W=4.0)
    R = torch.from_numpy(workloads.random_block(H.n, 32, seed=11)).to(DEV, dtype)
    monkeypatch.setenv("MBL_PCG_GRAPH", "0")
    W_direct = H.pcg(R, 0.07, 40)
    monkeypatch.setenv("MBL_PCG_GRAPH", "1")
    for _ in range(3):
        W_graph = H.pcg(R, 0.07, 40)
        assert torch.equal(W_direct, W_graph)
        _ = (R * 2).sum().item()  # eager work and a synchronisation in between


def test_pcg_fp32_close_to_fp64():
    L = 14
    h, H = _ham(L, W=4.0)
    st, Ho = _oracle(L, h)
    sigma = 0.1
    R = workloads.random_block(H.n, 8, seed=9)
    W32 = H.pcg(torch.from_numpy(R).to(DEV, torch.float32), sigma, 3).double().cpu().numpy()
    Wr = opcg.pcg_fold(Ho, sigma, hamiltonian.fold_diagonal(Ho, sigma), R, 3)
    assert np.linalg.norm(W32 - Wr) <= 1e-4 * np.linalg.norm(Wr)


@pytest.mark.parametrize("n,p,q", [(1000, 16, 16), (5003, 48, 48), (777, 17, 100), (20000, 192, 64), (3, 5, 7)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_gram_parity(n, p, q, dtype):
    A = workloads.random_block(n, p, seed=1)
    B = workloads.random_block(n, q, seed=2)
    At, Bt = torch.from_numpy(A).to(DEV, dtype), torch.from_numpy(B).to(DEV, dtype)
    G = api.gram(At, Bt).cpu().numpy()
    Ar, Br = At.double().cpu().numpy(), Bt.double().cpu().numpy()
    want = Ar.T @ Br
    scale = np.abs(Ar).T @ np.abs(Br)
    tol = 1e-13 if dtype == torch.float64 else 1e-5
    assert np.all(np.abs(G - want) <= tol * scale + 1e-300)
    G2 = api.gram(At, Bt).cpu().numpy()
    assert np.array_equal(G, G2)  # fixed-order reduction: bitwise repeatable


@pytest.mark.parametrize("n,m", [(1000, 48), (777, 17), (20000, 192), (5003, 130), (65, 64)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_gram_symmetric_path(n, m, dtype):
    """A^T A forms only the tiles on and above the diagonal and mirrors the rest."""
    A = workloads.random_block(n, m, seed=5)
    At = torch.from_numpy(A).to(DEV, dtype)
    G = api.gram(At, At).cpu().numpy()
    Ar = At.double().cpu().numpy()
    tol = 1e-13 if dtype == torch.float64 else 1e-5
    assert np.all(np.abs(G - Ar.T @ Ar) <= tol * (np.abs(Ar).T @ np.abs(Ar)) + 1e-300)
    assert np.array_equal(G, G.T)
    # the general path on a copy (different pointer) agrees to rounding
    G2 = api.gram(At, At.clone()).cpu().numpy()
    assert np.all(np.abs(G - G2) <= 2 * tol * (np.abs(Ar).T @ np.abs(Ar)) + 1e-300)


@pytest.mark.parametrize("n,p,q", [(1000, 48, 16), (777, 17, 5), (20000, 192, 64)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_combine_parity(n, p, q, dtype):
    A = workloads.random_block(n, p, seed=3)
    Cm = workloads.random_block(p, q, seed=4)
    At = torch.from_numpy(A).to(DEV, dtype)
    Y = api.block_combine(At, torch.from_numpy(Cm).to(DEV)).double().cpu().numpy()
    Ar = At.double().cpu().numpy()
    Cr = Cm.astype(np.float32).astype(np.float64) if dtype == torch.float32 else Cm
    want = Ar @ Cr
    tol = 1e-13 if dtype == torch.float64 else 1e-5
    assert np.all(np.abs(Y - want) <= tol * (np.abs(Ar) @ np.abs(Cr)) + 1e-300)


@pytest.mark.parametrize("m", [1, 2, 3, 7, 33, 48, 95, 96, 97, 192, 384])
def test_small_eigh(m):
    rng = np.random.default_rng(m)
    A = rng.standard_normal((m, m))
    A = A + A.T
    if m >= 48:
        A[0, 0] += 1e-9  # near-degenerate pairs are fine for Jacobi
    w, V = api.small_eigh(torch.from_numpy(A).to(DEV))
    w, V = w.cpu().numpy(), V.cpu().numpy()
    wr = np.linalg.eigvalsh(A)
    np.testing.assert_allclose(w, wr, rtol=0, atol=1e-12 * np.abs(wr).max())
    np.testing.assert_allclose(V.T @ V, np.eye(m), atol=1e-12)
    np.testing.assert_allclose(A @ V, V * w[None, :], atol=1e-11 * np.abs(wr).max())


def test_small_eigh_graded_psd_keeps_small_eigenvalues():
    """Jacobi on a Gram matrix B^T B keeps tiny eigenvalues to high relative accuracy."""
    rng = np.random.default_rng(0)
    U, _ = np.linalg.qr(rng.standard_normal((60, 60)))
    s = np.logspace(0, -6, 60)
    B = U * s[None, :]
    A = B.T @ B
    w, V = api.small_eigh(torch.from_numpy(A).to(DEV))
    np.testing.assert_allclose(np.sort(w.cpu().numpy()), np.sort(s ** 2), rtol=1e-6)


@pytest.mark.parametrize("L,W,Delta", [(10, 2.0, 1.0), (12, 8.0, 1.0), (14, 4.0, 0.0)])
def test_spectrum_bounds(L, W, Delta):
    h, H = _ham(L, W=W, Delta=Delta)
    st, Ho = _oracle(L, h, Delta=Delta)
    w = np.linalg.eigvalsh(Ho.toarray())
    lo, hi = H.spectrum_bounds(1e-12)
    assert abs(lo - w[0]) < 1e-10 and abs(hi - w[-1]) < 1e-10


def test_invalid_arguments_raise():
    with pytest.raises(api.MblError):
        api.Hamiltonian(13, np.zeros(13), Sz=0.0)  # odd L has no S^z = 0 sector
    with pytest.raises(api.MblError):
        api.Hamiltonian(4, np.array([0, np.nan, 0, 0.0]))
    h, H = _ham(8)
    with pytest.raises(api.MblError):
        H.solve(0.0, nev=9, block=8)
    with pytest.raises(api.MblError):
        H.solve(0.0, nev=2, block=40)  # 2 * block > n = 70


@pytest.mark.parametrize("L", [30, 32])
def test_largest_chains(L):
    """The largest sectors the library takes: L = 30 (n = 155,117,520) and the
    maximum L = 32 (n = 601,080,390; state words use bit 31).  The sector list
    bit-exact against the oracle's enumeration, ranks of sampled states
    (and -1 off the sector), and 400 sampled rows of the FP64 apply (two
    columns) against the oracle's row-wise apply."""
    h = workloads.disorder(L, 4.0, 0)
    H = api.Hamiltonian(L, h)
    st = basis.enumerate_sector(L, L // 2)
    assert H.n == len(st) == math.comb(L, L // 2)
    assert np.array_equal(H.states(), st)
    rng = np.random.default_rng(L)
    edges = np.array([0, 1, 31, 32, 63, 64, H.n // 2, H.n - 2, H.n - 1])
    rows = np.unique(np.concatenate([edges, rng.integers(0, H.n, 391)]))
    q = np.concatenate([st[rows], np.array([st[-1] | np.uint64(1), (1 << L) - 1], np.uint64)])
    assert np.array_equal(H.rank(q), np.concatenate([rows, [-1, -1]]))
    g = torch.Generator(device=DEV)
    g.manual_seed(L)
    X = torch.randn(H.n, 2, dtype=torch.float64, device=DEV, generator=g)
    Y = H.apply(X, -0.29)
    fetch = lambda idx: X[torch.from_numpy(np.asarray(idx)).to(DEV)].cpu().numpy()
    Yr, B = hamiltonian.apply_rows(L, st, 1.0, 1.0, h, rows, -0.29, fetch)
    got = Y[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    assert np.all(np.abs(got - Yr) <= 1e-13 * B + 1e-300)
    del X, Y, st
    H.close()
    torch.cuda.empty_cache()
