"""GPU tests of the boundary's memory, stop and timing behaviour.

* Every device byte the library uses goes through the installed allocator
  callbacks and is given back to the allocator that made it.
* A solve stops on its time limit or cancel flag with its best pairs
  (MBL_ECANCELLED); the server cancels queued and running requests.
* Per-phase timers; both choices of the wanted Ritz pairs reach the same
  pairs, including a pair mirrored about sigma (equal fold eigenvalues).
"""

import ctypes as C
import threading
import time

import numpy as np
import pytest
import torch

from oracle import hamiltonian, linalg, spectrum
from paper_2012_00217_amd import workloads

pytestmark = pytest.mark.gpu

api = pytest.importorskip("paper_2012_00217_amd.api")


def _cfg(L, W, seed=0, eps=0.5):
    h = workloads.disorder(L, W, seed)
    st, Ho = hamiltonian.sector_matrix(L, L // 2, 1.0, 1.0, h)
    w = np.linalg.eigvalsh(Ho.toarray()) if len(st) <= 13000 else None
    return h, Ho, w


class Counting:
    """Allocator callbacks over torch's caching allocator that count bytes."""

    def __init__(self):
        self.live = {}
        self.allocs = self.frees = 0
        self.peak = 0
        self.lock = threading.Lock()

    def alloc(self, n, s):
        p = torch._C._cuda_cudaCachingAllocator_raw_alloc(int(n), int(s or 0))
        with self.lock:
            self.live[p] = n
            self.allocs += 1
            self.peak = max(self.peak, sum(self.live.values()))
        return p

    def free(self, p, s):
        with self.lock:
            assert p in self.live, "freed a pointer this allocator did not make"
            del self.live[p]
            self.frees += 1
        torch._C._cuda_cudaCachingAllocator_raw_delete(int(p))


def test_every_workspace_byte_goes_through_the_allocator():
    L = 12
    h, Ho, w = _cfg(L, 8.0)
    cnt = Counting()
    api.use_allocator(cnt.alloc, cnt.free)
    try:
        H = api.Hamiltonian(L, h)
        tables = sum(cnt.live.values())
        assert tables >= H.n * (4 + 8)  # state list and diagonal
        sigma = w[0] + 0.5 * (w[-1] - w[0])
        ev, V, rs, info = H.solve(sigma, 8, 16, tol=1e-10)
        torch.cuda.synchronize()
        # only the tables are still held; the solve's work space came and went
        assert sum(cnt.live.values()) == tables
        assert cnt.peak > tables + 3 * 16 * H.n * 8
        want = np.sort(w[np.argsort(np.abs(w - sigma), kind="stable")[:8]])
        assert np.abs(ev - want).max() < 1e-10
        H2 = api.Hamiltonian(L, h)
    finally:
        api.use_torch_allocator()
    # buffers are returned to the allocator that made them, even after a switch
    H.close()
    H2.close()
    assert cnt.live == {} and cnt.allocs == cnt.frees > 0


def test_solve_time_limit_returns_best_pairs():
    L = 16
    h, Ho, w = _cfg(L, 4.0)
    H = api.Hamiltonian(L, h)
    sigma = w[0] + 0.5 * (w[-1] - w[0])
    t0 = time.perf_counter()
    ev, V, rs, info = H.solve(sigma, 16, 32, tol=1e-10, max_seconds=0.02, raise_on_noconv=False)
    el = time.perf_counter() - t0
    assert info["status"] == "MBL_ECANCELLED"
    assert el < 5.0
    assert np.all(np.isfinite(ev)) and np.all(np.isfinite(rs)) and np.all(rs >= 0)
    # the returned residuals are the true ones for the returned pairs
    np.testing.assert_allclose(rs, linalg.residual_norms(Ho, ev, V.cpu().numpy()),
                               rtol=1e-6, atol=1e-12)
    with pytest.raises(api.MblError):
        H.solve(sigma, 16, 32, tol=1e-10, max_seconds=-1.0)


def test_solve_cancel_flag():
    L = 14
    h, Ho, w = _cfg(L, 4.0)
    H = api.Hamiltonian(L, h)
    sigma = w[0] + 0.5 * (w[-1] - w[0])
    flag = C.c_int(1)
    ev, V, rs, info = H.solve(sigma, 8, 16, tol=1e-10, cancel=flag, raise_on_noconv=False)
    assert info["status"] == "MBL_ECANCELLED" and info["iters"] == 0
    flag.value = 0
    ev, V, rs, info = H.solve(sigma, 8, 16, tol=1e-10, cancel=flag)
    assert info["status"] == "MBL_OK"


def test_server_cancels_queued_and_running_requests():
    slow = {"L": 20, "h": workloads.disorder(20, 2.0, 1), "eps": 0.5, "nev": 16, "block": 32,
            "tol": 1e-12, "precision": "f64", "seed": 7}
    quick = {"L": 12, "h": workloads.disorder(12, 8.0, 0), "eps": 0.5, "nev": 8, "block": 16,
             "tol": 1e-10, "precision": "f64", "seed": 7}
    with api.Server(max_slots=1) as srv:
        ta = srv.submit(slow)
        tb = srv.submit(quick)
        time.sleep(0.5)
        srv.cancel(tb)  # still queued behind the running solve
        srv.cancel(ta)  # running
        rb = srv.wait(tb)
        ra = srv.wait(ta)
        assert rb["status"] == "MBL_ECANCELLED"
        assert ra["status"] in ("MBL_ECANCELLED", "MBL_OK")
        with pytest.raises(api.MblError):
            srv.cancel(ta)  # finished
        # the server keeps serving
        rc = srv.wait(srv.submit(quick))
        assert rc["status"] == "MBL_OK"


def test_phase_timers():
    L = 14
    h, Ho, w = _cfg(L, 4.0)
    H = api.Hamiltonian(L, h)
    sigma = w[0] + 0.5 * (w[-1] - w[0])
    ev, V, rs, info = H.solve(sigma, 8, 16, tol=1e-10, timing=True)
    assert info["t_apply"] > 0 and info["t_gram"] > 0 and info["t_small"] > 0
    assert info["t_pcg"] > 0 and info["cg_apply1_launches"][0] > 0
    # every CG step is counted once per kernel and column chunk; the timed
    # launches are a sample of them
    steps, nl = info["pcg_steps"], info["cg_launches_all"][0]
    assert nl % steps == 0 and nl >= info["cg_apply1_launches"][0]
    nch = nl // steps
    assert info["cg_apply2_ms_all"][0] >= info["cg_apply2_ms"][0] > 0
    n = H.n
    assert info["cg_apply1_bytes_all"][0] == pytest.approx(steps * (2 * n * 16 * 8 + 12 * n * nch))
    assert info["cg_apply2_bytes_all"][0] == pytest.approx(steps * (6 * n * 16 * 8 + 20 * n * nch))
    ev, V, rs, info = H.solve(sigma, 8, 16, tol=1e-10)
    assert info["t_apply"] == 0 and info["t_gram"] == 0


@pytest.mark.parametrize("select", ["fold", "theta"])
def test_wanted_set_choices_reach_the_same_pairs(select, monkeypatch):
    """The wanted pairs picked among the Ritz pairs by their fold quotient
    theta^2 + |r|^2 (default) or by |theta| alone: the same converged pairs."""
    L = 12
    h, Ho, w = _cfg(L, 8.0)
    H = api.Hamiltonian(L, h)
    sigma = w[0] + 0.5 * (w[-1] - w[0])
    monkeypatch.setenv("MBL_SELECT", select)
    ev, V, rs, info = H.solve(sigma, 8, 16, tol=1e-10)
    want = np.sort(w[np.argsort(np.abs(w - sigma), kind="stable")[:8]])
    assert np.abs(ev - want).max() < 1e-10
    assert linalg.residual_norms(Ho, ev, V.cpu().numpy()).max() <= 1e-10


def test_pair_mirrored_about_sigma():
    """sigma exactly halfway between two neighbouring eigenvalues: they have
    the same fold eigenvalue, and both must come out resolved."""
    L = 12
    h, Ho, w = _cfg(L, 8.0)
    k = len(w) // 2
    sigma = 0.5 * (w[k] + w[k + 1])
    H = api.Hamiltonian(L, h)
    ev, V, rs, info = H.solve(sigma, 8, 16, tol=1e-10)
    want = np.sort(w[np.argsort(np.abs(w - sigma), kind="stable")[:8]])
    assert np.abs(ev - want).max() < 1e-10
    assert w[k] in want and w[k + 1] in want
    assert linalg.residual_norms(Ho, ev, V.cpu().numpy()).max() <= 1e-10


@pytest.mark.parametrize("guard", [1.0, 0.25, 0.05])
def test_guard_column_cg_fraction(guard):
    """The guard columns (block columns beyond nev) may run a fraction of the
    CG steps: the same converged pairs, fewer column-steps."""
    L = 14
    h, Ho, w = _cfg(L, 4.0)
    H = api.Hamiltonian(L, h)
    sigma = w[0] + 0.5 * (w[-1] - w[0])
    ev, V, rs, info = H.solve(sigma, 8, 24, tol=1e-10, guard_cg=guard)
    want = np.sort(w[np.argsort(np.abs(w - sigma), kind="stable")[:8]])
    assert np.abs(ev - want).max() < 1e-10
    assert linalg.residual_norms(Ho, ev, V.cpu().numpy()).max() <= 1e-10
    if guard < 1.0:
        assert info["pcg_columns"] < 24 * info["pcg_steps"]
    with pytest.raises(api.MblError):
        H.solve(sigma, 8, 24, tol=1e-10, guard_cg=1.5)
