"""Batch and serving entry points: results equal the single-solve path
(bitwise: every solve is a deterministic kernel sequence), parity with the
oracle on a stratified sample, footprint admission and server statistics."""

import math
import re

import numpy as np
import pytest
import torch

from oracle import hamiltonian, linalg, spectrum
from paper_2012_00217_amd import workloads

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_2012_00217_amd.api")


def _problems():
    probs = []
    for j, (L, W) in enumerate([(12, 2.0), (14, 4.0), (12, 8.0), (14, 6.0), (16, 4.0), (12, 6.0)]):
        probs.append({"L": L, "h": workloads.disorder(L, W, 100 + j), "eps": 0.5, "nev": 8,
                      "block": 16, "tol": 1e-10, "precision": "f64", "seed": 7})
    return probs


def test_batch_equals_single_solves_and_oracle():
    probs = _problems()
    res = api.batch_solve(probs, concurrency=4, vectors=True)
    for d, r in zip(probs, res):
        assert r["status"] == "MBL_OK", r
        H = api.Hamiltonian(d["L"], d["h"])
        ev, V, rs, info = H.solve(r["sigma"], d["nev"], d["block"], tol=d["tol"], seed=d["seed"])
        assert np.array_equal(ev, r["evals"]) and torch.equal(V, r["evecs"])
        st, Ho = hamiltonian.sector_matrix(d["L"], d["L"] // 2, 1.0, 1.0, d["h"])
        w_ref, _ = spectrum.nearest(Ho, r["sigma"], d["nev"])
        assert np.max(np.abs(r["evals"] - w_ref)) <= 1e-10
        assert np.max(linalg.residual_norms(Ho, r["evals"], r["evecs"].cpu().numpy())) <= 1e-10
        lo, hi = spectrum.bounds(Ho)
        assert abs(r["sigma"] - (lo + 0.5 * (hi - lo))) < 1e-9


@pytest.mark.parametrize("conc", [8, 12])
def test_fused_cg_batch_is_bitwise_the_unfused_batch(conc, monkeypatch, capfd):
    """Concurrent solves of one chain length share their CG launches (one
    launch per kernel for the group); every problem keeps the bits of its own
    launch, so the batch with and without fusion, and single solves, agree
    bitwise.  Mixed L and W, FP64 and mixed precision."""
    probs = []
    for j, (L, W) in enumerate([(14, 2.0), (16, 4.0), (14, 6.0), (16, 8.0), (14, 4.0),
                                (16, 2.0), (14, 8.0), (16, 6.0), (18, 4.0), (18, 6.0)]):
        probs.append({"L": L, "h": workloads.disorder(L, W, 200 + j), "eps": 0.5, "nev": 16,
                      "block": 32, "tol": 1e-10, "precision": "mixed" if j % 3 == 2 else "f64",
                      "seed": 7})
    monkeypatch.setenv("MBL_FUSE_STATS", "1")
    monkeypatch.setenv("MBL_BATCH_FUSE", "1")
    # a long gather window: the solves of one L start together, so their CG
    # calls arrive within it and share launches whatever the thread timing
    monkeypatch.setenv("MBL_FUSE_WAIT_MS", "200")
    # with 10 workers and groups of at most 8 calls, full groups close and the
    # next calls start new ones
    fused = api.batch_solve(probs, concurrency=conc, vectors=True)
    m = re.search(r"fused CG: (\d+) groups, (\d+) calls", capfd.readouterr().err)
    assert m, "no fusion statistics"
    groups, calls = int(m.group(1)), int(m.group(2))
    assert calls > groups > 0  # some CG calls ran together
    monkeypatch.setenv("MBL_BATCH_FUSE", "0")
    plain = api.batch_solve(probs, concurrency=conc, vectors=True)
    for d, a, b in zip(probs, fused, plain):
        assert a["status"] == b["status"] == "MBL_OK"
        assert np.array_equal(a["evals"], b["evals"]) and torch.equal(a["evecs"], b["evecs"])
    for d, a in list(zip(probs, fused))[::3]:
        H = api.Hamiltonian(d["L"], d["h"])
        ev, V, rs, info = H.solve(a["sigma"], d["nev"], d["block"], tol=d["tol"], seed=d["seed"],
                                  precision=d["precision"])
        assert np.array_equal(ev, a["evals"]) and torch.equal(V, a["evecs"])
        st, Ho = hamiltonian.sector_matrix(d["L"], d["L"] // 2, 1.0, 1.0, d["h"])
        assert np.max(linalg.residual_norms(Ho, a["evals"], a["evecs"].cpu().numpy())) <= 1e-10


def test_batch_reports_per_problem_errors():
    probs = _problems()[:2]
    probs[1]["nev"] = 40  # nev > block
    res = api.batch_solve(probs, concurrency=2)
    assert res[0]["status"] == "MBL_OK"
    assert res[1]["status"] == "MBL_EINVAL"


def test_server_results_equal_alone_and_in_the_mix():
    probs = _problems()
    with api.Server(max_slots=3) as srv:
        tickets = [srv.submit(dict(d, want_vectors=True)) for d in probs]
        outs = []
        for t, d in zip(tickets, probs):
            V = torch.empty((math.comb(d["L"], d["L"] // 2), d["nev"]), dtype=torch.float64,
                            device="cuda")
            r = srv.wait(t, vectors_out=V)
            outs.append((r, V))
        st = srv.stats()
    assert st["completed"] == len(probs) and st["rejected"] == 0
    assert 0 < st["p50_latency"] <= st["p99_latency"]
    alone = api.batch_solve(probs, concurrency=1, vectors=True)
    for (r, V), a in zip(outs, alone):
        assert r["status"] == "MBL_OK"
        assert np.array_equal(r["evals"], a["evals"]) and torch.equal(V, a["evecs"])


def test_server_admission_refuses_oversized_request():
    d = _problems()[0]
    budget = api.footprint_bytes(14, 16, "f64") + 1000
    with api.Server(max_slots=2, hbm_budget=budget) as srv:
        t_small = srv.submit(d)  # L=12 fits
        with pytest.raises(api.MblError) as e:
            srv.submit(dict(d, L=16, h=workloads.disorder(16, 4.0, 1)))
        assert "exceeds the budget" in str(e.value)
        r = srv.wait(t_small)
        assert r["status"] == "MBL_OK"
        assert srv.stats()["rejected"] == 1
        assert srv.stats()["peak_bytes"] <= budget


def test_server_wait_timeout_returns_none():
    d = dict(_problems()[4], L=18, h=workloads.disorder(18, 4.0, 3), nev=16, block=32)
    with api.Server(max_slots=1) as srv:
        t = srv.submit(d)
        assert srv.wait(t, timeout=0.0) is None
        r = srv.wait(t)
        assert r["status"] == "MBL_OK"


def test_heterogeneous_mix_equals_alone_and_oracle():
    """Precisions, odd L with S^z = 1/2 and other couplings served side by side:
    every result is bitwise the one-at-a-time result and matches the oracle."""
    specs = [(13, 0.5, 1.0, 1.0, "mixed"), (12, 1.0, 0.8, 1.6, "pcg32"), (14, 0.0, 1.0, 0.0, "f64"),
             (11, -0.5, 1.2, 0.7, "mixed"), (12, 0.0, 1.0, 1.0, "pcg32")]
    probs = []
    for j, (L, Sz, J, Delta, prec) in enumerate(specs):
        probs.append({"L": L, "Sz": Sz, "J": J, "Delta": Delta, "h": workloads.disorder(L, 5.0, 200 + j),
                      "eps": 0.3 + 0.1 * j, "nev": 6, "block": 12, "tol": 1e-10, "precision": prec,
                      "seed": 11})
    with api.Server(max_slots=4) as srv:
        tickets = [srv.submit(d) for d in probs]
        mixed = [srv.wait(t) for t in tickets]
    alone = api.batch_solve(probs, concurrency=1)
    for d, r, a in zip(probs, mixed, alone):
        assert r["status"] == "MBL_OK", r
        assert np.array_equal(r["evals"], a["evals"])
        k = int(round(d["Sz"] + d["L"] / 2))
        st, Ho = hamiltonian.sector_matrix(d["L"], k, d["J"], d["Delta"], d["h"])
        w_ref, _ = spectrum.nearest(Ho, r["sigma"], d["nev"])
        assert np.max(np.abs(r["evals"] - w_ref)) <= 1e-10
