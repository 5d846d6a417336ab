"""The seeded input generators shared by the GPU path and the oracle: the input
recipe of the benchmark workloads (fields h_i ~ U[-W, W] per realisation, the
batched problem mix, the Poisson request stream)."""

import numpy as np

from paper_2012_00217_amd import workloads


def test_disorder_is_seeded_uniform_in_range():
    h = workloads.disorder(20, 4.0, 0)
    assert h.shape == (20,) and np.all(np.abs(h) <= 4.0)
    assert np.array_equal(h, workloads.disorder(20, 4.0, 0))
    assert not np.array_equal(h, workloads.disorder(20, 4.0, 1))
    big = workloads.disorder(200_000, 3.0, 7)
    # U[-W, W]: mean 0, variance W^2 / 3 (5-sigma bounds of the sample moments)
    assert abs(big.mean()) < 5 * np.sqrt(3.0 / 200_000)
    assert abs(big.var() - 3.0) < 5 * np.sqrt(4 * 81 / 45 / 200_000)


def test_batch_problems_mix_and_per_problem_seeds():
    probs = workloads.batch_problems()
    assert len(probs) == 256
    Ls = {p["L"] for p in probs}
    Ws = {p["W"] for p in probs}
    assert Ls == {14, 16, 18} and Ws == {2.0, 4.0, 6.0, 8.0}
    combos = {(p["L"], p["W"]) for p in probs}
    assert len(combos) == 12  # every (L, W) pair occurs
    for j, p in enumerate(probs):
        assert p["seed"] == j and len(p["h"]) == p["L"] and np.all(np.abs(p["h"]) <= p["W"])
    # problem j depends on j alone, not on the batch size
    short = workloads.batch_problems(count=10)
    for a, b in zip(short, probs[:10]):
        assert a["L"] == b["L"] and a["W"] == b["W"] and np.array_equal(a["h"], b["h"])


def test_request_stream_is_poisson_with_the_stated_mix():
    rate = 2.0
    reqs = workloads.request_stream(4000, rate)
    t = np.array([r["t"] for r in reqs])
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert np.all(gaps > 0)
    # exponential gaps: mean 1/rate, coefficient of variation 1
    assert abs(gaps.mean() * rate - 1.0) < 5 / np.sqrt(4000)
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.1
    for r in reqs:
        assert r["L"] in (16, 18, 20, 22, 24, 26)
        assert 1.0 <= r["W"] <= 10.0 and np.all(np.abs(r["h"]) <= r["W"])
        assert r["eps"] in (0.1, 0.5, 0.9) and len(r["h"]) == r["L"]
    assert {r["L"] for r in reqs} == {16, 18, 20, 22, 24, 26}
    # request q's content depends on q alone
    few = workloads.request_stream(5, rate)
    for a, b in zip(few, reqs[:5]):
        assert a["L"] == b["L"] and a["W"] == b["W"] and np.array_equal(a["h"], b["h"])
        assert a["eps"] == b["eps"]
