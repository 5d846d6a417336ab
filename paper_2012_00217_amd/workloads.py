"""Seeded synthetic inputs shaped like the paper's workloads.

The paper's workloads are disorder realisations of the random-field chain: the
fields h_i are drawn from U[-w, w] each time H is instantiated (Sec. 2.1); the
study sweeps realisations, disorder strengths and spectral regions (Sec. 3.1).
There is no dataset.  This module only draws numbers -- it holds none of the
solver's arithmetic -- and both the GPU path and the CPU oracle consume the
arrays it returns, so both sides see identical inputs.
"""

import numpy as np


def disorder(L, W, seed):
    """Random fields h_i ~ U[-W, W], i = 0..L-1, from numpy's PCG64 stream."""
    return np.random.default_rng(seed).uniform(-W, W, L)


def random_block(n, b, seed, dtype=np.float64):
    """n x b block of N(0, 1) entries, row-major, contiguous."""
    return np.random.default_rng(seed).standard_normal((n, b)).astype(dtype)


def batch_problems(count=256, seed_base=0, Ls=(14, 16, 18), Ws=(2, 4, 6, 8)):
    """Problem list of the batched workload: problem j draws L, W and h from seed j."""
    probs = []
    for j in range(count):
        rng = np.random.default_rng(seed_base + j)
        L = int(rng.choice(Ls))
        W = float(rng.choice(Ws))
        h = rng.uniform(-W, W, L)
        probs.append({"L": L, "W": W, "h": h, "seed": seed_base + j})
    return probs


def request_stream(count, rate_hz, seed=10_000, Ls=(16, 18, 20, 22, 24, 26),
                   eps_choices=(0.1, 0.5, 0.9)):
    """Poisson arrivals of solve requests with mixed L, W ~ U[1, 10] and eps."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, count))
    reqs = []
    for q in range(count):
        r = np.random.default_rng(seed + 1 + q)
        L = int(r.choice(Ls))
        W = float(r.uniform(1.0, 10.0))
        reqs.append({"t": float(t[q]), "L": L, "W": W, "h": r.uniform(-W, W, L),
                     "eps": float(r.choice(eps_choices)), "seed": seed + 1 + q})
    return reqs
