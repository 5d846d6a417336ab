"""mbl_gram_noalloc: the Gram with its partial sums in the library's fixed
per-GPU scratch array instead of allocated memory.

Checked against mbl_gram (the allocating entry point, same kernels and
reduction order: bitwise equal) and against an FP64 torch product (to the
Gram bar of the kernel tests), on two calls in a row, the second smaller, so
that the second call runs over the first one's leftovers in the scratch.
No device allocation happens inside the call: the counting allocator sees
none.
"""

import ctypes as C

import numpy as np
import pytest
import torch

from paper_2012_00217_amd import workloads

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_2012_00217_amd.api")


def _block(n, b, seed, dtype):
    return torch.from_numpy(workloads.random_block(n, b, seed=seed)).to("cuda", dtype)


def _check(A, B):
    ref = api.gram(A, B)
    out = torch.full((A.shape[1], B.shape[1]), float("nan"), dtype=torch.float64, device="cuda")
    api.gram_noalloc(A, B, out)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    exact = A.double().T.contiguous() @ B.double()
    tol = (1e-13 if A.dtype == torch.float64 else 2e-6) * (
        A.double().abs().T.contiguous() @ B.double().abs())
    assert torch.all((out - exact).abs() <= tol + 1e-300)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("shapes", [
    # (n, p, q, same operand) first call, then a smaller one
    ((184756, 64, 64, True), (12870, 32, 32, True)),
    ((705432, 128, 128, False), (48620, 16, 40, False)),
    ((300001, 384, 384, True), (1000, 7, 7, True)),
])
def test_noalloc_gram_matches_gram_two_calls(dtype, shapes):
    for i, (n, p, q, same) in enumerate(shapes):
        A = _block(n, p, 10 + i, dtype)
        B = A if same else _block(n, q, 20 + i, dtype)
        _check(A, B)


def test_noalloc_gram_allocates_nothing():
    A = _block(20000, 64, 3, torch.float64)
    B = _block(20000, 48, 4, torch.float64)
    out = torch.empty((64, 48), dtype=torch.float64, device="cuda")
    calls = []

    def alloc(n, s):
        calls.append(n)
        return torch._C._cuda_cudaCachingAllocator_raw_alloc(int(n), int(s or 0))

    def free(p, s):
        torch._C._cuda_cudaCachingAllocator_raw_delete(int(p))

    api.use_allocator(alloc, free)
    try:
        api.gram_noalloc(A, B, out)
        torch.cuda.synchronize()
        assert calls == []
        api.gram(A, B)  # the allocating entry point goes through the callback
        torch.cuda.synchronize()
        assert len(calls) >= 1
    finally:
        api.use_torch_allocator()
    assert torch.equal(out, api.gram(A, B))


def test_noalloc_gram_rejects_shapes_beyond_the_scratch():
    # 4096 x 4096 partials (128 MiB) exceed the fixed 64 MiB array
    A = _block(64, 4096, 5, torch.float32)
    out = torch.zeros((4096, 4096), dtype=torch.float64, device="cuda")
    with pytest.raises(api.MblError, match="bytes of partial sums"):
        api.gram_noalloc(A, A, out)
    assert torch.count_nonzero(out) == 0


def test_noalloc_gram_under_graph_capture():
    """The use the entry point is for: captured into a graph (torch.cuda.graph)
    and replayed, with eager work and synchronisations between the replays;
    every replay equals mbl_gram on the inputs of that moment."""
    A = _block(50000, 64, 7, torch.float32)
    B = _block(50000, 96, 8, torch.float32)
    out = torch.zeros((64, 96), dtype=torch.float64, device="cuda")
    api.gram_noalloc(A, B, out)  # first use on this GPU outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        api.gram_noalloc(A, B, out)
    for k in range(3):
        A.mul_(1.5)
        B.add_(0.25)
        _ = (A * 2).sum().item()  # eager work and a synchronisation between replays
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, api.gram(A, B)), k
