"""Device memory through the caller's allocator (ah_set_allocator, here
torch's caching allocator): the library's objects are counted by torch,
come back to it when destroyed, and give the same results as with the
library's own pool."""
import gc

import numpy as np
import pytest
import torch

from gpu_cases import case, gpu_system

pytestmark = pytest.mark.gpu


def test_torch_allocator_roundtrip():
    from paper_2010_11130_amd import Hierarchy, use_torch_allocator
    v, c, prob, p = case("slab")
    g0 = gpu_system(v, c, prob, p)
    x0, i0 = Hierarchy(g0, max_coarse=40).solve(tol=1e-10)
    x0 = x0.cpu().numpy()
    del g0
    gc.collect()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    use_torch_allocator(True)
    try:
        g = gpu_system(v, c, prob, p)
        H = Hierarchy(g, max_coarse=40)
        x, info = H.solve(tol=1e-10)
        torch.cuda.synchronize()
        during = torch.cuda.memory_allocated()
        assert info["iters"] == i0["iters"]
        assert np.array_equal(x.cpu().numpy(), x0)
        # system, hierarchy and solver workspace (several MB) come from torch
        assert during - before > (4 << 20)
        del H, g, x
        gc.collect()
        torch.cuda.synchronize()
        after = torch.cuda.memory_allocated()
        assert after - before < (1 << 20), (before, during, after)
    finally:
        use_torch_allocator(False)
    # back on the library pool
    g2 = gpu_system(v, c, prob, p)
    x2, _ = Hierarchy(g2, max_coarse=40).solve(tol=1e-10)
    assert np.array_equal(x2.cpu().numpy(), x0)


def test_library_cache_reuses_and_trims():
    """The library's caching allocator: repeated hierarchies of one system
    (setup + solve, destroyed each time) take no new device memory after the
    first, give the same solution bit for bit, and ah_pool_trim gives the
    cached blocks back to the device."""
    from paper_2010_11130_amd import Hierarchy, pool_trim
    v, c, prob, p = case("kuhn_nu4")
    g = gpu_system(v, c, prob, p)
    torch.cuda.synchronize()
    pool_trim()
    free0 = torch.cuda.mem_get_info()[0]
    xs, frees = [], []
    for _ in range(4):
        H = Hierarchy(g, max_coarse=40, block_air=1)
        x, info = H.solve(tol=1e-10)
        assert info["converged"]
        xs.append(x.cpu().numpy())
        del H, x
        gc.collect()
        torch.cuda.synchronize()
        frees.append(torch.cuda.mem_get_info()[0])
    for x in xs[1:]:
        assert np.array_equal(x, xs[0])
    # the first pass maps the cache's blocks, the later ones reuse them
    assert frees[1] == frees[2] == frees[3], frees
    assert frees[1] < free0
    pool_trim()
    assert torch.cuda.mem_get_info()[0] > frees[3]
