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
