"""The allocation-free solve (``air_solve_noalloc``) against ``air_solve``:
the same hierarchy and right-hand side give the same solution and iteration
count, on two calls in a row (the second on a smaller system, so the shared
scratch array holds the first call's contents), with the FP64 and the FP32
cycle; workspaces beyond the scratch array are rejected before any device
work."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_cases import case, gpu_system

pytestmark = pytest.mark.gpu


def _solve_both(name, precision, restart):
    from paper_2010_11130_amd import Hierarchy
    v, c, prob, p = case(name)
    g = gpu_system(v, c, prob, p)
    H = Hierarchy(g, max_coarse=40, fp32_cycle=1 if precision else 0)
    rhs = torch.as_tensor(np.random.default_rng(41).standard_normal(g.n), device="cuda")
    x_ref, i_ref = H.solve(rhs, tol=1e-10, precision=precision, restart=restart)
    out = torch.full((g.n,), np.nan, dtype=torch.float64, device="cuda")
    x_na, i_na = H.solve(rhs, out=out, noalloc=True, tol=1e-10, precision=precision, restart=restart)
    torch.cuda.synchronize()
    return g.n, x_ref.cpu().numpy(), i_ref, x_na.cpu().numpy(), i_na


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_air_solve_twice(precision):
    sizes = []
    for name in ("slab", "c1"):          # larger system first, then a smaller one
        print("case", name, "precision", precision, flush=True)
        n, x_ref, i_ref, x_na, i_na = _solve_both(name, precision, 100)
        sizes.append(n)
        assert i_na["converged"] and i_ref["converged"]
        assert i_na["iters"] == i_ref["iters"], (i_na["iters"], i_ref["iters"])
        assert np.all(np.isfinite(x_na))
        assert np.linalg.norm(x_na - x_ref) <= 1e-10 * np.linalg.norm(x_ref)
    assert sizes[1] < sizes[0]


def test_noalloc_rejects_oversized_workspace():
    from paper_2010_11130_amd import Hierarchy, AirHdgError
    from paper_2010_11130_amd._lib import AH_EUNSUPPORTED
    v, c, prob, p = case("slab")
    g = gpu_system(v, c, prob, p)
    H = Hierarchy(g, max_coarse=40)
    out = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    # 5,184 unknowns: restart 129 exceeds the cap; restart 128 needs about
    # 11 MB and fits; BiCGSTAB is not offered without allocation
    with pytest.raises(AirHdgError) as e:
        H.solve(out=out, noalloc=True, restart=129)
    assert e.value.status == AH_EUNSUPPORTED
    with pytest.raises(AirHdgError) as e:
        H.solve(out=out, noalloc=True, method=1)
    assert e.value.status == AH_EUNSUPPORTED
    x, info = H.solve(out=out, noalloc=True, restart=128, tol=1e-10)
    assert info["converged"]


def test_noalloc_takes_no_device_memory_and_rejects_large_systems():
    """On a hierarchy that has never solved, the allocation-free solve leaves
    the free device memory unchanged (its 51 MB workspace lives in the static
    array), while air_solve then takes its workspace from the library pool;
    a system whose workspace exceeds the array is rejected."""
    from paper_2010_11130_amd import Hierarchy, AirHdgError
    from paper_2010_11130_amd._lib import AH_EUNSUPPORTED
    from workloads import kuhn_cube_mesh
    from workloads.problems import SmoothPlusFront
    prob = SmoothPlusFront(1e-4)
    v, c = kuhn_cube_mesh(12)
    g = gpu_system(v, c, prob, 1)
    H = Hierarchy(g, max_coarse=40)
    out = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    x, info = H.solve(out=out, noalloc=True, restart=50, tol=1e-8)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    print("n", g.n, "free before/after noalloc", free0, free1, flush=True)
    assert info["converged"]
    assert free0 - free1 < 8 << 20
    x2, info2 = H.solve(restart=50, tol=1e-8)
    assert info2["iters"] == info["iters"]
    assert np.linalg.norm((x2 - out).cpu().numpy()) <= 1e-10 * np.linalg.norm(x2.cpu().numpy())
    v, c = kuhn_cube_mesh(16)
    g2 = gpu_system(v, c, prob, 1)
    H2 = Hierarchy(g2, max_coarse=40)
    out2 = torch.zeros(g2.n, dtype=torch.float64, device="cuda")
    with pytest.raises(AirHdgError, match="exceeds") as e:
        H2.solve(out=out2, noalloc=True, restart=100)
    assert e.value.status == AH_EUNSUPPORTED
