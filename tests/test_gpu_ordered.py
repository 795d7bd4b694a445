"""GPU parity of the ordered Gauss-Seidel relaxations (relax 2: all points,
relax 3: F points then all points; flow order of Lemma 3.1, Section 3.3;
Gauss-Seidel across levels, Jacobi inside a level) against the oracle: the
flow order bit for bit, one V-cycle and its transpose to 1e-10 (FP32 cycle
1e-5), FGMRES solutions to 1e-10 with iteration counts within one, and the
exact one-step solve of pure advection."""
import numpy as np
import pytest
import torch

from oracle import air as oair
from oracle import adjoint as oadj
from oracle.drivers import setup_problem, air_fgmres_solve
from gpu_cases import case, gpu_system, to_scipy

pytestmark = pytest.mark.gpu

SMALL_COARSE = 40
RELAX = {2: "ordered", 3: "ordered_fa"}
CASES = ["c1", "c1_p3", "slab", "slab_nu0", "kuhn_nu0", "kuhn_nu4", "layer", "c5"]


@pytest.fixture(scope="module")
def built():
    cache = {}

    def get(name):
        if name not in cache:
            v, c, prob, p = case(name)
            cache[name] = (gpu_system(v, c, prob, p), setup_problem(v, c, prob, p))
        return cache[name]
    return get


def _hier(g, relax, **kw):
    from paper_2010_11130_amd import Hierarchy
    return Hierarchy(g, max_coarse=SMALL_COARSE, relax=relax, **kw)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("ratio", [1.5, 1.0])
def test_flow_order_parity(built, name, ratio):
    """Levels, rounds and cycle breaks equal the oracle's order of the same
    matrix (the GPU's level 0) and of the oracle's own scaled matrix."""
    print("case", name, ratio, flush=True)
    g, o = built(name)
    H = _hier(g, 2, order_ratio=ratio)
    lev, rounds, breaks = H.flow_levels()
    l0 = H.level(0)
    A = to_scipy(l0["rowptr"], l0["col"], l0["val"], l0["n"])
    ref, rr, rb = oair.flow_levels(A, o.b, ratio)
    assert np.array_equal(lev, ref)
    assert (rounds, breaks) == (rr, rb)
    ref2, _, _ = oair.flow_levels(o.Shat, o.b, ratio)
    assert np.array_equal(lev, ref2)


@pytest.mark.parametrize("name", ["c1", "slab", "kuhn_nu4", "layer", "c5"])
@pytest.mark.parametrize("relax", [2, 3])
@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("ratio", [1.5, 1.0])
def test_ordered_vcycle_parity(built, name, relax, transpose, fp32, ratio):
    print("case", name, relax, transpose, fp32, ratio, flush=True)
    g, o = built(name)
    H = _hier(g, relax, adjoint=1, fp32_cycle=1 if fp32 else 0, order_ratio=ratio)
    OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE, relax=RELAX[relax], block=o.b, order_ratio=ratio)
    r = np.random.default_rng(7).standard_normal(g.n)
    z = H.vcycle(torch.as_tensor(r, device="cuda"), precision=1 if fp32 else 0,
                 transpose=transpose).cpu().numpy()
    zo = oair.vcycle_T(OH, r) if transpose else oair.vcycle(OH, r)
    tol = 1e-5 if fp32 else 1e-10
    assert np.linalg.norm(z - zo) <= tol * np.linalg.norm(zo)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("relax", [2, 3])
def test_ordered_solve_parity(built, name, relax):
    print("case", name, relax, flush=True)
    g, o = built(name)
    H = _hier(g, relax)
    OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE, relax=RELAX[relax], block=o.b)
    x, info = H.solve(tol=1e-12)
    xo, io = air_fgmres_solve(o, tol=1e-12, hier=OH)
    assert info["converged"]
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
    tol = 1e-10 if name.startswith("c1") else 1e-8
    _, i8 = H.solve(tol=tol)
    _, io8 = air_fgmres_solve(o, tol=tol, hier=OH)
    assert abs(i8["iters"] - io8["iters"]) <= 1, (i8["iters"], io8["iters"])


@pytest.mark.parametrize("name", ["kuhn_nu0", "layer", "slab_nu0"])
def test_ordered_sweep_solves_pure_advection(built, name):
    """Pure advection on an acyclic flow: the ordered sweep inverts level 0
    exactly, so FGMRES stops after one step (Lemma 3.1).  Where the facet
    graph of the mesh has cycles (the rotating flow of the slab), the oracle
    breaks the same number of them and the sweep is no longer exact, but the
    solve still converges in a few steps."""
    print("case", name, flush=True)
    g, o = built(name)
    H = _hier(g, 2)
    _, rounds, breaks = H.flow_levels()
    x, info = H.solve(tol=1e-10)
    assert info["converged"] and info["true_relres"] <= 1e-10
    if breaks == 0:
        assert info["iters"] == 1
    else:
        _, orounds, obreaks = oair.flow_levels(o.Shat, g.b)
        assert (orounds, obreaks) == (rounds, breaks)
        assert info["iters"] <= 10, info["iters"]


@pytest.mark.parametrize("relax", [2, 3])
def test_ordered_adjoint_and_fp32_solves(built, relax):
    print("case c5", relax, flush=True)
    g, o = built("c5")
    H = _hier(g, relax, adjoint=1, fp32_cycle=1)
    gvec = torch.as_tensor(np.random.default_rng(4).standard_normal(g.n), device="cuda")
    lam, ia = H.solve_adjoint(gvec, tol=1e-12)
    assert ia["converged"]
    lam_o = oadj.adjoint_direct(o, gvec.cpu().numpy())
    assert np.linalg.norm(lam.cpu().numpy() - lam_o) <= 1e-9 * np.linalg.norm(lam_o)
    x, info = H.solve(tol=1e-10, precision=1)
    x64, _ = H.solve(tol=1e-10)
    assert info["converged"]
    assert np.linalg.norm((x - x64).cpu().numpy()) <= 1e-8 * np.linalg.norm(x64.cpu().numpy())


def test_ordered_needs_scaled_system():
    from paper_2010_11130_amd import Hierarchy, AirHdgError
    v, c, prob, p = case("slab")
    g = gpu_system(v, c, prob, p, block_scale=False)
    with pytest.raises(AirHdgError):
        Hierarchy(g, max_coarse=SMALL_COARSE, relax=2)


def test_relax_bad_parameter(built):
    from paper_2010_11130_amd import Hierarchy, AirHdgError
    g, _ = built("c1")
    with pytest.raises(AirHdgError):
        Hierarchy(g, relax=4)
    with pytest.raises(AirHdgError):
        Hierarchy(g, relax=2, order_ratio=0.5)


@pytest.mark.parametrize("name", ["slab", "layer", "kuhn_nu4"])
@pytest.mark.parametrize("relax", [2, 3])
def test_ordered_bicgstab_parity(built, name, relax):
    """The ordered relaxations under the paper's Krylov method (BiCGSTAB,
    Section 4): solution to 1e-10 and step count within one."""
    from oracle.drivers import air_bicgstab_solve
    print("case", name, relax, flush=True)
    g, o = built(name)
    H = _hier(g, relax)
    OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE, relax=RELAX[relax], block=o.b)
    x, info = H.solve(tol=1e-12, method=1)
    xo, io = air_bicgstab_solve(o, tol=1e-12, hier=OH)
    assert info["converged"] and io["converged"]
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
    _, i8 = H.solve(tol=1e-8, method=1)
    _, io8 = air_bicgstab_solve(o, tol=1e-8, hier=OH)
    assert abs(i8["iters"] - io8["iters"]) <= 1, (i8["iters"], io8["iters"])


@pytest.mark.parametrize("relax", [2, 3])
@pytest.mark.parametrize("fp32", [False, True])
def test_ordered_cycles_repeat_bit_for_bit(built, relax, fp32):
    """Six cycles on one hierarchy, with other GPU work and synchronizations
    between them, give the same result bit for bit (the level sweeps take no
    decision from the order in which workgroups run), and that result
    matches the oracle."""
    print("case slab", relax, fp32, flush=True)
    g, o = built("slab")
    H = _hier(g, relax, fp32_cycle=1 if fp32 else 0)
    other = _hier(built("c5")[0], 0)
    OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE, relax=RELAX[relax], block=o.b)
    r = np.random.default_rng(9).standard_normal(g.n)
    rt = torch.as_tensor(r, device="cuda")
    zs = []
    for _ in range(6):
        zs.append(H.vcycle(rt, precision=1 if fp32 else 0).cpu().numpy())
        other.solve(tol=1e-8)
        torch.cuda.synchronize()
    for z in zs[1:]:
        assert np.array_equal(z, zs[0])
    zo = oair.vcycle(OH, r)
    tol = 1e-5 if fp32 else 1e-10
    assert np.linalg.norm(zs[0] - zo) <= tol * np.linalg.norm(zo)


@pytest.mark.parametrize("name", ["c1", "slab", "kuhn_nu4", "c5"])
@pytest.mark.parametrize("relax", [2, 3])
def test_ordered_with_block_air(built, name, relax):
    """The ordered relaxations on a block AIR hierarchy (the F points of
    relax 3 are whole facet blocks): one cycle and its transpose to 1e-10,
    the solve to 1e-10 and the iteration counts within +-1 of the oracle."""
    print("case", name, relax, "block AIR", flush=True)
    g, o = built(name)
    H = _hier(g, relax, adjoint=1, block_air=1)
    OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE, relax=RELAX[relax], block=o.b, block_air=True)
    r = np.random.default_rng(8).standard_normal(g.n)
    for transpose in (False, True):
        z = H.vcycle(torch.as_tensor(r, device="cuda"), transpose=transpose).cpu().numpy()
        zo = oair.vcycle_T(OH, r) if transpose else oair.vcycle(OH, r)
        assert np.linalg.norm(z - zo) <= 1e-10 * np.linalg.norm(zo), transpose
    x, info = H.solve(tol=1e-12)
    xo, _ = air_fgmres_solve(o, tol=1e-12, hier=OH)
    assert info["converged"]
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
    tol = 1e-10 if name.startswith("c1") else 1e-8
    _, i8 = H.solve(tol=tol)
    _, io8 = air_fgmres_solve(o, tol=tol, hier=OH)
    assert abs(i8["iters"] - io8["iters"]) <= 1, (i8["iters"], io8["iters"])
