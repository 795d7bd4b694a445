"""Solver code paths that the library picks by problem size, forced on the
small parity cases and compared with the oracle:
  * FGMRES with the delayed CGS2 orthogonalisation (default from 2^21
    unknowns; AH_DCGS_MIN=0 here); the oracle orthogonalises by modified
    Gram-Schmidt, so the two differ only in rounding;
  * coarse levels swept through their F and C point lists after an explicit
    interpolation (default from 2^16 rows; AH_LIST_MIN=0 here), with 2, 4
    and 8 lanes per row (AH_GC);
  * PMIS by rounds of separate launches (default above 8192 points;
    AH_PMIS_WG_MAX=0 here), over all points or over the points still
    undecided (default from 2^20 points; AH_PMIS_LIST_MIN=0 here).

Tolerances as in the other parity tests: solution at tol 1e-12 within 1e-10
relative of the oracle's, iteration counts at the workload tolerance within
+-1 of the oracle's; FP32 cycle within 1e-8 of the direct solve at 1e-10;
adjoint within 1e-10 of the direct transposed solve."""
import numpy as np
import pytest
import torch

from oracle import air as oair, adjoint as oadj
from oracle.drivers import setup_problem, air_fgmres_solve, direct_solve
from gpu_cases import case, gpu_system

pytestmark = pytest.mark.gpu

SMALL_COARSE = 40


@pytest.fixture(scope="module")
def built():
    cache = {}

    def get(name):
        if name not in cache:
            v, c, prob, p = case(name)
            cache[name] = (gpu_system(v, c, prob, p), setup_problem(v, c, prob, p))
        return cache[name]
    return get


@pytest.fixture
def dcgs(monkeypatch):
    monkeypatch.setenv("AH_DCGS_MIN", "0")


@pytest.mark.parametrize("name", ["c1", "slab", "kuhn_nu0", "kuhn_nu4", "kuhn_nu2", "c5", "layer"])
def test_dcgs2_solve_parity(built, dcgs, name):
    from paper_2010_11130_amd import Hierarchy
    print("case", name, flush=True)
    g, o = built(name)
    H = Hierarchy(g, max_coarse=SMALL_COARSE)
    x, info = H.solve(tol=1e-12)
    OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE)
    xo, io = air_fgmres_solve(o, tol=1e-12, hier=OH)
    assert info["converged"]
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
    tol = 1e-10 if name.startswith("c1") else 1e-8
    _, i8 = H.solve(tol=tol)
    _, io8 = air_fgmres_solve(o, tol=tol, hier=OH)
    assert abs(i8["iters"] - io8["iters"]) <= 1, (i8["iters"], io8["iters"])


@pytest.mark.parametrize("name", ["c1", "slab", "kuhn_nu4"])
def test_dcgs2_restarts_and_fp32_cycle(built, dcgs, name):
    from paper_2010_11130_amd import Hierarchy
    print("case", name, flush=True)
    g, o = built(name)
    xo = direct_solve(o)
    H = Hierarchy(g, max_coarse=SMALL_COARSE, fp32_cycle=1)
    for restart in (1, 3, 7):
        x, info = H.solve(tol=1e-11, restart=restart, maxit=2000)
        assert info["converged"], restart
        assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-9 * np.linalg.norm(xo), restart
    x, info = H.solve(tol=1e-10, precision=1)
    assert info["converged"]
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-8 * np.linalg.norm(xo)


@pytest.mark.parametrize("precision", [0, 1])
def test_dcgs2_adjoint(built, dcgs, precision):
    from paper_2010_11130_amd import Hierarchy
    g, o = built("c5")
    H = Hierarchy(g, max_coarse=SMALL_COARSE, adjoint=1, fp32_cycle=precision)
    rhs = np.random.default_rng(51).standard_normal(g.n)
    lam, info = H.solve_adjoint(torch.as_tensor(rhs, device="cuda"), tol=1e-12, precision=precision)
    assert info["converged"]
    ref = oadj.adjoint_direct(o, rhs)
    assert np.linalg.norm(lam.cpu().numpy() - ref) <= 1e-10 * np.linalg.norm(ref)


def test_dcgs2_iteration_limit_and_same_iterations_as_cgs2(built, monkeypatch):
    """maxit caps the finished columns (AH_ENOCONV, best iterate written),
    and the two orthogonalisations take the same number of iterations."""
    from paper_2010_11130_amd import Hierarchy
    g, o = built("kuhn_nu4")
    monkeypatch.setenv("AH_DCGS_MIN", "0")
    Hd = Hierarchy(g, max_coarse=SMALL_COARSE)
    x, info = Hd.solve(tol=1e-12, maxit=3)
    assert not info["converged"] and info["iters"] == 3 and info["status"] == 1
    assert np.all(np.isfinite(x.cpu().numpy()))
    _, idc = Hd.solve(tol=1e-9)
    monkeypatch.setenv("AH_DCGS_MIN", str(1 << 40))
    Hc = Hierarchy(g, max_coarse=SMALL_COARSE)
    _, icg = Hc.solve(tol=1e-9)
    assert abs(idc["iters"] - icg["iters"]) <= 1, (idc["iters"], icg["iters"])


@pytest.fixture(params=["2", "4", "8"])
def coarse_lists(request, monkeypatch):
    monkeypatch.setenv("AH_LIST_MIN", "0")
    monkeypatch.setenv("AH_GC", request.param)
    return request.param


@pytest.mark.parametrize("name", ["c1", "slab", "kuhn_nu4", "c5"])
@pytest.mark.parametrize("fp32", [False, True])
def test_coarse_list_sweeps_vcycle(built, coarse_lists, name, fp32):
    from paper_2010_11130_amd import Hierarchy
    print("case", name, fp32, coarse_lists, flush=True)
    g, o = built(name)
    H = Hierarchy(g, max_coarse=SMALL_COARSE, fp32_cycle=1 if fp32 else 0)
    OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE)
    r = np.random.default_rng(52).standard_normal(g.n)
    z = H.vcycle(torch.as_tensor(r, device="cuda"), precision=1 if fp32 else 0).cpu().numpy()
    zo = oair.vcycle(OH, r)
    err = np.linalg.norm(z - zo) / np.linalg.norm(zo)
    if not fp32:
        assert err <= 1e-10
    else:
        z32 = oair.vcycle(OH, r, dtype=np.float32).astype(np.float64)
        assert err <= 4.0 * np.linalg.norm(z32 - zo) / np.linalg.norm(zo) + 1e-12


@pytest.mark.parametrize("name", ["c1", "slab", "kuhn_nu4", "layer"])
def test_coarse_list_sweeps_solve(built, coarse_lists, name):
    from paper_2010_11130_amd import Hierarchy
    print("case", name, coarse_lists, flush=True)
    g, o = built(name)
    H = Hierarchy(g, max_coarse=SMALL_COARSE, relax=1 if name == "layer" else 0)
    x, info = H.solve(tol=1e-12)
    OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE, relax="F" if name == "layer" else "FFC")
    xo, io = air_fgmres_solve(o, tol=1e-12, hier=OH)
    assert info["converged"]
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)


@pytest.mark.parametrize("delayed", [False, True])
def test_workspace_reuse_across_restarts_and_precisions(built, monkeypatch, delayed):
    """One hierarchy solved with a long restart in FP64, then with shorter
    and growing restarts in FP32 and FP64 (regression: the basis of a
    precision first used with a short restart was sized for that restart,
    not for the workspace's capacity, and a later longer restart wrote past
    it).  Every solve matches a fresh hierarchy's solve of the same
    settings bit for bit."""
    from paper_2010_11130_amd import Hierarchy
    if delayed:
        monkeypatch.setenv("AH_DCGS_MIN", "0")
    g, o = built("kuhn_nu4")
    print("case kuhn_nu4 workspace reuse, delayed", delayed, flush=True)
    H = Hierarchy(g, max_coarse=SMALL_COARSE, fp32_cycle=1)
    H.solve(tol=1e-10, restart=30, precision=0)
    for prec, m in ((1, 5), (1, 8), (1, 30), (0, 5), (0, 12)):
        x, info = H.solve(tol=1e-10, restart=m, precision=prec)
        F = Hierarchy(g, max_coarse=SMALL_COARSE, fp32_cycle=1)
        xf, infof = F.solve(tol=1e-10, restart=m, precision=prec)
        assert info["converged"] and info["iters"] == infof["iters"], (prec, m)
        assert np.array_equal(x.cpu().numpy(), xf.cpu().numpy()), (prec, m)
        del F


@pytest.mark.parametrize("name", ["c1", "slab", "kuhn_nu4", "c5", "layer"])
@pytest.mark.parametrize("block_air", [0, 1])
@pytest.mark.parametrize("listed", [False, True])
def test_pmis_rounds_paths(built, monkeypatch, name, block_air, listed):
    """PMIS by rounds of separate launches (default above 8192 points;
    AH_PMIS_WG_MAX=0 here), over all points in every round or (``listed``,
    default from 2^20 points; AH_PMIS_LIST_MIN=0) over the points still
    undecided: the same rounds, so C/F splitting and one-point P bit for bit
    equal to the oracle's on every level, scalar and block AIR."""
    from paper_2010_11130_amd import Hierarchy
    print("case", name, block_air, listed, flush=True)
    monkeypatch.setenv("AH_PMIS_WG_MAX", "0")
    monkeypatch.setenv("AH_PMIS_LIST_MIN", "0" if listed else str(1 << 40))
    g, o = built(name)
    H = Hierarchy(g, max_coarse=SMALL_COARSE, block_air=block_air)
    kw = {"block_air": True, "block": o.b} if block_air else {}
    OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE, **kw)
    assert H.info["n"] == [lev.A.shape[0] for lev in OH.levels]
    for l in range(OH.nlev - 1):
        lv = H.level(l)
        ol = OH.levels[l]
        assert np.array_equal(lv["cf"].cpu().numpy(), ol.cf), l
        Pd = ol.P.tocsr()
        opc = np.full(ol.A.shape[0], -1)
        opc[np.repeat(np.arange(Pd.shape[0]), np.diff(Pd.indptr))] = Pd.indices
        assert np.array_equal(lv["pcol"].cpu().numpy(), opc), l


@pytest.mark.parametrize("name", ["c1", "slab", "kuhn_nu4", "c5", "layer"])
@pytest.mark.parametrize("fp32", [False, True])
def test_coarse_list_sweeps_sweep_ordered(built, monkeypatch, name, fp32):
    """Coarse levels swept from their lists at any size, no single-workgroup
    tail (AH_LIST_MIN=0, AH_TAIL_MAX=0), scalar AIR: their sweeps read a copy
    of the rows' entries in sweep order (F rows, then C rows).  The sums per
    row are those of the list sweeps over the CSR (AH_SWO=0), so the cycle and
    the solve agree bit for bit; the cycle also against the oracle's."""
    from paper_2010_11130_amd import Hierarchy
    print("case", name, fp32, flush=True)
    monkeypatch.setenv("AH_LIST_MIN", "0")
    monkeypatch.setenv("AH_TAIL_MAX", "0")
    g, o = built(name)
    prec = 1 if fp32 else 0
    r = torch.as_tensor(np.random.default_rng(53).standard_normal(g.n), device="cuda")
    out = {}
    for swo in ("1", "0"):
        monkeypatch.setenv("AH_SWO", swo)
        H = Hierarchy(g, max_coarse=SMALL_COARSE, fp32_cycle=prec)
        z = H.vcycle(r, precision=prec).cpu().numpy()
        x, info = H.solve(tol=1e-10, precision=prec)
        assert info["converged"]
        out[swo] = (z, x.cpu().numpy(), info["iters"])
    assert np.array_equal(out["1"][0], out["0"][0])
    assert np.array_equal(out["1"][1], out["0"][1])
    assert out["1"][2] == out["0"][2]
    if not fp32:
        OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE)
        zo = oair.vcycle(OH, r.cpu().numpy())
        assert np.linalg.norm(out["1"][0] - zo) <= 1e-10 * np.linalg.norm(zo)
