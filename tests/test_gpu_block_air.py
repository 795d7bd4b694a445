"""Block AIR on level 0 (``block_air=1``: the facet blocks are the unknowns of
the coarsening, coarser levels scalar) on the HIP path against the oracle's:
C/F splitting and one-point interpolation bit for bit on every level, lAIR
restriction and coarse matrices to 1e-10, solutions at tol 1e-12 to 1e-10,
iteration counts at the workload tolerance within +-1; with a separate
restriction threshold too; and the parameter checks of the entry point."""
import numpy as np
import pytest

from oracle import air as oair
from oracle.drivers import setup_problem, air_fgmres_solve
from gpu_cases import case, gpu_system, to_scipy, rel_sparse_diff

pytestmark = pytest.mark.gpu

SMALL_COARSE = 40


def _compare(H, OH):
    assert H.info["levels"] == OH.nlev
    assert H.info["n"] == [lev.A.shape[0] for lev in OH.levels]
    assert H.info["n_fallback"] == OH.n_fallback
    for l in range(OH.nlev - 1):
        lv = H.level(l)
        ol = OH.levels[l]
        assert np.array_equal(lv["cf"].cpu().numpy(), ol.cf), l
        Pd = ol.P.tocsr()
        assert np.all(np.diff(Pd.indptr) <= 1)
        opc = np.full(ol.A.shape[0], -1)
        opc[np.repeat(np.arange(Pd.shape[0]), np.diff(Pd.indptr))] = Pd.indices
        assert np.array_equal(lv["pcol"].cpu().numpy(), opc), l
        R = to_scipy(lv["Rptr"], lv["Rcol"], lv["Rval"], ol.R.shape[0], ol.R.shape[1])
        assert rel_sparse_diff(R, ol.R) < 1e-10, l
        nxt = H.level(l + 1)
        Ac = to_scipy(nxt["rowptr"], nxt["col"], nxt["val"], nxt["n"])
        assert rel_sparse_diff(Ac, OH.levels[l + 1].A) < 1e-10, l


@pytest.mark.parametrize("name", ["c1", "slab", "kuhn_nu4", "kuhn_nu2", "c5", "layer"])
def test_block_air_hierarchy_and_solve_parity(name):
    from paper_2010_11130_amd import Hierarchy
    print("case", name, flush=True)
    v, c, prob, p = case(name)
    g = gpu_system(v, c, prob, p)
    o = setup_problem(v, c, prob, p)
    H = Hierarchy(g, max_coarse=SMALL_COARSE, block_air=1)
    OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE, block_air=True, block=o.b)
    # every row of a level-0 block shares its block's label
    cf0 = H.level(0)["cf"].cpu().numpy().reshape(-1, o.b)
    assert np.all(cf0 == cf0[:, :1])
    _compare(H, OH)
    x, info = H.solve(tol=1e-12)
    xo, _ = air_fgmres_solve(o, tol=1e-12, hier=OH)
    assert info["converged"]
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
    tol = 1e-10 if name.startswith("c1") else 1e-8
    _, i8 = H.solve(tol=tol)
    _, io8 = air_fgmres_solve(o, tol=tol, hier=OH)
    assert abs(i8["iters"] - io8["iters"]) <= 1, (i8["iters"], io8["iters"])


def test_block_air_restriction_threshold():
    from paper_2010_11130_amd import Hierarchy
    v, c, prob, p = case("kuhn_nu4")
    print("case kuhn_nu4 theta 0.2 theta_r 0.3", flush=True)
    g = gpu_system(v, c, prob, p)
    o = setup_problem(v, c, prob, p)
    H = Hierarchy(g, max_coarse=SMALL_COARSE, block_air=1, theta=0.2, theta_r=0.3)
    OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE, block_air=True, block=o.b, theta=0.2, theta_r=0.3)
    _compare(H, OH)


def test_block_air_rejects_unsupported_settings():
    from paper_2010_11130_amd import Hierarchy
    from paper_2010_11130_amd._lib import AirHdgError
    v, c, prob, p = case("c1")
    g = gpu_system(v, c, prob, p)
    for kw in ({"lair_distance": 2}, {"coarsening": 1}, {"block_air": 2}):
        kw = dict(kw)
        kw.setdefault("block_air", 1)
        with pytest.raises(AirHdgError):
            Hierarchy(g, **kw)
    gu = gpu_system(v, c, prob, p, block_scale=False)
    with pytest.raises(AirHdgError):
        Hierarchy(gu, block_air=1)


@pytest.mark.parametrize("name", ["c1", "kuhn_nu4", "c5"])
@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("fp32", [False, True])
def test_block_air_vcycle_parity(name, transpose, fp32):
    """One V-cycle of the block-AIR hierarchy and its transpose, FP64 to
    1e-10; the FP32 cycle within a small factor of the oracle's FP32
    emulation of the same cycle."""
    import torch
    from paper_2010_11130_amd import Hierarchy
    print("case", name, transpose, fp32, flush=True)
    v, c, prob, p = case(name)
    g = gpu_system(v, c, prob, p)
    o = setup_problem(v, c, prob, p)
    H = Hierarchy(g, max_coarse=SMALL_COARSE, block_air=1, adjoint=1, fp32_cycle=1 if fp32 else 0)
    OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE, block_air=True, block=o.b)
    r = np.random.default_rng(5).standard_normal(g.n)
    z = H.vcycle(torch.as_tensor(r, device="cuda"), precision=1 if fp32 else 0, transpose=transpose).cpu().numpy()
    zo = oair.vcycle_T(OH, r) if transpose else oair.vcycle(OH, r)
    err = np.linalg.norm(z - zo) / np.linalg.norm(zo)
    if not fp32:
        assert err <= 1e-10
        return
    z32 = oair.vcycle_T(OH, r, dtype=np.float32) if transpose else oair.vcycle(OH, r, dtype=np.float32)
    err32 = np.linalg.norm(z32.astype(np.float64) - zo) / np.linalg.norm(zo)
    print("fp32 cycle error: hip %.3e  emulated %.3e" % (err, err32), flush=True)
    assert err32 < 1e-5
    assert err <= 4.0 * err32 + 1e-12


@pytest.mark.parametrize("precision", [0, 1])
def test_block_air_adjoint_solve(precision):
    """The adjoint solve S^T lam = g with the transposed block-AIR hierarchy
    against the oracle's dense adjoint, FP64 and FP32 cycles."""
    import torch
    from oracle import adjoint as oadj
    from oracle.drivers import direct_solve
    from paper_2010_11130_amd import Hierarchy
    v, c, prob, p = case("c5")
    print("case c5 adjoint precision", precision, flush=True)
    g = gpu_system(v, c, prob, p)
    o = setup_problem(v, c, prob, p)
    H = Hierarchy(g, max_coarse=SMALL_COARSE, block_air=1, adjoint=1, fp32_cycle=precision)
    target = direct_solve(o) + 0.1 * np.random.default_rng(9).standard_normal(o.n)
    lam, info = H.solve(tol=1e-13, precision=precision)
    assert info["converged"]
    gvec = lam - torch.as_tensor(target, device="cuda")
    adj, ainfo = H.solve_adjoint(gvec, tol=1e-13, precision=precision)
    assert ainfo["converged"]
    adj_o = oadj.adjoint_direct(o, direct_solve(o) - target)
    assert np.linalg.norm(adj.cpu().numpy() - adj_o) <= 1e-9 * np.linalg.norm(adj_o)


@pytest.fixture
def level1_lists(monkeypatch):
    """Coarse levels swept from their F and C lists at any size and no
    single-workgroup tail, so level 1 of the small cases takes the sweeps of
    the large ones (read by full blocks under block AIR)."""
    monkeypatch.setenv("AH_LIST_MIN", "0")
    monkeypatch.setenv("AH_TAIL_MAX", "0")


@pytest.mark.parametrize("name", ["kuhn_nu4", "c5", "slab"])
@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("lanes", ["auto", "8"])
def test_block_air_level1_full_block_sweeps(level1_lists, monkeypatch, name, fp32, lanes):
    """Level 1 under block AIR is made of b x b blocks; its sweeps read it by
    full blocks (one column index per block; the CSR values in place where
    the rows of a block row share one block pattern, a zero-filled side array
    elsewhere), a lane per block (lanes per row by precision, or 8).  One V-cycle
    against the oracle's (FP64 1e-10; FP32 within 4x the oracle's FP32
    emulation), the same cycle with the copy switched off (AH_L1B=0, the CSR
    sweeps) to 1e-13 in FP64, and the solution and iteration count against
    the oracle's solve."""
    import torch
    from paper_2010_11130_amd import Hierarchy
    print("case", name, fp32, lanes, flush=True)
    if lanes != "auto":
        monkeypatch.setenv("AH_L1LP", lanes)
    v, c, prob, p = case(name)
    g = gpu_system(v, c, prob, p)
    o = setup_problem(v, c, prob, p)
    prec = 1 if fp32 else 0
    H = Hierarchy(g, max_coarse=SMALL_COARSE, block_air=1, fp32_cycle=prec)
    assert H.info["levels"] > 2
    nnz1 = H.info["nnz"][1]
    assert nnz1 <= H.info["block_view_values"] <= 1.25 * nnz1, (H.info["block_view_values"], nnz1)
    OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE, block_air=True, block=o.b)
    r = np.random.default_rng(7).standard_normal(g.n)
    z = H.vcycle(torch.as_tensor(r, device="cuda"), precision=prec).cpu().numpy()
    zo = oair.vcycle(OH, r)
    err = np.linalg.norm(z - zo) / np.linalg.norm(zo)
    monkeypatch.setenv("AH_L1B", "0")
    Hc = Hierarchy(g, max_coarse=SMALL_COARSE, block_air=1, fp32_cycle=prec)
    assert Hc.info["block_view_values"] == 0
    zc = Hc.vcycle(torch.as_tensor(r, device="cuda"), precision=prec).cpu().numpy()
    if fp32:
        z32 = oair.vcycle(OH, r, dtype=np.float32)
        err32 = np.linalg.norm(z32.astype(np.float64) - zo) / np.linalg.norm(zo)
        print("fp32 cycle error: full blocks %.3e  csr %.3e  emulated %.3e"
              % (err, np.linalg.norm(zc - zo) / np.linalg.norm(zo), err32), flush=True)
        assert err <= 4.0 * err32 + 1e-12
    else:
        assert err <= 1e-10
        assert np.linalg.norm(z - zc) <= 1e-13 * np.linalg.norm(zc)
    x, info = H.solve(tol=1e-12 if not fp32 else 1e-10, precision=prec)
    assert info["converged"]
    xo, io = air_fgmres_solve(o, tol=1e-12, hier=OH)
    assert np.linalg.norm(x.cpu().numpy() - xo) <= (1e-10 if not fp32 else 1e-8) * np.linalg.norm(xo)
    if not fp32:
        _, i8 = H.solve(tol=1e-8)
        _, io8 = air_fgmres_solve(o, tol=1e-8, hier=OH)
        assert abs(i8["iters"] - io8["iters"]) <= 1, (i8["iters"], io8["iters"])


@pytest.mark.parametrize("name", ["kuhn_nu4", "c5", "slab"])
@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("level1", [False, True])
def test_block_air_sweep_ordered_level0(monkeypatch, name, fp32, level1):
    """Level 0 under block AIR is swept from a copy with its block rows in
    sweep order (F blocks, then C blocks), reading the interpolated
    correction from the coarse vector and the F blocks' values from compact
    vectors, and level 1 (when it is read by full blocks: ``level1``, coarse
    levels swept from their lists at any size) from a copy of its F rows,
    then its C rows.  The sums per row are the same as over the natural order
    with the F and C lists after an interpolation pass (AH_SWO=0), so the
    cycle and the solve agree bit for bit; the cycle also against the
    oracle's."""
    import torch
    from paper_2010_11130_amd import Hierarchy
    print("case", name, fp32, level1, flush=True)
    if level1:
        monkeypatch.setenv("AH_LIST_MIN", "0")
        monkeypatch.setenv("AH_TAIL_MAX", "0")
    v, c, prob, p = case(name)
    g = gpu_system(v, c, prob, p)
    o = setup_problem(v, c, prob, p)
    prec = 1 if fp32 else 0
    r = torch.as_tensor(np.random.default_rng(11).standard_normal(g.n), device="cuda")
    out = {}
    for swo in ("1", "0"):
        monkeypatch.setenv("AH_SWO", swo)
        H = Hierarchy(g, max_coarse=SMALL_COARSE, block_air=1, fp32_cycle=prec)
        assert (H.info["block_view_values"] > 0) == level1
        # the copy in sweep order comes with the sweeps that read P e_c from e_c
        assert H.info["level0_no_interp_pass"] == (1 if swo == "1" else 0)
        z = H.vcycle(r, precision=prec).cpu().numpy()
        x, info = H.solve(tol=1e-10, precision=prec)
        assert info["converged"]
        out[swo] = (z, x.cpu().numpy(), info["iters"])
    assert np.array_equal(out["1"][0], out["0"][0])
    assert np.array_equal(out["1"][1], out["0"][1])
    assert out["1"][2] == out["0"][2]
    if not fp32:
        OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE, block_air=True, block=o.b)
        zo = oair.vcycle(OH, r.cpu().numpy())
        assert np.linalg.norm(out["1"][0] - zo) <= 1e-10 * np.linalg.norm(zo)


@pytest.mark.parametrize("name", ["kuhn_nu4", "c5"])
@pytest.mark.parametrize("level1", [False, True])
def test_block_air_single_f_sweep(monkeypatch, name, level1):
    """Block AIR with one F sweep per level (relax = 1, the oracle's "F"):
    the sweep-ordered level-0 copy and (``level1``) level 1 by full blocks
    stop after their first sweep.  One V-cycle against the oracle's to 1e-10
    and the solve to 1e-10 of the oracle's."""
    import torch
    from paper_2010_11130_amd import Hierarchy
    print("case", name, level1, flush=True)
    if level1:
        monkeypatch.setenv("AH_LIST_MIN", "0")
        monkeypatch.setenv("AH_TAIL_MAX", "0")
    v, c, prob, p = case(name)
    g = gpu_system(v, c, prob, p)
    o = setup_problem(v, c, prob, p)
    H = Hierarchy(g, max_coarse=SMALL_COARSE, block_air=1, relax=1)
    assert (H.info["block_view_values"] > 0) == level1
    OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE, block_air=True, block=o.b, relax="F")
    r = np.random.default_rng(13).standard_normal(g.n)
    z = H.vcycle(torch.as_tensor(r, device="cuda")).cpu().numpy()
    zo = oair.vcycle(OH, r)
    assert np.linalg.norm(z - zo) <= 1e-10 * np.linalg.norm(zo)
    x, info = H.solve(tol=1e-12)
    xo, io = air_fgmres_solve(o, tol=1e-12, hier=OH)
    assert info["converged"]
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)


@pytest.mark.parametrize("name", ["kuhn_nu4", "kuhn_nu2", "c5", "slab"])
def test_block_air_restriction_by_blocks(monkeypatch, name):
    """Under block AIR the level-0 restriction R = [Z I] runs by coarse blocks
    (Z's b x b blocks, one column index per block, the identity on the
    block's own rows).  One V-cycle against the CSR restriction (AH_RZB=0)
    to 1e-13 (the sums differ in order only) and against the oracle's to
    1e-10, in FP64; the FP32 cycle within 4x the oracle's FP32 emulation;
    the solve to 1e-10 of the oracle's."""
    import torch
    from paper_2010_11130_amd import Hierarchy
    print("case", name, flush=True)
    v, c, prob, p = case(name)
    g = gpu_system(v, c, prob, p)
    o = setup_problem(v, c, prob, p)
    r = torch.as_tensor(np.random.default_rng(17).standard_normal(g.n), device="cuda")
    z = {}
    for rzb in ("1", "0"):
        monkeypatch.setenv("AH_RZB", rzb)
        H = Hierarchy(g, max_coarse=SMALL_COARSE, block_air=1, fp32_cycle=1)
        z[rzb] = (H.vcycle(r).cpu().numpy(), H.vcycle(r, precision=1).cpu().numpy())
        if rzb == "1":
            x, info = H.solve(tol=1e-12)
    OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE, block_air=True, block=o.b)
    zo = oair.vcycle(OH, r.cpu().numpy())
    assert np.linalg.norm(z["1"][0] - z["0"][0]) <= 1e-13 * np.linalg.norm(z["0"][0])
    assert np.linalg.norm(z["1"][0] - zo) <= 1e-10 * np.linalg.norm(zo)
    z32 = oair.vcycle(OH, r.cpu().numpy(), dtype=np.float32).astype(np.float64)
    err32 = np.linalg.norm(z32 - zo) / np.linalg.norm(zo)
    assert np.linalg.norm(z["1"][1] - zo) / np.linalg.norm(zo) <= 4.0 * err32 + 1e-12
    xo, io = air_fgmres_solve(o, tol=1e-12, hier=OH)
    assert info["converged"]
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
