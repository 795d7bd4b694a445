"""Ruge-Stueben first-pass coarsening (the single-process form of the
Falgout coarsening of Section 4, ``coarsening=1``) on the HIP path against
the oracle's: C/F splitting and one-point interpolation bit for bit on every
level, lAIR restriction and coarse matrices to 1e-10, solutions at tol 1e-12
to 1e-10, iteration counts at the workload tolerance within +-1."""
import numpy as np
import pytest

from oracle import air as oair
from oracle.drivers import setup_problem, air_fgmres_solve
from gpu_cases import case, gpu_system, to_scipy, rel_sparse_diff

pytestmark = pytest.mark.gpu

SMALL_COARSE = 40


@pytest.mark.parametrize("name", ["c1", "slab", "kuhn_nu4", "kuhn_nu2", "c5", "layer"])
def test_rs_hierarchy_and_solve_parity(name):
    from paper_2010_11130_amd import Hierarchy
    print("case", name, flush=True)
    v, c, prob, p = case(name)
    g = gpu_system(v, c, prob, p)
    o = setup_problem(v, c, prob, p)
    H = Hierarchy(g, max_coarse=SMALL_COARSE, coarsening=1)
    OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE, coarsening="rs")
    assert H.info["levels"] == OH.nlev
    assert H.info["n"] == [lev.A.shape[0] for lev in OH.levels]
    for l in range(OH.nlev - 1):
        lv = H.level(l)
        ol = OH.levels[l]
        assert np.array_equal(lv["cf"].cpu().numpy(), ol.cf), l
        Pd = ol.P.tocsr()
        opc = np.full(ol.A.shape[0], -1)
        opc[np.repeat(np.arange(Pd.shape[0]), np.diff(Pd.indptr))] = Pd.indices
        assert np.array_equal(lv["pcol"].cpu().numpy(), opc), l
        R = to_scipy(lv["Rptr"], lv["Rcol"], lv["Rval"], ol.R.shape[0], ol.R.shape[1])
        assert rel_sparse_diff(R, ol.R) < 1e-10, l
        nxt = H.level(l + 1)
        Ac = to_scipy(nxt["rowptr"], nxt["col"], nxt["val"], nxt["n"])
        assert rel_sparse_diff(Ac, OH.levels[l + 1].A) < 1e-10, l
    x, info = H.solve(tol=1e-12)
    xo, _ = air_fgmres_solve(o, tol=1e-12, hier=OH)
    assert info["converged"]
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
    tol = 1e-10 if name.startswith("c1") else 1e-8
    _, i8 = H.solve(tol=tol)
    _, io8 = air_fgmres_solve(o, tol=tol, hier=OH)
    assert abs(i8["iters"] - io8["iters"]) <= 1, (i8["iters"], io8["iters"])
