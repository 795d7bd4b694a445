"""HIP path vs oracle, element by element on the same seeded inputs.

Tolerances (FP64 everywhere unless stated):
  * assembled scaled matrix, right-hand side, inverse facet blocks,
    Dirichlet traces: 1e-12 relative to the largest entry (different element
    bases and summation orders on the two sides; cond(A_K) <~ 1e3);
  * C/F splitting, one-point interpolation columns: bit-exact (integers);
  * lAIR restriction and coarse matrices: 1e-10 relative (they inherit the
    level matrices' rounding through small dense solves);
  * one V-cycle: 1e-10 relative; FP32 cycle: within 4x the error of the
    oracle's FP32 emulation of the same cycle (a few 1e-7);
  * solution at tol 1e-12: 1e-10 relative; iterations at the workload
    tolerance within +-1;
  * FP32 cycle: solution within 1e-8 of the FP64 oracle at tol 1e-10.
"""
import numpy as np
import pytest
import torch

from oracle import air as oair, krylov as okry, adjoint as oadj
from oracle.drivers import setup_problem, air_fgmres_solve, direct_solve, problem_g
from oracle.hdg import reconstruct as oreconstruct
from gpu_cases import case, gpu_system, to_scipy, rel_sparse_diff

pytestmark = pytest.mark.gpu

CASES = ["c1", "c1_p3", "slab", "slab_nu0", "kuhn_nu0", "kuhn_nu4", "kuhn_nu2", "c5", "kuhn_p3", "layer", "layer_p2"]
SMALL_COARSE = 40


def _both(name):
    v, c, prob, p = case(name)
    g = gpu_system(v, c, prob, p)
    o = setup_problem(v, c, prob, p)
    return g, o, prob


@pytest.fixture(scope="module")
def built():
    cache = {}

    def get(name):
        if name not in cache:
            cache[name] = _both(name)
        return cache[name]
    return get


@pytest.mark.parametrize("name", CASES)
def test_assembly_parity(built, name):
    print("case", name, flush=True)
    g, o, _ = built(name)
    assert g.n == o.n
    ex = g.export()
    S = to_scipy(ex["rowptr"], ex["col"], ex["val"], g.n)
    assert rel_sparse_diff(S, o.Shat) < 1e-12
    hh = ex["hhat"].cpu().numpy()
    assert np.abs(hh - o.Hhat).max() <= 1e-12 * max(np.abs(o.Hhat).max(), 1e-300)
    dinv = ex["dinv"].cpu().numpy()
    assert np.abs(dinv - o.Dinv).max() <= 1e-11 * np.abs(o.Dinv).max()
    lamd = ex["lam_dir"].cpu().numpy()
    assert np.abs(lamd - o.lamD_full).max() <= 1e-12 * max(np.abs(o.lamD_full).max(), 1.0)


@pytest.mark.parametrize("name", CASES)
def test_hierarchy_parity(built, name):
    from paper_2010_11130_amd import Hierarchy
    print("case", name, flush=True)
    g, o, _ = built(name)
    H = Hierarchy(g, max_coarse=SMALL_COARSE)
    OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE)
    assert H.info["levels"] == OH.nlev
    assert H.info["n"] == [lev.A.shape[0] for lev in OH.levels]
    for l in range(OH.nlev):
        lv = H.level(l)
        A = to_scipy(lv["rowptr"], lv["col"], lv["val"], lv["n"])
        assert rel_sparse_diff(A, OH.levels[l].A) < (1e-12 if l == 0 else 1e-10), l
        if l + 1 < OH.nlev:
            ol = OH.levels[l]
            assert np.array_equal(lv["cf"].cpu().numpy(), ol.cf), l
            pc = lv["pcol"].cpu().numpy()
            Pd = ol.P.tocsr()
            opc = np.full(ol.A.shape[0], -1)
            rows = np.repeat(np.arange(Pd.shape[0]), np.diff(Pd.indptr))
            opc[rows] = Pd.indices
            assert np.array_equal(pc, opc), l
            R = to_scipy(lv["Rptr"], lv["Rcol"], lv["Rval"], ol.R.shape[0], ol.R.shape[1])
            assert rel_sparse_diff(R, ol.R) < 1e-10, l


@pytest.fixture(params=["tail", "tail_global", "notail"])
def tail_mode(request, monkeypatch):
    """Run the coarse end of the cycle in the single-workgroup kernel (levels
    up to 6000 rows) from its LDS image or from global memory, or level by
    level with grid-wide kernels."""
    monkeypatch.setenv("AH_TAIL_MAX", "0" if request.param == "notail" else "6000")
    monkeypatch.setenv("AH_TAIL_LDS", "0" if request.param == "tail_global" else "1")
    return request.param


@pytest.mark.parametrize("name", ["c1", "slab", "kuhn_nu4", "c5"])
@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("fp32", [False, True])
def test_vcycle_parity(built, name, transpose, fp32, tail_mode):
    from paper_2010_11130_amd import Hierarchy
    print("case", name, transpose, fp32, tail_mode, flush=True)
    g, o, _ = built(name)
    H = Hierarchy(g, max_coarse=SMALL_COARSE, adjoint=1, fp32_cycle=1 if fp32 else 0)
    OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE)
    r = np.random.default_rng(5).standard_normal(g.n)
    z = H.vcycle(torch.as_tensor(r, device="cuda"), precision=1 if fp32 else 0,
                 transpose=transpose).cpu().numpy()
    zo = oair.vcycle_T(OH, r) if transpose else oair.vcycle(OH, r)
    err = np.linalg.norm(z - zo) / np.linalg.norm(zo)
    if not fp32:
        assert err <= 1e-10
        return
    # FP32 cycle: the tolerance is what FP32 arithmetic gives for this cycle
    # on this input, measured by the oracle's FP32 emulation of the same
    # cycle (operators rounded to FP32, FP32 accumulation, FP64 coarsest
    # solve).  The HIP path rounds in another order (fused multiply-adds,
    # other summation orders), so it may differ from the emulation by errors
    # of the same size, not by more than a small factor.
    z32 = (oair.vcycle_T(OH, r, dtype=np.float32) if transpose else oair.vcycle(OH, r, dtype=np.float32))
    err32 = np.linalg.norm(z32.astype(np.float64) - zo) / np.linalg.norm(zo)
    print("fp32 cycle error: hip %.3e  emulated %.3e" % (err, err32), flush=True)
    assert err32 < 1e-5
    assert err <= 4.0 * err32 + 1e-12


@pytest.mark.parametrize("name", CASES)
def test_solve_parity(built, name, tail_mode):
    from paper_2010_11130_amd import Hierarchy
    print("case", name, tail_mode, flush=True)
    g, o, _ = built(name)
    H = Hierarchy(g, max_coarse=SMALL_COARSE)
    x, info = H.solve(tol=1e-12)
    OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE)
    xo, io = air_fgmres_solve(o, tol=1e-12, hier=OH)
    xg = x.cpu().numpy()
    assert info["converged"]
    assert np.linalg.norm(xg - xo) <= 1e-10 * np.linalg.norm(xo)
    tol = 1e-10 if name.startswith("c1") else 1e-8
    _, i8 = H.solve(tol=tol)
    _, io8 = air_fgmres_solve(o, tol=tol, hier=OH)
    assert abs(i8["iters"] - io8["iters"]) <= 1, (i8["iters"], io8["iters"])


@pytest.mark.parametrize("name", ["c1", "slab", "slab_nu0", "kuhn_nu0", "kuhn_nu4"])
def test_fp32_cycle_accuracy(built, name):
    from paper_2010_11130_amd import Hierarchy
    print("case", name, flush=True)
    g, o, _ = built(name)
    H = Hierarchy(g, max_coarse=SMALL_COARSE, fp32_cycle=1)
    x, info = H.solve(tol=1e-10, precision=1)
    xo = direct_solve(o)
    assert info["converged"]
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-8 * np.linalg.norm(xo)


@pytest.mark.parametrize("name", ["c1", "slab", "kuhn_nu2", "c5"])
def test_reconstruct_parity(built, name):
    print("case", name, flush=True)
    g, o, _ = built(name)
    xo = direct_solve(o)
    U = g.reconstruct(torch.as_tensor(xo, device="cuda")).cpu().numpy()
    Uo = oreconstruct(o, xo)
    assert np.abs(U - Uo).max() <= 1e-10 * np.abs(Uo).max()


def test_empty_free_set():
    from paper_2010_11130_amd import Hierarchy
    v, c, prob, p = case("one_tet")
    g = gpu_system(v, c, prob, p)
    assert g.n == 0
    H = Hierarchy(g)
    x, info = H.solve(tol=1e-10)
    assert info["converged"] and info["iters"] == 0


def test_single_level_direct():
    from paper_2010_11130_amd import Hierarchy
    v, c, prob, p = case("c1")
    g = gpu_system(v, c, prob, p)
    H = Hierarchy(g, max_coarse=5000)
    assert H.info["levels"] == 1
    x, info = H.solve(tol=1e-12)
    o = setup_problem(v, c, prob, p)
    xo = direct_solve(o)
    assert info["iters"] == 1
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)


def test_adjoint_and_gradients_c5(built):
    from paper_2010_11130_amd import Hierarchy
    g, o, prob = built("c5")
    H = Hierarchy(g, max_coarse=SMALL_COARSE, adjoint=1)
    lam, _ = H.solve(tol=1e-13)
    rng = np.random.default_rng(9)
    target = direct_solve(o) + 0.1 * rng.standard_normal(o.n)
    gvec = lam - torch.as_tensor(target, device="cuda")
    adj, info = H.solve_adjoint(gvec, tol=1e-13)
    assert info["converged"]
    lam_o = direct_solve(o)
    adj_o = oadj.adjoint_direct(o, lam_o - target)
    assert np.linalg.norm(adj.cpu().numpy() - adj_o) <= 1e-9 * np.linalg.norm(adj_o)
    dq, dnu = g.grad(lam, adj)
    g_fn = problem_g(prob, o.mesh, o.kinds, 0.0, 1.0)
    J, dc_o, dnu_o, _ = oadj.misfit_and_grads(o, lam_o, target, prob.a, prob.f, g_fn, prob.basis)
    assert abs(dnu - dnu_o) <= 1e-8 * abs(dnu_o)
    # source gradient: contract dJ/df_q with the Gaussian basis on the device
    from paper_2010_11130_amd import source_gauss_T
    xe, _ = g.mesh.quad_points(g.p)
    dc = source_gauss_T(xe.reshape(-1, 3), prob.centers, prob.width, dq.reshape(-1)).cpu().numpy()
    assert np.abs(dc - dc_o).max() <= 1e-8 * np.abs(dc_o).max()


def _gpu_march(mesh_fn, slabs, prob, p, tol=1e-12, same_mesh=False, dt=None):
    """Slab march on the HIP path: per slab assemble (inflow = previous trace),
    set up, solve."""
    from paper_2010_11130_amd import Mesh, System, Hierarchy
    from gpu_cases import boundary_data, kinds_for
    lams = []
    prev = None
    mesh0 = None
    for k in range(slabs):
        if same_mesh and mesh0 is not None:
            m, v, fv, bf, kinds, xb0 = mesh0
        else:
            v, c = mesh_fn(k)
            m = Mesh(v, c)
            fv, _ = m.facets()
            bf = m.boundary_facets()
            isb = np.zeros(m.nf, dtype=bool)
            isb[bf] = True
            kinds = kinds_for(v, fv, isb)
            m.set_bc(kinds)
            _, xb0 = m.quad_points(p)
            mesh0 = (m, v, fv, bf, kinds, xb0)
        xb = xb0.clone()
        if same_mesh:
            xb[..., 0] += k * dt
            vs = v.copy()
            vs[:, 0] += k * dt
        else:
            vs = v
        g = boundary_data(prob, vs, fv, bf, kinds, xb)
        if prev is not None:
            prev[0].trace_to_inflow(prev[1], m, g)
        a = torch.as_tensor(np.ascontiguousarray(prob.a_vertices(vs)), device="cuda")
        s = System(m, p, prob.nu, a, None, g)
        H = Hierarchy(s, max_coarse=SMALL_COARSE)
        x, info = H.solve(tol=tol)
        assert info["converged"]
        lams.append(x.cpu().numpy())
        prev = (s, x)
    return lams


def test_slab_march_parity_fixed_mesh():
    from workloads import slab_prism_tet_mesh
    from workloads.problems import slab_hill
    from oracle.drivers import solve_slabs
    n, S, p, dt = 8, 4, 2, 1.0 / 64
    prob = slab_hill(1e-4)
    lg = _gpu_march(lambda k: slab_prism_tet_mesh(n, dt), S, prob, p, same_mesh=True, dt=dt)
    _, _, lo = solve_slabs(lambda k: slab_prism_tet_mesh(n, dt, t0=k * dt), S, prob, p, err=False)
    for k in range(S):
        assert np.linalg.norm(lg[k] - lo[k]) <= 1e-10 * np.linalg.norm(lo[k]), k


def test_slab_march_parity_moving_mesh():
    from workloads import pulse_slab_mesh
    from workloads.problems import paper_pulse
    from oracle.drivers import solve_slabs
    N, S, p = 4, 3, 2
    prob = paper_pulse(1e-2)
    lg = _gpu_march(lambda k: pulse_slab_mesh(N, k), S, prob, p)
    _, _, lo = solve_slabs(lambda k: pulse_slab_mesh(N, k), S, prob, p, err=False)
    for k in range(S):
        assert np.linalg.norm(lg[k] - lo[k]) <= 1e-10 * np.linalg.norm(lo[k]), k


@pytest.mark.parametrize("max_coarse", [40, 100, 200])
def test_coarsest_solver_paths(max_coarse):
    """The coarsest level is inverted by Gauss-Jordan in LDS (n <= 64), LU in
    LDS (n <= 128) or in global memory; each path against the oracle."""
    from paper_2010_11130_amd import Hierarchy
    v, c, prob, p = case("slab")
    g = gpu_system(v, c, prob, p)
    o = setup_problem(v, c, prob, p)
    H = Hierarchy(g, max_coarse=max_coarse)
    OH = oair.setup(o.Shat, max_coarse=max_coarse)
    assert H.info["n"] == [lev.A.shape[0] for lev in OH.levels]
    print("coarsest", H.info["n"][-1], flush=True)
    r = np.random.default_rng(2).standard_normal(g.n)
    z = H.vcycle(torch.as_tensor(r, device="cuda")).cpu().numpy()
    zo = oair.vcycle(OH, r)
    assert np.linalg.norm(z - zo) <= 1e-10 * np.linalg.norm(zo)


def test_update_neumann_reproduces_assembly():
    """Assembling with other Neumann data and then setting the data with
    hdg_update_neumann gives the right-hand side of a direct assembly bit for
    bit (both routes add the Neumann term in the same kernel), and the
    Neumann term matters (the other data give another right-hand side)."""
    from paper_2010_11130_amd import System
    v, c, prob, p = case("slab")
    s1 = gpu_system(v, c, prob, p)
    m, xe, xb, f, g, a = s1._keep_alive
    kb = torch.as_tensor(m.kind[m.boundary_facets()], device="cuda")[:, None]
    g_other = torch.where(kb == 2, torch.full_like(g, 0.37), g).contiguous()
    s2 = System(m, p, prob.nu, a, f, g_other)
    h_other = s2.export()["hhat"].clone()
    s2.update_neumann(g)
    e1, e2 = s1.export(), s2.export()
    assert torch.equal(e1["hhat"], e2["hhat"])
    assert torch.equal(e1["val"], e2["val"])
    assert not torch.equal(h_other, e1["hhat"])
    # the matrix did not change, so a hierarchy of s2 solves the new data
    o = setup_problem(v, c, prob, p)
    assert np.abs(e2["hhat"].cpu().numpy() - o.Hhat).max() <= 1e-12 * np.abs(o.Hhat).max()


def _march_inputs(n, S, p, dt, prob):
    from paper_2010_11130_amd import Mesh
    from gpu_cases import boundary_data, kinds_for
    from workloads import slab_prism_tet_mesh
    v, c = slab_prism_tet_mesh(n, dt)
    m = Mesh(v, c)
    fv, _ = m.facets()
    bf = m.boundary_facets()
    isb = np.zeros(m.nf, dtype=bool)
    isb[bf] = True
    kinds = kinds_for(v, fv, isb)
    m.set_bc(kinds)
    _, xb0 = m.quad_points(p)
    gs = []
    for k in range(S):
        xb = xb0.clone()
        xb[..., 0] += k * dt
        vs = v.copy()
        vs[:, 0] += k * dt
        gs.append(boundary_data(prob, vs, fv, bf, kinds, xb))
    a = torch.as_tensor(np.ascontiguousarray(prob.a_vertices(v)), device="cuda")
    return m, a, gs


@pytest.mark.parametrize("precision", [0, 1])
def test_pipelined_march_matches_sequential_and_oracle(precision):
    """The two-stream march (slab k+1 assembled and set up on a second stream
    while slab k solves) equals the sequential march bit for bit, and both
    match the oracle's slab march."""
    from paper_2010_11130_amd import SlabMarch
    from workloads import slab_prism_tet_mesh
    from workloads.problems import slab_hill
    from oracle.drivers import solve_slabs
    n, S, p, dt = 8, 5, 2, 1.0 / 64
    prob = slab_hill(1e-4)
    res = {}
    for pipelined in (False, True):
        m, a, gs = _march_inputs(n, S, p, dt, prob)
        lams = []
        march = SlabMarch(m, p, prob.nu, a, air_kw={"max_coarse": SMALL_COARSE, "fp32_cycle": precision},
                          solve_kw={"tol": 1e-12, "precision": precision})
        march.run(gs, pipelined=pipelined, on_slab=lambda k, s, h, x, info: lams.append(x.clone()))
        torch.cuda.synchronize()
        res[pipelined] = [x.cpu().numpy() for x in lams]
        print("pipelined", pipelined, "slabs", len(lams), flush=True)
    for k in range(S):
        assert np.array_equal(res[False][k], res[True][k]), k
    _, _, lo = solve_slabs(lambda k: slab_prism_tet_mesh(n, dt, t0=k * dt), S, prob, p, err=False)
    tol = 1e-10 if precision == 0 else 1e-8
    for k in range(S):
        assert np.linalg.norm(res[True][k] - lo[k]) <= tol * np.linalg.norm(lo[k]), k


@pytest.mark.parametrize("name", ["c1", "slab", "kuhn_nu4", "c5"])
def test_bicgstab_parity(built, name):
    """BiCGSTAB (the paper's Krylov method) against the oracle's: solution at
    tol 1e-12, steps at the workload tolerance within one."""
    from paper_2010_11130_amd import Hierarchy
    from oracle.drivers import air_bicgstab_solve
    print("case", name, flush=True)
    g, o, _ = built(name)
    H = Hierarchy(g, max_coarse=SMALL_COARSE)
    OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE)
    x, info = H.solve(tol=1e-12, method=1)
    xo, io = air_bicgstab_solve(o, tol=1e-12, hier=OH)
    assert info["converged"] and io["converged"]
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
    tol = 1e-10 if name.startswith("c1") else 1e-8
    _, i8 = H.solve(tol=tol, method=1)
    _, io8 = air_bicgstab_solve(o, tol=tol, hier=OH)
    assert abs(i8["iters"] - io8["iters"]) <= 1, (i8["iters"], io8["iters"])


def test_bicgstab_fp32_cycle_and_adjoint(built):
    from paper_2010_11130_amd import Hierarchy
    g, o, _ = built("c5")
    H = Hierarchy(g, max_coarse=SMALL_COARSE, fp32_cycle=1, adjoint=1)
    ref = direct_solve(o)
    x, info = H.solve(tol=1e-10, method=1, precision=1)
    assert info["converged"]
    assert np.linalg.norm(x.cpu().numpy() - ref) <= 1e-8 * np.linalg.norm(ref)
    gvec = torch.as_tensor(np.random.default_rng(3).standard_normal(g.n), device="cuda")
    lam, ia = H.solve_adjoint(gvec, tol=1e-12, method=1)
    assert ia["converged"]
    lam_o = oadj.adjoint_direct(o, gvec.cpu().numpy())
    assert np.linalg.norm(lam.cpu().numpy() - lam_o) <= 1e-9 * np.linalg.norm(lam_o)


@pytest.mark.parametrize("name", ["slab", "c1"])
def test_unscaled_system_parity(name):
    """The "no block inverse" system (S unscaled): assembly, hierarchy and one
    V-cycle against the oracle's."""
    from paper_2010_11130_amd import Hierarchy
    v, c, prob, p = case(name)
    g = gpu_system(v, c, prob, p, block_scale=False)
    o = setup_problem(v, c, prob, p, block_scale=False)
    ex = g.export()
    S = to_scipy(ex["rowptr"], ex["col"], ex["val"], g.n)
    assert rel_sparse_diff(S, o.Shat) < 1e-12
    hh = ex["hhat"].cpu().numpy()
    assert np.abs(hh - o.Hhat).max() <= 1e-12 * np.abs(o.Hhat).max()
    assert np.array_equal(ex["dinv"].cpu().numpy(), o.Dinv)
    H = Hierarchy(g, max_coarse=SMALL_COARSE)
    OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE)
    assert H.info["n"] == [lev.A.shape[0] for lev in OH.levels]
    for l in range(OH.nlev - 1):
        assert np.array_equal(H.level(l)["cf"].cpu().numpy(), OH.levels[l].cf), l
    r = np.random.default_rng(6).standard_normal(g.n)
    z = H.vcycle(torch.as_tensor(r, device="cuda")).cpu().numpy()
    zo = oair.vcycle(OH, r)
    assert np.linalg.norm(z - zo) <= 1e-10 * np.linalg.norm(zo)


def test_all_at_once_equals_slab_march_pure_advection():
    """At nu = 0 the all-at-once space-time system on the stacked slabs and the
    slab march (Section 2.4) are the same discrete problem: the last slab's
    element solution agrees.  (With nu > 0 the penalty on the interior time
    planes couples both sides in the all-at-once system only.)"""
    from paper_2010_11130_amd import SlabMarch, Hierarchy
    from workloads import stacked_prism_tet_mesh
    from workloads.problems import slab_hill
    n, S, p, dt = 6, 3, 2, 1.0 / 8
    prob = slab_hill(0.0)
    v, c = stacked_prism_tet_mesh(n, S, T=S * dt)
    g = gpu_system(v, c, prob, p)
    H = Hierarchy(g, max_coarse=SMALL_COARSE)
    x, info = H.solve(tol=1e-13)
    assert info["converged"]
    U = g.reconstruct(x).cpu().numpy()[(S - 1) * 6 * n * n:]
    m, a, gs = _march_inputs(n, S, p, dt, prob)
    out = {}
    march = SlabMarch(m, p, prob.nu, a, air_kw={"max_coarse": SMALL_COARSE}, solve_kw={"tol": 1e-13})
    march.run(gs, pipelined=False, on_slab=lambda k, s, h, xx, inf: out.__setitem__("U", s.reconstruct(xx)))
    Ul = out["U"].cpu().numpy()
    assert np.linalg.norm(U - Ul) <= 1e-10 * np.linalg.norm(Ul)


LAIR_VARIANTS = {"d2": dict(lair_distance=2), "theta_r": dict(theta=0.2, theta_r=0.3),
                 "d2_theta_r": dict(lair_distance=2, theta=0.2, theta_r=0.3)}


@pytest.mark.parametrize("variant", sorted(LAIR_VARIANTS))
@pytest.mark.parametrize("name", ["c1", "slab", "kuhn_nu4", "c5", "layer"])
def test_lair_variant_parity(built, name, variant):
    """Distance-two neighbourhoods and a separate restriction threshold:
    C/F splitting and P bit for bit, R and the coarse operators to 1e-10,
    the solution to 1e-10 and the iteration count within one."""
    from paper_2010_11130_amd import Hierarchy
    print("case", name, variant, flush=True)
    g, o, _ = built(name)
    kw = LAIR_VARIANTS[variant]
    okw = {"theta": kw.get("theta", 0.25), "theta_r": kw.get("theta_r"), "distance": kw.get("lair_distance", 1)}
    H = Hierarchy(g, max_coarse=SMALL_COARSE, **kw)
    OH = oair.setup(o.Shat, max_coarse=SMALL_COARSE, **okw)
    assert H.info["n"] == [lev.A.shape[0] for lev in OH.levels]
    for l in range(OH.nlev - 1):
        lv = H.level(l)
        ol = OH.levels[l]
        assert np.array_equal(lv["cf"].cpu().numpy(), ol.cf), l
        R = to_scipy(lv["Rptr"], lv["Rcol"], lv["Rval"], ol.R.shape[0], ol.R.shape[1])
        assert rel_sparse_diff(R, ol.R) < 1e-10, l
        A = to_scipy(H.level(l + 1)["rowptr"], H.level(l + 1)["col"], H.level(l + 1)["val"], H.info["n"][l + 1])
        assert rel_sparse_diff(A, OH.levels[l + 1].A) < 1e-10, l
    x, info = H.solve(tol=1e-12)
    xo, io = air_fgmres_solve(o, tol=1e-12, hier=OH)
    assert info["converged"]
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
    _, i8 = H.solve(tol=1e-8)
    _, io8 = air_fgmres_solve(o, tol=1e-8, hier=OH)
    assert abs(i8["iters"] - io8["iters"]) <= 1, (i8["iters"], io8["iters"])


def test_lair_distance_bad_parameter(built):
    from paper_2010_11130_amd import Hierarchy, AirHdgError
    g, _, _ = built("c1")
    with pytest.raises(AirHdgError):
        Hierarchy(g, lair_distance=3)


def test_coarsest_large_many_workgroup_inverse():
    """A coarsest level above the LDS sizes (the stalled coarsening of a
    pure-advection slab, max_coarse large): the dense inverse by
    Gauss-Jordan over many workgroups, one cycle against the oracle."""
    from paper_2010_11130_amd import Hierarchy
    v, c, prob, p = case("slab")
    g = gpu_system(v, c, prob, p)
    o = setup_problem(v, c, prob, p)
    H = Hierarchy(g, max_coarse=1500)
    OH = oair.setup(o.Shat, max_coarse=1500)
    assert H.info["n"] == [lev.A.shape[0] for lev in OH.levels]
    print("coarsest", H.info["n"][-1], flush=True)
    assert H.info["n"][-1] > 128
    r = np.random.default_rng(3).standard_normal(g.n)
    z = H.vcycle(torch.as_tensor(r, device="cuda")).cpu().numpy()
    zo = oair.vcycle(OH, r)
    assert np.linalg.norm(z - zo) <= 1e-10 * np.linalg.norm(zo)
    x, info = H.solve(tol=1e-12)
    xo, _ = air_fgmres_solve(o, tol=1e-12, hier=OH)
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-10 * np.linalg.norm(xo)
