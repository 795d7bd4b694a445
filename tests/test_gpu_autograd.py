"""The differentiation form end to end through the autograd Functions of the
binding (``GaussSource``, ``HDGSolve``, ``AIRSolve``), in FP64 and with the
FP32 cycle, against the oracle's dense adjoint and against central finite
differences of the HIP path's own forward solves; and the FP32-cycle adjoint
solve against the oracle's direct transposed solve.

Tolerances:
  * gradients vs the oracle's dense adjoint (forward and adjoint solves to
    1e-13): 1e-8 relative;
  * gradients vs central differences (h = 1e-6, forward solves to 1e-13):
    1e-6 relative (J is quadratic in the amplitudes and in the right-hand
    side, so the difference quotient is exact up to rounding there; in nu
    its truncation error is O(h^2));
  * FP32-cycle adjoint solution at tol 1e-12: 1e-10 relative (the outer
    FGMRES, the products with S_hat^T and the true residual are FP64).
"""
import numpy as np
import pytest
import torch

from oracle import adjoint as oadj
from oracle.drivers import setup_problem, direct_solve, problem_g
from gpu_cases import case, gpu_system, boundary_data, kinds_for
from workloads import kuhn_cube_mesh, map_vertices_c5
from workloads.problems import GaussianSources, c5_sources

pytestmark = pytest.mark.gpu

SMALL_COARSE = 40
NU = 1e-3
P = 2


class Tiny:
    """Mapped 2^3 Kuhn mesh (C5 shapes), p = 2, 16 Gaussian sources; the same
    seeded problem on the HIP path and in the oracle."""

    def __init__(self, n=2, nsrc=16):
        from paper_2010_11130_amd import Mesh
        v, c = kuhn_cube_mesh(n)
        v = map_vertices_c5(v)
        self.v, self.c = v, c
        self.centers, c_target, c_eval = c5_sources(nsrc)
        self.width = 0.1
        self.c_eval = c_eval
        m = Mesh(v, c)
        fv, _ = m.facets()
        bf = m.boundary_facets()
        isb = np.zeros(m.nf, dtype=bool)
        isb[bf] = True
        kinds = kinds_for(v, fv, isb)
        m.set_bc(kinds)
        self.mesh = m
        self.xe, xb = m.quad_points(P)
        prob = GaussianSources(NU, self.centers, c_eval)
        self.prob = prob
        self.g_q = boundary_data(prob, v, fv, bf, kinds, xb)
        self.a_vert = torch.as_tensor(np.ascontiguousarray(prob.a_vertices(v)), device="cuda")
        # oracle at the evaluation point, and the target trace
        self.o = setup_problem(v, c, prob, P)
        ot = setup_problem(v, c, GaussianSources(NU, self.centers, c_target), P)
        self.target_np = direct_solve(ot)
        self.target = torch.as_tensor(self.target_np, device="cuda")
        self.lam_o = direct_solve(self.o)
        g_fn = problem_g(prob, self.o.mesh, self.o.kinds, 0.0, 1.0)
        self.J_o, self.dc_o, self.dnu_o, self.adj_o = oadj.misfit_and_grads(
            self.o, self.lam_o, self.target_np, prob.a, prob.f, g_fn, prob.basis, dense=True)

    def J(self, c, nu, precision, tol=1e-13):
        from paper_2010_11130_amd import GaussSource, HDGSolve
        f_q = GaussSource.apply(c, self.xe, self.centers, self.width)
        lam = HDGSolve.apply(f_q, nu, self.mesh, P, self.a_vert, self.g_q, tol, precision,
                             {"max_coarse": SMALL_COARSE})
        return 0.5 * ((lam - self.target) ** 2).sum(), lam


@pytest.fixture(scope="module")
def tiny():
    return Tiny()


@pytest.mark.parametrize("precision", [0, 1])
def test_hdgsolve_gradients_match_dense_adjoint(tiny, precision):
    print("case tiny-c5 HDGSolve precision", precision, flush=True)
    c = torch.as_tensor(tiny.c_eval, device="cuda").clone().requires_grad_(True)
    nu = torch.tensor(NU, dtype=torch.float64, requires_grad=True)
    J, lam = tiny.J(c, nu, precision)
    assert np.linalg.norm(lam.detach().cpu().numpy() - tiny.lam_o) <= 1e-10 * np.linalg.norm(tiny.lam_o)
    assert abs(J.item() - tiny.J_o) <= 1e-10 * abs(tiny.J_o)
    J.backward()
    dc = c.grad.cpu().numpy()
    assert np.linalg.norm(dc - tiny.dc_o) <= 1e-8 * np.linalg.norm(tiny.dc_o)
    assert abs(nu.grad.item() - tiny.dnu_o) <= 1e-8 * abs(tiny.dnu_o)


@pytest.mark.parametrize("precision", [0, 1])
def test_hdgsolve_gradients_match_central_differences(tiny, precision):
    print("case tiny-c5 FD precision", precision, flush=True)
    c0 = torch.as_tensor(tiny.c_eval, device="cuda")
    c = c0.clone().requires_grad_(True)
    nu = torch.tensor(NU, dtype=torch.float64, requires_grad=True)
    J, _ = tiny.J(c, nu, precision)
    J.backward()
    h = 1e-6
    rng = np.random.default_rng(31)
    with torch.no_grad():
        for k in range(3):
            d = torch.as_tensor(rng.standard_normal(c0.numel()), device="cuda")
            jp, _ = tiny.J(c0 + h * d, NU, precision)
            jm, _ = tiny.J(c0 - h * d, NU, precision)
            fd = (jp.item() - jm.item()) / (2 * h)
            ad = float((c.grad * d).sum())
            assert abs(fd - ad) <= 1e-6 * abs(ad), (k, fd, ad)
        jp, _ = tiny.J(c0, NU + h, precision)
        jm, _ = tiny.J(c0, NU - h, precision)
        fd = (jp.item() - jm.item()) / (2 * h)
        assert abs(fd - nu.grad.item()) <= 1e-6 * abs(nu.grad.item()), (fd, nu.grad.item())


@pytest.mark.parametrize("precision", [0, 1])
def test_airsolve_backward_is_the_transposed_solve(tiny, precision):
    from paper_2010_11130_amd import System, Hierarchy, AIRSolve
    print("case tiny-c5 AIRSolve precision", precision, flush=True)
    f_q = tiny.prob.f(tiny.xe).contiguous()
    s = System(tiny.mesh, P, NU, tiny.a_vert, f_q, tiny.g_q)
    H = Hierarchy(s, max_coarse=SMALL_COARSE, adjoint=1, fp32_cycle=precision)
    rng = np.random.default_rng(32)
    rhs_np = rng.standard_normal(s.n)
    rhs = torch.as_tensor(rhs_np, device="cuda").requires_grad_(True)
    lam = AIRSolve.apply(rhs, H, 1e-13, precision)
    lam_o = np.linalg.solve(tiny.o.S.toarray(), rhs_np)
    assert np.linalg.norm(lam.detach().cpu().numpy() - lam_o) <= 1e-10 * np.linalg.norm(lam_o)
    J = 0.5 * ((lam - tiny.target) ** 2).sum()
    J.backward()
    ref = oadj.adjoint_dense(tiny.o, lam_o - tiny.target_np)
    assert np.linalg.norm(rhs.grad.cpu().numpy() - ref) <= 1e-9 * np.linalg.norm(ref)
    # central differences along a seeded direction (J is quadratic in rhs)
    d = rng.standard_normal(s.n)
    h = 1e-6
    with torch.no_grad():
        Jp = 0.5 * float(((AIRSolve.apply(rhs + h * torch.as_tensor(d, device="cuda"), H, 1e-13, precision)
                           - tiny.target) ** 2).sum())
        Jm = 0.5 * float(((AIRSolve.apply(rhs - h * torch.as_tensor(d, device="cuda"), H, 1e-13, precision)
                           - tiny.target) ** 2).sum())
    ad = float(rhs.grad.cpu().numpy() @ d)
    assert abs((Jp - Jm) / (2 * h) - ad) <= 1e-6 * abs(ad)


def test_gauss_source_forward_and_transpose(tiny):
    from paper_2010_11130_amd import GaussSource
    c = torch.as_tensor(tiny.c_eval, device="cuda").clone().requires_grad_(True)
    f = GaussSource.apply(c, tiny.xe, tiny.centers, tiny.width)
    Phi = tiny.prob.basis(tiny.xe.cpu().numpy())            # [ne][nq][K]
    f_ref = Phi @ tiny.c_eval
    assert np.abs(f.detach().cpu().numpy() - f_ref).max() <= 1e-13 * np.abs(f_ref).max()
    y = np.random.default_rng(33).standard_normal(f_ref.shape)
    (f * torch.as_tensor(y, device="cuda")).sum().backward()
    ref = np.einsum("eqk,eq->k", Phi, y)
    assert np.abs(c.grad.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


def test_autograd_raises_without_convergence(tiny):
    from paper_2010_11130_amd import System, Hierarchy, AIRSolve, AirHdgError
    f_q = tiny.prob.f(tiny.xe).contiguous()
    s = System(tiny.mesh, P, NU, tiny.a_vert, f_q, tiny.g_q)
    H = Hierarchy(s, max_coarse=SMALL_COARSE, adjoint=1)
    rhs = torch.as_tensor(np.random.default_rng(34).standard_normal(s.n), device="cuda")
    with pytest.raises(AirHdgError, match="AIRSolve forward"):
        AIRSolve.apply(rhs, H, 1e-12, 0, 1)
    rhs.requires_grad_(True)
    lam = AIRSolve.apply(rhs, H, 1e-12, 0, 1000, 1)     # forward converges, adjoint capped at 1
    with pytest.raises(AirHdgError, match="AIRSolve adjoint"):
        lam.sum().backward()


@pytest.mark.parametrize("name", ["c1", "slab", "kuhn_nu4", "c5"])
def test_fp32_cycle_adjoint_solve(name):
    from paper_2010_11130_amd import Hierarchy
    print("case", name, flush=True)
    v, c, prob, p = case(name)
    g = gpu_system(v, c, prob, p)
    o = setup_problem(v, c, prob, p)
    H = Hierarchy(g, max_coarse=SMALL_COARSE, adjoint=1, fp32_cycle=1)
    rhs = np.random.default_rng(35).standard_normal(g.n)
    lam64, i64 = H.solve_adjoint(torch.as_tensor(rhs, device="cuda"), tol=1e-12, precision=0)
    lam32, i32 = H.solve_adjoint(torch.as_tensor(rhs, device="cuda"), tol=1e-12, precision=1)
    ref = oadj.adjoint_direct(o, rhs)
    assert i32["converged"] and i64["converged"]
    for lam in (lam64, lam32):
        assert np.linalg.norm(lam.cpu().numpy() - ref) <= 1e-10 * np.linalg.norm(ref)
    # the FP32 transposed cycle is about as strong a preconditioner as the
    # FP64 one at this tolerance
    assert i32["iters"] <= i64["iters"] + 2, (i32["iters"], i64["iters"])
