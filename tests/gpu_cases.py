"""Builds the same seeded problem on the HIP path and in the oracle (test
helper; imports both sides, which share only ``workloads``)."""
import numpy as np
import scipy.sparse as sp
import torch

from workloads import (square_tri_mesh, slab_prism_tet_mesh, kuhn_cube_mesh, map_vertices_c5,
                       pulse_slab_mesh, boundary_kinds)
from workloads.problems import (C1Advection1D, slab_hill, SmoothPlusFront, GaussianSources,
                                PolynomialProblem, c5_sources, paper_pulse, MovingInternalLayer)


def case(name):
    """(vert, cell, problem, p) of a named parity case."""
    if name == "c1":
        v, c = square_tri_mesh(16)
        return v, c, C1Advection1D(1e-4), 1
    if name == "c1_p3":
        v, c = square_tri_mesh(6)
        return v, c, C1Advection1D(1e-3), 3
    if name == "slab":
        v, c = slab_prism_tet_mesh(8, 1.0 / 64)
        return v, c, slab_hill(1e-4), 2
    if name == "slab_nu0":
        v, c = slab_prism_tet_mesh(8, 1.0 / 64)
        return v, c, slab_hill(0.0), 2
    if name in ("kuhn_nu0", "kuhn_nu4", "kuhn_nu2"):
        nu = {"kuhn_nu0": 0.0, "kuhn_nu4": 1e-4, "kuhn_nu2": 1e-2}[name]
        v, c = kuhn_cube_mesh(6)
        return v, c, SmoothPlusFront(nu, width=0.1), 1
    if name == "layer":
        v, c = kuhn_cube_mesh(6)
        return v, c, MovingInternalLayer(), 1
    if name == "layer_p2":
        v, c = kuhn_cube_mesh(4)
        return v, c, MovingInternalLayer(), 2
    if name == "c5":
        v, c = kuhn_cube_mesh(3)
        v = map_vertices_c5(v)
        centers, ct, ce = c5_sources(16)
        return v, c, GaussianSources(1e-3, centers, ce), 2
    if name == "kuhn_p3":
        v, c = kuhn_cube_mesh(2)
        return v, c, PolynomialProblem(2, 3, 1e-2, seed=3, a_lin=np.zeros((2, 3))), 3
    if name == "one_tet":
        v = np.array([[0, 0, 0], [0.3, 1, 0], [0.2, 0.1, 1], [1, 0.2, 0.3]])
        c = np.array([[0, 1, 2, 3]])
        return v, c, SmoothPlusFront(1e-2, width=0.3), 2
    raise KeyError(name)


def kinds_for(vert, fv, isb):
    return boundary_kinds(vert, fv, isb)


def boundary_data(prob, vert, fv, bf, kinds, xb):
    """g at the boundary-facet quadrature points: g_D on Dirichlet facets,
    g_N = u(t0) on initial-plane facets, 0 on final-plane facets."""
    t = vert[fv[bf]][:, :, 0]
    tmin = vert[:, 0].min()
    bot = torch.as_tensor(np.all(np.abs(t - tmin) <= 1e-12, axis=1), device="cuda")[:, None]
    kb = torch.as_tensor(kinds[bf], device="cuda")[:, None]
    gD = prob.g_dirichlet(xb)
    gN0 = prob.g_neumann(xb, True)
    gN1 = prob.g_neumann(xb, False)
    return torch.where(kb == 1, gD, torch.where(bot, gN0, gN1)).contiguous()


def gpu_system(vert, cell, prob, p, keep=True, block_scale=True, at_points=False):
    """The problem assembled on the HIP path; ``at_points``: the velocity is
    passed at the quadrature points (``hdg_assemble_q``) instead of the
    vertices."""
    from paper_2010_11130_amd import Mesh, System
    m = Mesh(vert, cell)
    fv, _ = m.facets()
    bf = m.boundary_facets()
    isb = np.zeros(m.nf, dtype=bool)
    isb[bf] = True
    kinds = kinds_for(vert, fv, isb)
    m.set_bc(kinds)
    xe, xb = m.quad_points(p)
    f = prob.f(xe).contiguous()
    g = boundary_data(prob, vert, fv, bf, kinds, xb)
    if at_points:
        a = (prob.a(xe).contiguous(), prob.a(m.facet_points(p)).contiguous())
        s = System(m, p, prob.nu, None, f, g, keep=keep, block_scale=block_scale, a_q=a)
    else:
        a = torch.as_tensor(np.ascontiguousarray(prob.a_vertices(vert)), device="cuda")
        s = System(m, p, prob.nu, a, f, g, keep=keep, block_scale=block_scale)
    s._keep_alive = (m, xe, xb, f, g, a)
    return s


def to_scipy(rowptr, col, val, n, ncol=None):
    return sp.csr_matrix((val.cpu().numpy(), col.cpu().numpy().astype(np.int64),
                          rowptr.cpu().numpy()), shape=(n, ncol if ncol is not None else n))


def rel_sparse_diff(A, B):
    d = (A - B).tocsr()
    m = np.abs(B.data).max() if B.nnz else 1.0
    return (np.abs(d.data).max() if d.nnz else 0.0) / m
