"""Whole solves with the oracle: all-at-once (Section 2.2) and slab-by-slab
(Section 2.4), with either a sparse direct solve of the condensed system or
AIR-preconditioned FGMRES on the scaled system (Section 4 solver settings)."""
import numpy as np
import scipy.sparse.linalg as spla

from workloads import boundary_kinds
from .hdg import Mesh, assemble, reconstruct, l2_error, NEUMANN, DIRICHLET
from .quad import simplex_rule, bary
from .basis import lagrange
from . import air, krylov


def problem_g(prob, mesh, kinds, t_min, t_max):
    """Boundary data callback: Dirichlet ``g_D``; Neumann ``g = u(t0)`` on the
    initial plane and ``0`` on the final plane (Section 2.1)."""
    tf = mesh.vert[mesh.facet_vert][:, :, 0]
    bot = np.all(np.abs(tf - t_min) <= 1e-12, axis=1)

    def g(Xq, fids):
        out = np.zeros(Xq.shape[:2])
        k = kinds[fids]
        d = k == DIRICHLET
        if np.any(d):
            out[d] = prob.g_dirichlet(Xq[d])
        nb = (k == NEUMANN) & bot[fids]
        if np.any(nb):
            out[nb] = prob.g_neumann(Xq[nb], True)
        nt = (k == NEUMANN) & ~bot[fids]
        if np.any(nt):
            out[nt] = prob.g_neumann(Xq[nt], False)
        return out
    return g


def setup_problem(vert, cell, prob, p, alpha=None, g_fn=None, block_scale=True):
    mesh = Mesh(vert, cell)
    t_min, t_max = float(mesh.vert[:, 0].min()), float(mesh.vert[:, 0].max())
    kinds = boundary_kinds(mesh.vert, mesh.facet_vert, mesh.is_boundary, t_min, t_max)
    if g_fn is None:
        g_fn = problem_g(prob, mesh, kinds, t_min, t_max)
    sys = assemble(mesh, p, prob.nu, prob.a, prob.f, kinds, g_fn, alpha=alpha, block_scale=block_scale)
    return sys


def direct_solve(sys):
    """Sparse LU of the (unscaled) condensed free system ``S Lambda = H``."""
    return spla.spsolve(sys.S.tocsc(), sys.H)


def air_bicgstab_solve(sys, air_params=None, tol=1e-8, maxit=1000, x0=None, hier=None):
    """BiCGSTAB on ``S_hat Lambda = H_hat`` preconditioned on the right by one
    lAIR V-cycle (the paper's solver, Section 4)."""
    if hier is None:
        hier = air.setup(sys.Shat, **(air_params or {}))
    x, info = krylov.bicgstab(sys.Shat, sys.Hhat, lambda r: air.vcycle(hier, r), tol=tol, maxit=maxit, x0=x0)
    info["hier"] = hier
    return x, info


def air_fgmres_solve(sys, air_params=None, tol=1e-8, restart=100, maxit=1000, x0=None,
                     hier=None):
    """FGMRES on ``S_hat Lambda = H_hat`` preconditioned by one lAIR V-cycle."""
    if hier is None:
        hier = air.setup(sys.Shat, **(air_params or {}))
    x, info = krylov.fgmres(sys.Shat, sys.Hhat, lambda r: air.vcycle(hier, r), tol=tol,
                            restart=restart, maxit=maxit, x0=x0)
    info["hier"] = hier
    return x, info


def solve_all_at_once(vert, cell, prob, p, solver="direct", **kw):
    sys = setup_problem(vert, cell, prob, p)
    if solver == "direct":
        lam = direct_solve(sys)
        info = {}
    else:
        lam, info = air_fgmres_solve(sys, **kw)
    U = reconstruct(sys, lam)
    return sys, lam, U, info


def match_time_faces(mesh_lo, mesh_hi):
    """For every facet of ``mesh_hi`` on its initial plane, the facet of
    ``mesh_lo`` on its final plane with the same spatial vertex coordinates."""
    def key(mesh, fids):
        P = mesh.vert[mesh.facet_vert[fids]][:, :, 1:]
        ks = []
        for f in range(len(fids)):
            pts = sorted(tuple(np.round(v, 12)) for v in P[f])
            ks.append(tuple(pts))
        return ks
    tlo = mesh_lo.vert[:, 0].max()
    thi = mesh_hi.vert[:, 0].min()
    top = np.nonzero(mesh_lo.is_boundary & np.all(
        np.abs(mesh_lo.vert[mesh_lo.facet_vert][:, :, 0] - tlo) <= 1e-12, axis=1))[0]
    bot = np.nonzero(mesh_hi.is_boundary & np.all(
        np.abs(mesh_hi.vert[mesh_hi.facet_vert][:, :, 0] - thi) <= 1e-12, axis=1))[0]
    d = dict(zip(key(mesh_lo, top), top))
    return bot, np.array([d[k] for k in key(mesh_hi, bot)])


def trace_at_points(sys, lam_full, fid, Xq):
    """Evaluate the facet trace of facet ``fid`` at space-time points ``Xq[nq][D]``
    lying on it, via the facet barycentric coordinates of the points."""
    mesh = sys.mesh
    V = mesh.vert[mesh.facet_vert[fid]]          # sorted vertices [D][D]
    D = mesh.D
    # solve for mu (sum mu = 1) in least squares: V^T mu = X
    M = np.concatenate([V.T, np.ones((1, D))], axis=0)
    rhs = np.concatenate([Xq.T, np.ones((1, Xq.shape[0]))], axis=0)
    mu = np.linalg.lstsq(M, rhs, rcond=None)[0].T
    Psi, _ = lagrange(D - 1, sys.p, mu)
    b = sys.b
    return Psi @ lam_full[fid * b:(fid + 1) * b]


def solve_slabs(mesh_fn, nslab, prob, p, solver="direct", err=True, last_u=False, **kw):
    """Slab-by-slab march (Section 2.4): slab ``n+1`` takes as inflow data on its
    initial plane the trace ``lambda_h`` of slab ``n`` on its final plane (which
    equals ``u_h`` there: the outflow facet equation gives ``lambda = u``).
    Returns (L2 error, infos, per-slab solutions) and, with ``last_u``, the
    element solution of the last slab."""
    from .hdg import full_trace
    prev = None
    err2 = 0.0
    infos = []
    lams = []
    for k in range(nslab):
        vert, cell = mesh_fn(k)
        mesh = Mesh(vert, cell)
        t_min, t_max = float(mesh.vert[:, 0].min()), float(mesh.vert[:, 0].max())
        kinds = boundary_kinds(mesh.vert, mesh.facet_vert, mesh.is_boundary, t_min, t_max)
        g0 = problem_g(prob, mesh, kinds, t_min, t_max)
        if prev is not None:
            psys, plam_full = prev
            bot, top = match_time_faces(psys.mesh, mesh)
            fmap = dict(zip(bot, top))

            def g_fn(Xq, fids, g0=g0, fmap=fmap, psys=psys, plam=plam_full):
                out = g0(Xq, fids)
                for i, f in enumerate(fids):
                    if f in fmap:
                        out[i] = trace_at_points(psys, plam, fmap[f], Xq[i])
                return out
        else:
            g_fn = g0
        sys = assemble(mesh, p, prob.nu, prob.a, prob.f, kinds, g_fn)
        if solver == "direct":
            lam = direct_solve(sys)
            info = {}
        else:
            lam, info = air_fgmres_solve(sys, **kw)
        infos.append(info)
        lams.append(lam)
        U = reconstruct(sys, lam)
        if err:
            err2 += l2_error(sys, U, prob.u) ** 2
        prev = (sys, full_trace(sys, lam))
    if last_u:
        return np.sqrt(err2), infos, lams, U
    return np.sqrt(err2), infos, lams
