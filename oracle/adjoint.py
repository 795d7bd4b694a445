"""Adjoint solve and gradients (oracle).

Not a passage of the paper: the differentiation form solves the transposed
condensed system with the transposed AIR cycle and differentiates a misfit
``J = 1/2 ||Lambda - Lambda_target||^2`` of the free facet DOFs with respect to
the source amplitudes and to ``nu``.

With ``K = [A B; C D]`` the uncondensed system (Section 2.5) and
``psi = (w, lam)`` solving ``K^T psi = (0, dJ/dLambda)``:
  * ``S^T lam = dJ/dLambda`` with ``S = D - C A^-1 B`` (the condensed adjoint),
  * ``w_K = -A_K^-T C_K^T lam_K`` element by element,
  * ``dJ/dtheta = w^T (dF - dA U - dB Lambda) + lam^T (dG - dC U - dD Lambda)``.
Scaled form: ``S = D_b S_hat`` so ``S^T lam = g`` <=> ``S_hat^T mu = g`` with
``lam = D_b^-T mu``.  The blocks are affine in nu (``tau = nu alpha / h_K``), so
``dX/dnu = X(nu=1) - X(nu=0)``.
"""
import numpy as np
import scipy.sparse.linalg as spla

from . import air, krylov
from .hdg import assemble, reconstruct, full_trace
from .quad import simplex_rule, bary
from .basis import lagrange


def adjoint_solve(sys, hier, g, tol=1e-12, restart=100, maxit=1000):
    """``S^T lam = g`` by FGMRES on ``S_hat^T`` with the transposed V-cycle."""
    ShT = sys.Shat.T.tocsr()
    mu, info = krylov.fgmres(ShT, g, lambda r: air.vcycle_T(hier, r), tol=tol,
                             restart=restart, maxit=maxit)
    b = sys.b
    lam = np.einsum("fnm,fn->fm", sys.Dinv, mu.reshape(-1, b)).ravel()   # D_b^-T mu
    return lam, info


def adjoint_dense(sys, g):
    """Dense reference: ``S^T lam = g`` by LU of the unscaled matrix."""
    return np.linalg.solve(sys.S.toarray().T, g)


def adjoint_direct(sys, g):
    return spla.spsolve(sys.S.T.tocsc(), g)


def element_adjoint(sys, lam_free):
    """``w_K = -A_K^-T C_K^T lam_K`` (zero adjoint trace on Dirichlet facets)."""
    lam = np.zeros(sys.mesh.nf * sys.b)
    lam[sys.free_dofs] = lam_free
    LK = lam[sys.elem_dof]
    rhs = -np.einsum("emj,em->ej", sys.C, LK)
    w = np.linalg.solve(np.transpose(sys.A, (0, 2, 1)), rhs[..., None])[..., 0]
    return w, LK


def grad_source(sys, w, basis_fn):
    """``dJ/dc_k = sum_K w_K . int_K phi_k v`` with the assembly's volume rule."""
    mesh, p, D = sys.mesh, sys.p, sys.mesh.D
    xv, wv = simplex_rule(D, p + 2)
    lamv = bary(xv)
    phiv, _ = lagrange(D, p, lamv)
    Xv = np.einsum("qk,ekc->eqc", lamv, mesh.X)
    Wv = wv[None, :] * np.abs(mesh.detJ)[:, None]
    wq = np.einsum("ei,qi->eq", w, phiv) * Wv          # dJ/df at each quadrature point
    Phi = basis_fn(Xv)                                  # [ne][nq][K]
    return np.einsum("eq,eqk->k", wq, Phi)


def nu_derivative_blocks(sys, a_fn, f_fn, g_fn):
    """``dA/dnu, dB/dnu, dC/dnu, dD/dnu`` from the affine dependence on nu."""
    s1 = assemble(sys.mesh, sys.p, 1.0, a_fn, f_fn, sys.kinds, g_fn, alpha=sys.alpha, blocks_only=True)
    s0 = assemble(sys.mesh, sys.p, 0.0, a_fn, f_fn, sys.kinds, g_fn, alpha=sys.alpha, blocks_only=True)
    return (s1.A - s0.A, s1.B - s0.B, s1.C - s0.C, s1.Dm - s0.Dm)


def grad_nu(sys, lam_free, w, LK, U, dblocks):
    A1, B1, C1, D1 = dblocks
    LamK = full_trace(sys, sys._lam_fwd)[sys.elem_dof]
    t1 = -np.einsum("ei,eij,ej->", w, A1, U) - np.einsum("ei,eim,em->", w, B1, LamK)
    t2 = -np.einsum("em,emj,ej->", LK, C1, U) - np.einsum("em,emn,en->", LK, D1, LamK)
    return t1 + t2


def misfit_and_grads(sys, lam_fwd, lam_target, a_fn, f_fn, g_fn, basis_fn, hier=None,
                     dense=False, tol=1e-12):
    """``J``, ``dJ/dc`` (through ``basis_fn``) and ``dJ/dnu`` at the forward
    solution ``lam_fwd``."""
    g = lam_fwd - lam_target
    J = 0.5 * float(g @ g)
    if dense:
        lam = adjoint_dense(sys, g)
    elif hier is None:
        lam = adjoint_direct(sys, g)
    else:
        lam, _ = adjoint_solve(sys, hier, g, tol=tol)
    w, LK = element_adjoint(sys, lam)
    U = reconstruct(sys, lam_fwd)
    sys._lam_fwd = lam_fwd
    dc = grad_source(sys, w, basis_fn)
    dnu = grad_nu(sys, lam, w, LK, U, nu_derivative_blocks(sys, a_fn, f_fn, g_fn))
    return J, dc, dnu, lam
