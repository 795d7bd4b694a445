"""Space-time HDG discretization (oracle): topology, element blocks, static
condensation, global facet system, Dirichlet elimination, block scaling,
reconstruction and the space-time L2 error.

Paper passages followed:
  * space-time problem and boundary conditions: Section 2.1
    (equations advdif / stadvdif: ``a_hat = (1, a)``, Neumann total flux with
    the inflow indicator, Dirichlet data);
  * finite element spaces ``V_h``, ``M_h`` and the bilinear form: Section 2.3
    (equations st-hdg, bilin; upwind flux ``sigma_a``; interior-penalty flux
    ``sigma_d`` with ``tau = nu alpha / h_K``, equation IPpenalty);
  * block system ``[A B; C D]`` and static condensation ``S = D - C A^-1 B``,
    ``H = G - C A^-1 F``: Section 2.5 (equations linsys, systemLambda);
  * ``alpha = 10 p^2`` and the left facet-block-diagonal scaling: Section 4
    (solver settings paragraph).

Readings where the paper is silent (listed in the design notes):
  * ``h_K = |det J_K|^(1/D)`` (the D-th root of the reference map's Jacobian
    determinant; the longest-edge reading is unstable at alpha = 10p^2 on
    the moving-domain slabs of Section 4.1);
  * the penalty term acts on every facet of K, time-like facets included;
  * Dirichlet trace = facet-wise L2 projection of ``g_D`` onto ``P_p(F)``;
  * facets are numbered by the lexicographic order of their sorted vertex-id
    tuples; facet DOF ``f*b + m`` with ``m`` the facet-lattice node;
  * the scaled system's facet diagonal blocks are set to the identity.

Expanding the bilinear form with ``a+ = (a_n+|a_n|)/2``, ``a- = (a_n-|a_n|)/2``
(``a_n = n_t + a.n``) gives, per element K (rows = test, cols = trial,
``grad`` = spatial gradient only):

  A(u,v) = int_K (-u a_hat.grad_hat v + nu grad u.grad v)
           + sum_F int_F [(a+ + tau) u v - nu (grad u.n) v - nu u (grad v.n)]
  B(l,v) = sum_F int_F [(a- - tau) l v + nu l (grad v.n)]
  C(u,m) = sum_F int_F [-(a+ + tau) u m + nu (grad u.n) m]
  D(l,m) = sum_F int_F [-(a- - tau) l m] + [F in dE_N] int_F a+ l m
  F(v)   = int_K f v,     G(m) = [F in dE_N] int_F g m
"""
import math
import numpy as np
import scipy.sparse as sp

from .quad import simplex_rule, bary
from .basis import lagrange, lagrange_ref_grad, ndofs

DIRICHLET = 1
NEUMANN = 2


class Mesh:
    """Space-time simplex mesh with facets numbered by sorted vertex tuples."""

    def __init__(self, vert, cell):
        self.vert = np.asarray(vert, dtype=np.float64)
        self.cell = np.asarray(cell, dtype=np.int64)
        D = self.vert.shape[1]
        self.D = D
        self.d = D - 1
        ne = self.cell.shape[0]
        self.ne = ne
        loc = np.array([[k for k in range(D + 1) if k != lf] for lf in range(D + 1)])
        fglob = self.cell[:, loc]                                  # [ne][D+1][D]
        order = np.argsort(fglob, axis=2, kind="stable")
        sglob = np.take_along_axis(fglob, order, axis=2)
        # local vertex index of the s-th (sorted) vertex of local facet lf
        self.facet_loc = loc[np.arange(D + 1)[None, :, None], order]
        uniq, inv = np.unique(sglob.reshape(-1, D), axis=0, return_inverse=True)
        self.facet_vert = uniq
        self.nf = uniq.shape[0]
        self.elem_facet = inv.reshape(ne, D + 1)
        cnt = np.bincount(inv.ravel(), minlength=self.nf)
        if cnt.max() > 2:
            raise ValueError("non-manifold mesh: a facet is shared by more than two elements")
        self.is_boundary = cnt == 1
        # geometry
        X = self.vert[self.cell]                                   # [ne][D+1][D]
        J = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))     # columns = edges from vertex 0
        self.X = X
        self.detJ = np.linalg.det(J)
        if np.any(np.abs(self.detJ) <= 1e-300):
            raise ValueError("degenerate element")
        self.Jinv = np.linalg.inv(J)
        self.volK = np.abs(self.detJ) / math.factorial(D)
        # length measure of K in the penalty (equation IPpenalty):
        # h_K = |det J_K|^(1/D) = (D! |K|)^(1/D)
        self.hK = np.abs(self.detJ) ** (1.0 / D)
        # physical gradients of barycentric coordinates: grad lam_a = Jinv[a-1, :]
        gl = np.concatenate([-self.Jinv.sum(1, keepdims=True), self.Jinv], axis=1)
        self.grad_lam = gl                                         # [ne][D+1][D]


def facet_geometry(mesh, lf):
    """Outward unit normal ``[ne][D]`` and measure ``[ne]`` of local facet lf."""
    g = mesh.grad_lam[:, lf, :]
    gn = np.linalg.norm(g, axis=1)
    nvec = -g / gn[:, None]
    area = mesh.D * mesh.volK * gn
    return nvec, area


def facet_points_bary(mesh, lf, mu):
    """Element barycentric coordinates ``[ne][nq][D+1]`` of points given by
    facet barycentrics ``mu[nq][D]`` over the facet's sorted vertices."""
    ne, D = mesh.ne, mesh.D
    lam = np.zeros((ne, mu.shape[0], D + 1))
    rows = np.arange(ne)
    for s in range(D):
        lam[rows, :, mesh.facet_loc[:, lf, s]] = mu[None, :, s]
    return lam


class System:
    pass


def assemble(mesh, p, nu, a_fn, f_fn, kinds, g_fn, alpha=None, chunk=4096, blocks_only=False, block_scale=True):
    """Element blocks, condensation, global facet system (Sections 2.3, 2.5).

    ``a_fn(X)`` -> ``[..., d]``, ``f_fn(X)`` -> ``[...]``; ``kinds[nf]`` in
    {0 interior, 1 Dirichlet, 2 Neumann}; ``g_fn(Xq, facet_ids)`` returns the
    Dirichlet or Neumann data ``[nsel][nqf]`` at those facets' points.
    """
    D = mesh.D
    if alpha is None:
        alpha = 10.0 * p * p
    nu_ = ndofs(D, p)
    b = ndofs(D - 1, p)
    nl = (D + 1) * b
    ne = mesh.ne
    nq1 = p + 2
    xv, wv = simplex_rule(D, nq1)
    lamv = bary(xv)
    phiv, grefv = lagrange_ref_grad(D, p, lamv)
    xf, wf = simplex_rule(D - 1, nq1)
    muf = bary(xf)
    Psi, _ = lagrange(D - 1, p, muf)                      # [nqf][b]
    wf_eff = wf * math.factorial(D - 1)                   # weights summing to 1

    A = np.zeros((ne, nu_, nu_)); B = np.zeros((ne, nu_, nl))
    C = np.zeros((ne, nl, nu_)); Dm = np.zeros((ne, nl, nl))
    F = np.zeros((ne, nu_)); G = np.zeros((ne, nl))
    tau_all = nu * alpha / mesh.hK
    kinds = np.asarray(kinds)
    lamD_full = np.zeros((mesh.nf, b))

    for e0 in range(0, ne, chunk):
        sl = slice(e0, min(ne, e0 + chunk))
        Jinv = mesh.Jinv[sl]
        X = mesh.X[sl]
        ad = np.abs(mesh.detJ[sl])
        tau = tau_all[sl]
        # volume terms
        gv = np.einsum("eab,qia->eqib", Jinv, grefv)               # grad_hat phi
        Xv = np.einsum("qk,ekc->eqc", lamv, X)
        Wv = wv[None, :] * ad[:, None]
        ahat = np.concatenate([np.ones(Xv.shape[:2] + (1,)), a_fn(Xv)], axis=-1)
        adv = np.einsum("eqb,eqib->eqi", ahat, gv)                 # a_hat . grad_hat v
        A[sl] -= np.einsum("eq,qj,eqi->eij", Wv, phiv, adv)
        A[sl] += nu * np.einsum("eq,eqjb,eqib->eij", Wv, gv[..., 1:], gv[..., 1:])
        F[sl] = np.einsum("eq,eq,qi->ei", Wv, f_fn(Xv), phiv)
        # facet terms
        for lf in range(D + 1):
            sub = _Sub(mesh, sl)
            lamK = facet_points_bary(sub, lf, muf)
            phi, gref = lagrange_ref_grad(D, p, lamK)
            gp = np.einsum("eab,eqia->eqib", Jinv, gref)
            Xq = np.einsum("eqk,ekc->eqc", lamK, X)
            nvec, area = facet_geometry(sub, lf)
            W = wf_eff[None, :] * area[:, None]
            an = nvec[:, None, 0] + np.einsum("eqc,ec->eq", a_fn(Xq), nvec[:, 1:])
            ap = 0.5 * (an + np.abs(an))
            am = 0.5 * (an - np.abs(an))
            dn = np.einsum("eqib,eb->eqi", gp[..., 1:], nvec[:, 1:])
            blk = slice(lf * b, (lf + 1) * b)
            tq = tau[:, None]
            A[sl] += np.einsum("eq,eqj,eqi->eij", W * (ap + tq), phi, phi)
            A[sl] -= nu * np.einsum("eq,eqj,eqi->eij", W, dn, phi)
            A[sl] -= nu * np.einsum("eq,eqj,eqi->eij", W, phi, dn)
            B[sl, :, blk] += np.einsum("eq,qm,eqi->eim", W * (am - tq), Psi, phi)
            B[sl, :, blk] += nu * np.einsum("eq,qm,eqi->eim", W, Psi, dn)
            C[sl, blk, :] -= np.einsum("eq,eqj,qm->emj", W * (ap + tq), phi, Psi)
            C[sl, blk, :] += nu * np.einsum("eq,eqj,qm->emj", W, dn, Psi)
            Dm[sl, blk, blk] -= np.einsum("eq,qm,qn->emn", W * (am - tq), Psi, Psi)
            fid = mesh.elem_facet[sl, lf]
            kf = kinds[fid]
            isN = kf == NEUMANN
            isD = kf == DIRICHLET
            if np.any(isN):
                Dm[sl, blk, blk] += np.einsum("eq,qm,qn->emn", W * ap * isN[:, None], Psi, Psi)
            if np.any(isN | isD):
                sel = np.nonzero(isN | isD)[0]
                g = np.asarray(g_fn(Xq[sel], fid[sel]), dtype=np.float64)
                selN = np.nonzero(isN[sel])[0]
                if selN.size:
                    G[e0 + sel[selN], blk] += np.einsum("eq,eq,qm->em", W[sel[selN]], g[selN], Psi)
                selD = np.nonzero(isD[sel])[0]
                if selD.size:
                    # L2 projection of g_D onto P_p(F)
                    Wd = W[sel[selD]]
                    Mf = np.einsum("eq,qm,qn->emn", Wd, Psi, Psi)
                    rhs = np.einsum("eq,eq,qm->em", Wd, g[selD], Psi)
                    lamD_full[fid[sel[selD]]] = np.linalg.solve(Mf, rhs[..., None])[..., 0]

    sys = System()
    sys.mesh, sys.p, sys.nu, sys.alpha, sys.b, sys.nu_dofs, sys.nl = mesh, p, nu, alpha, b, nu_, nl
    sys.A, sys.B, sys.C, sys.Dm, sys.F, sys.G = A, B, C, Dm, F, G
    sys.kinds = kinds
    sys.lamD_full = lamD_full
    if blocks_only:
        return sys
    _condense_and_assemble(sys)
    sys.lamD_full = lamD_full
    _dirichlet_and_scale(sys, block_scale)
    return sys


class _Sub:
    """Element-range view of a mesh (same attributes, sliced)."""

    def __init__(self, mesh, sl):
        self.ne = sl.stop - sl.start
        self.D = mesh.D
        self.facet_loc = mesh.facet_loc[sl]
        self.grad_lam = mesh.grad_lam[sl]
        self.volK = mesh.volK[sl]


def _condense_and_assemble(sys):
    """``S_K = D_K - C_K A_K^-1 B_K``, ``H_K = G_K - C_K A_K^-1 F_K`` (Section 2.5)
    and the sum over elements into the global facet system."""
    mesh, b, nl = sys.mesh, sys.b, sys.nl
    AinvB = np.linalg.solve(sys.A, sys.B)
    AinvF = np.linalg.solve(sys.A, sys.F[..., None])[..., 0]
    SK = sys.Dm - sys.C @ AinvB
    HK = sys.G - np.einsum("emj,ej->em", sys.C, AinvF)
    sys.SK, sys.HK = SK, HK
    gd = (mesh.elem_facet[:, :, None] * b + np.arange(b)[None, None, :]).reshape(mesh.ne, nl)
    sys.elem_dof = gd
    N = mesh.nf * b
    rows = np.repeat(gd[:, :, None], nl, axis=2).ravel()
    cols = np.repeat(gd[:, None, :], nl, axis=1).ravel()
    sys.S_all = sp.csr_matrix((SK.ravel(), (rows, cols)), shape=(N, N))
    sys.H_all = np.bincount(gd.ravel(), weights=HK.ravel(), minlength=N)


def _dirichlet_and_scale(sys, block_scale=True):
    """Eliminate Dirichlet facets (``mu = 0`` there, Section 2.3) and scale on
    the left by the inverse facet diagonal blocks (Section 4).  With
    ``block_scale=False`` (the "no block inverse" ablation of Section 4.1)
    ``S_hat = S``, ``H_hat = H`` and ``Dinv`` holds identity blocks."""
    mesh, b = sys.mesh, sys.b
    isdir = sys.kinds == DIRICHLET
    free_f = np.nonzero(~isdir)[0]
    dir_f = np.nonzero(isdir)[0]
    sys.free_facets, sys.dir_facets = free_f, dir_f
    fdofs = (free_f[:, None] * b + np.arange(b)).ravel()
    ddofs = (dir_f[:, None] * b + np.arange(b)).ravel()
    sys.free_dofs, sys.dir_dofs = fdofs, ddofs
    lamD = sys.lamD_full[dir_f].ravel()
    S_ff = sys.S_all[fdofs][:, fdofs].tocsr()
    S_fd = sys.S_all[fdofs][:, ddofs].tocsr()
    H = sys.H_all[fdofs] - S_fd @ lamD
    sys.S, sys.H = S_ff, H
    nfree = free_f.size
    n = nfree * b
    blocks = np.zeros((nfree, b, b))
    coo = S_ff.tocoo()
    rf, cf = coo.row // b, coo.col // b
    on = rf == cf
    blocks[rf[on], coo.row[on] % b, coo.col[on] % b] = coo.data[on]
    Dinv = np.linalg.inv(blocks)
    sys.Db, sys.Dinv = blocks, Dinv
    if not block_scale:
        sys.Dinv = np.broadcast_to(np.eye(b), (nfree, b, b)).copy()
        Shat = S_ff.copy()
        Shat.sort_indices()
        sys.Shat = Shat
        sys.Hhat = H.copy()
        sys.n = n
        return
    # scaled off-diagonal part + exact identity diagonal blocks
    off = sp.csr_matrix((coo.data[~on], (coo.row[~on], coo.col[~on])), shape=(n, n))
    bd_inv = sp.block_diag(list(Dinv), format="csr") if nfree else sp.csr_matrix((0, 0))
    Shat = ((bd_inv @ off) + sp.identity(n, format="csr")).tocsr()
    Shat.sort_indices()
    sys.Shat = Shat
    sys.Hhat = np.einsum("fmn,fn->fm", Dinv, H.reshape(nfree, b)).ravel()
    sys.n = n


def full_trace(sys, lam_free):
    """Facet vector over all facets: the solved free DOFs plus the Dirichlet traces."""
    out = sys.lamD_full.ravel().copy()
    out[sys.free_dofs] = lam_free
    return out


def reconstruct(sys, lam_free):
    """``U_K = A_K^-1 (F_K - B_K Lambda_K)`` (Section 2.5); the oracle's element
    basis is nodal, so ``U`` is ``u_h`` at the element lattice nodes."""
    lam = full_trace(sys, lam_free)
    LK = lam[sys.elem_dof]
    return np.linalg.solve(sys.A, (sys.F - np.einsum("eim,em->ei", sys.B, LK))[..., None])[..., 0]


def l2_error(sys, U, u_fn, extra=4):
    """Space-time L2 error ``||u - u_h||`` (Section 4.1) with an ``(p+extra)``-point
    collapsed rule (exact to degree ``2p+2 extra-1``)."""
    mesh, p, D = sys.mesh, sys.p, sys.mesh.D
    xv, wv = simplex_rule(D, p + extra)
    lamv = bary(xv)
    phiv, _ = lagrange(D, p, lamv)
    Xv = np.einsum("qk,ekc->eqc", lamv, mesh.X)
    uh = np.einsum("qi,ei->eq", phiv, U)
    err2 = np.einsum("q,e,eq->", wv, np.abs(mesh.detJ), (u_fn(Xv) - uh) ** 2)
    return math.sqrt(err2)


def eval_uh(sys, U, xi):
    """``u_h`` at reference points ``xi[nq][D]`` of every element: ``[ne][nq]``."""
    phi, _ = lagrange(sys.mesh.D, sys.p, bary(xi))
    return np.einsum("qi,ei->eq", phi, U)


def dense_full_solve(sys):
    """Solve the uncondensed block system ``[A B; C D][U; L] = [F; G]`` (Section
    2.5, equation linsys) densely, with the Dirichlet traces eliminated.
    Tiny meshes only; pins the static condensation."""
    mesh, b, nl, nuk = sys.mesh, sys.b, sys.nl, sys.nu_dofs
    ne = mesh.ne
    nU = ne * nuk
    nL = mesh.nf * b
    K = np.zeros((nU + nL, nU + nL))
    rhs = np.zeros(nU + nL)
    for e in range(ne):
        u = slice(e * nuk, (e + 1) * nuk)
        ld = nU + sys.elem_dof[e]
        K[u, u] += sys.A[e]
        K[np.ix_(range(u.start, u.stop), ld)] += sys.B[e]
        K[np.ix_(ld, range(u.start, u.stop))] += sys.C[e]
        K[np.ix_(ld, ld)] += sys.Dm[e]
        rhs[u] += sys.F[e]
        np.add.at(rhs, ld, sys.G[e])
    keep = np.concatenate([np.arange(nU), nU + sys.free_dofs])
    dcols = nU + sys.dir_dofs
    lamD = sys.lamD_full.ravel()[sys.dir_dofs]
    Kr = K[np.ix_(keep, keep)]
    rr = rhs[keep] - K[np.ix_(keep, dcols)] @ lamD
    sol = np.linalg.solve(Kr, rr)
    return sol[:nU].reshape(ne, nuk), sol[nU:]
