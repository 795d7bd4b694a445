"""Python binding of the airhdg C-ABI: argument marshalling only.

torch tensors provide device memory and the current HIP stream; every step
of the method runs in the library's HIP kernels.
"""
import ctypes as C

import numpy as np
import torch

from ._lib import (lib, check, destroy, HdgParams, AirParams, SetupInfo, SolveParams, SolveInfo,
                   AH_OK, AH_ENOCONV, AirHdgError)


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(x, dtype=torch.float64):
    if x is None:
        return None
    t = torch.as_tensor(x, dtype=dtype)
    if t.device.type != "cuda":
        t = t.cuda()
    return t.contiguous()


def _vec(t, n, name, shape=None, out=False):
    """Check a tensor argument that the library reads or writes as ``n``
    float64 values in device memory.  Inputs of another float type are
    widened and non-contiguous inputs copied (marshalling); an output must
    already be a contiguous float64 device tensor.  Raises ``ValueError``
    before any library call otherwise: the C-ABI cannot see sizes or types of
    device buffers."""
    if t is None:
        return None
    if not torch.is_tensor(t):
        if out:
            raise ValueError("%s: expected a torch tensor" % name)
        t = torch.as_tensor(np.asarray(t, dtype=np.float64))
    if out:
        if t.dtype != torch.float64:
            raise ValueError("%s: output must be float64, got %s" % (name, t.dtype))
    elif not t.dtype.is_floating_point:
        raise ValueError("%s: expected a floating-point tensor, got %s" % (name, t.dtype))
    if t.numel() != n:
        raise ValueError("%s: expected %d values%s, got %d (shape %s)"
                         % (name, n, "" if shape is None else " %s" % (shape,), t.numel(), tuple(t.shape)))
    if t.device.type != "cuda":
        raise ValueError("%s: expected a tensor in device memory, got device %s" % (name, t.device))
    if out:
        if not t.is_contiguous():
            raise ValueError("%s: output must be contiguous" % name)
        return t
    return t.to(torch.float64).contiguous()


_torch_alloc = None


def use_torch_allocator(on=True):
    """Route the library's device allocations through torch's caching
    allocator (``ah_set_allocator``), so the library and torch share one
    pool and ``torch.cuda.memory_allocated`` counts the library's objects;
    ``on=False`` restores the library's own pool.  Memory keeps the allocator
    it came from."""
    from ._lib import ALLOC_FN, FREE_FN
    global _torch_alloc
    if not on:
        check(lib().ah_set_allocator(ALLOC_FN(), FREE_FN(), None), "ah_set_allocator")
        return

    def alloc(ctx, nbytes, stream):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        except Exception:          # out of memory: the library reports AH_ENOMEM
            return None

    def free(ctx, ptr, nbytes, stream):
        torch.cuda.caching_allocator_delete(ptr)

    cbs = (ALLOC_FN(alloc), FREE_FN(free))
    check(lib().ah_set_allocator(cbs[0], cbs[1], None), "ah_set_allocator")
    _torch_alloc = cbs        # the callbacks must outlive every allocation made through them


def pool_trim():
    """Give the unused memory of the library's own pool back to the device
    (``ah_pool_trim``; waits for the device)."""
    check(lib().ah_pool_trim(), "ah_pool_trim")


def sizes(dim_st, p):
    """(nq, nqf, nu, b) for space-time dimension ``dim_st`` and degree ``p``."""
    a, b, c, d = C.c_int(), C.c_int(), C.c_int(), C.c_int()
    check(lib().ah_sizes(dim_st, p, C.byref(a), C.byref(b), C.byref(c), C.byref(d)), "ah_sizes")
    return a.value, b.value, c.value, d.value


def quad_rule(dim, n):
    """Conical-product rule on the reference simplex (host arrays)."""
    nq = n ** dim
    xi = np.zeros((nq, max(dim, 1)))
    w = np.zeros(nq)
    check(lib().ah_quad_rule(dim, n, xi.ctypes.data, w.ctypes.data), "ah_quad_rule")
    return xi[:, :dim], w


class Mesh:
    """Space-time simplex mesh; topology built on the host by the library."""

    def __init__(self, vert, cell):
        vert = np.ascontiguousarray(vert, dtype=np.float64)
        cell = np.ascontiguousarray(cell, dtype=np.int32)
        self.D = vert.shape[1]
        self.nv, self.ne = vert.shape[0], cell.shape[0]
        h = C.c_void_p()
        check(lib().ah_mesh_create(self.D, self.nv, vert.ctypes.data, self.ne, cell.ctypes.data,
                                   C.byref(h)), "ah_mesh_create")
        self.h = h
        nf, nbf = C.c_int64(), C.c_int64()
        check(lib().ah_mesh_sizes(h, C.byref(nf), C.byref(nbf)), "ah_mesh_sizes")
        self.nf, self.nbf = nf.value, nbf.value
        self.vert = vert
        self.kind = None

    def __del__(self, _destroy=destroy):
        if getattr(self, "h", None):
            _destroy("ah_mesh_destroy", self.h)
            self.h = None

    def facets(self):
        fv = np.zeros((self.nf, self.D), dtype=np.int32)
        fe = np.zeros((self.nf, 2), dtype=np.int32)
        check(lib().ah_mesh_facets(self.h, fv.ctypes.data, fe.ctypes.data), "ah_mesh_facets")
        return fv, fe

    def boundary_facets(self):
        ids = np.zeros(self.nbf, dtype=np.int32)
        if self.nbf:
            check(lib().ah_mesh_boundary_facets(self.h, ids.ctypes.data), "ah_mesh_boundary_facets")
        return ids

    def set_bc(self, kind):
        kind = np.ascontiguousarray(kind, dtype=np.int8)
        check(lib().ah_mesh_set_bc(self.h, kind.ctypes.data), "ah_mesh_set_bc")
        self.kind = kind

    def quad_points(self, p):
        """Element and boundary-facet quadrature points (device tensors)."""
        nq, nqf, _, _ = sizes(self.D, p)
        xe = torch.empty((self.ne, nq, self.D), dtype=torch.float64, device="cuda")
        xb = torch.empty((max(self.nbf, 1), nqf, self.D), dtype=torch.float64, device="cuda")
        check(lib().ah_quad_points(self.h, p, _p(xe), _p(xb), _stream()), "ah_quad_points")
        return xe, xb[:self.nbf]

    def facet_points(self, p):
        """Quadrature points of every facet, [nf][nqf][D] (device)."""
        _, nqf, _, _ = sizes(self.D, p)
        xf = torch.empty((max(self.nf, 1), nqf, self.D), dtype=torch.float64, device="cuda")
        check(lib().ah_quad_points_facets(self.h, p, _p(xf), _stream()), "ah_quad_points_facets")
        return xf[:self.nf]


class System:
    """Assembled, condensed and scaled facet system (``hdg_assemble``)."""

    def __init__(self, mesh, p, nu, a_vert=None, f_q=None, g_q=None, alpha=0.0, keep=True, block_scale=True,
                 a_q=None):
        """``a_vert``: velocity at the vertices ``[nv][d]`` (affine fields), or
        ``a_q = (a_elem, a_facet)``: velocity at the element quadrature points
        ``[ne][nq][d]`` and at every facet's points ``[nf][nqf][d]``
        (``hdg_assemble_q``)."""
        if mesh.kind is None:
            raise ValueError("boundary kinds not set (Mesh.set_bc)")
        if (a_vert is None) == (a_q is None):
            raise ValueError("give the velocity either at the vertices (a_vert) or at the quadrature points (a_q)")
        self.mesh = mesh
        self.p = p
        self.nu = float(nu)
        nq, nqf, _, _ = sizes(mesh.D, p)
        d = mesh.D - 1
        self._f = _vec(f_q, mesh.ne * nq, "f_q", (mesh.ne, nq))
        self._g = _vec(g_q, mesh.nbf * nqf, "g_q", (mesh.nbf, nqf))
        prm = HdgParams(p, float(alpha), 1 if keep else 0, 0 if block_scale else 1)
        h = C.c_void_p()
        if a_q is None:
            self._a = _vec(_dev(a_vert), mesh.nv * d, "a_vert", (mesh.nv, d))
            check(lib().hdg_assemble(mesh.h, C.byref(prm), float(nu), _p(self._a), _p(self._f), _p(self._g),
                                     _stream(), C.byref(h)), "hdg_assemble")
        else:
            self._a = None
            ae = _vec(a_q[0], mesh.ne * nq * d, "a_q[0]", (mesh.ne, nq, d))
            af = _vec(a_q[1], mesh.nf * nqf * d, "a_q[1]", (mesh.nf, nqf, d))
            self._aq = (ae, af)
            check(lib().hdg_assemble_q(mesh.h, C.byref(prm), float(nu), _p(ae), _p(af), _p(self._f), _p(self._g),
                                       _stream(), C.byref(h)), "hdg_assemble_q")
        self.h = h
        n, b, nnz = C.c_int64(), C.c_int(), C.c_int64()
        check(lib().ah_system_sizes(h, C.byref(n), C.byref(b), C.byref(nnz)), "ah_system_sizes")
        self.n, self.b, self.nnz = n.value, b.value, nnz.value
        self.nq, self.nqf, self.nu_dofs, _ = sizes(mesh.D, p)

    def __del__(self, _destroy=destroy):
        if getattr(self, "h", None):
            _destroy("ah_system_destroy", self.h)
            self.h = None

    def export(self):
        """Scaled CSR matrix, H_hat, D_b^-1 and the Dirichlet traces (device)."""
        rp = torch.empty(self.n + 1, dtype=torch.int64, device="cuda")
        ci = torch.empty(max(self.nnz, 1), dtype=torch.int32, device="cuda")
        va = torch.empty(max(self.nnz, 1), dtype=torch.float64, device="cuda")
        hh = torch.empty(max(self.n, 1), dtype=torch.float64, device="cuda")
        dinv = torch.empty((max(self.n // self.b, 1), self.b, self.b), dtype=torch.float64, device="cuda")
        lamd = torch.empty((self.mesh.nf, self.b), dtype=torch.float64, device="cuda")
        check(lib().ah_system_export(self.h, _p(rp), _p(ci), _p(va), _p(hh), _p(dinv), _p(lamd), _stream()),
              "ah_system_export")
        torch.cuda.synchronize()
        return {"rowptr": rp, "col": ci[:self.nnz], "val": va[:self.nnz], "hhat": hh[:self.n],
                "dinv": dinv[:self.n // self.b], "lam_dir": lamd}

    def reconstruct(self, lam):
        lam = _vec(lam, self.n, "lam")
        U = torch.empty((self.mesh.ne, self.nu_dofs), dtype=torch.float64, device="cuda")
        check(lib().hdg_reconstruct(self.h, _p(lam), _p(U), _stream()), "hdg_reconstruct")
        return U

    def trace_to_inflow(self, lam, next_mesh, g_q):
        """Write this system's final-plane trace ``lam`` into the inflow rows
        of ``g_q`` (boundary data of ``next_mesh``)."""
        lam = _vec(lam, self.n, "lam")
        _vec(g_q, next_mesh.nbf * self.nqf, "g_q", (next_mesh.nbf, self.nqf), out=True)
        check(lib().hdg_inflow_from_trace(self.h, _p(lam), next_mesh.h, _p(g_q), _stream()),
              "hdg_inflow_from_trace")
        return g_q

    def update_neumann(self, g_q):
        """New Neumann (inflow) data: recompute H and H_hat from ``g_q``
        without reassembling the matrix (``hdg_update_neumann``)."""
        self._g = _vec(g_q, self.mesh.nbf * self.nqf, "g_q", (self.mesh.nbf, self.nqf))
        check(lib().hdg_update_neumann(self.h, _p(self._g), _stream()), "hdg_update_neumann")
        return self

    def grad(self, lam_fwd, lam_adj, a_vert=None, want_f=True):
        """dJ/df at the element quadrature points and dJ/dnu (``hdg_assemble_grad``)."""
        lam_fwd = _vec(lam_fwd, self.n, "lam_fwd")
        lam_adj = _vec(lam_adj, self.n, "lam_adj")
        d = self.mesh.D - 1
        a = self._a if a_vert is None else _vec(_dev(a_vert), self.mesh.nv * d, "a_vert", (self.mesh.nv, d))
        dq = torch.empty((self.mesh.ne, self.nq), dtype=torch.float64, device="cuda") if want_f else None
        dnu = C.c_double()
        check(lib().hdg_assemble_grad(self.h, _p(a), _p(lam_fwd), _p(lam_adj),
                                      _p(dq), C.byref(dnu), _stream()), "hdg_assemble_grad")
        return dq, dnu.value


def air_params(**kw):
    p = AirParams()
    lib().ah_air_defaults(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def solve_params(**kw):
    p = SolveParams()
    lib().ah_solve_defaults(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


class Hierarchy:
    """lAIR hierarchy of a system (``air_setup``)."""

    def __init__(self, system, **kw):
        self.system = system
        self.prm = air_params(**kw)
        info = SetupInfo()
        h = C.c_void_p()
        check(lib().air_setup(system.h, C.byref(self.prm), _stream(), C.byref(h), C.byref(info)), "air_setup")
        self.h = h
        self.info = {"levels": info.levels, "n": list(info.n[:info.levels]),
                     "nnz": list(info.nnz[:info.levels]), "n_fallback": info.n_fallback,
                     "op_complexity": info.op_complexity, "t_setup_ms": info.t_setup_ms,
                     "block_view_values": info.block_view_values,
                     "level0_no_interp_pass": info.level0_no_interp_pass}

    def __del__(self, _destroy=destroy):
        if getattr(self, "h", None):
            _destroy("ah_hier_destroy", self.h)
            self.h = None

    def solve(self, rhs=None, x0=None, out=None, noalloc=False, **kw):
        """FGMRES + V-cycle: ``S Lambda = rhs`` (unscaled; ``None`` = assembled H).
        ``noalloc``: through ``air_solve_noalloc`` (workspace in the library's
        static scratch array; pass ``out`` to allocate nothing here either)."""
        prm = solve_params(**kw)
        n = self.system.n
        rhs = _vec(rhs, n, "rhs")
        x = _vec(out, n, "out", out=True) if out is not None else torch.empty(n, dtype=torch.float64,
                                                                               device="cuda")
        if x0 is not None:
            x.copy_(_vec(x0, n, "x0"))
            prm.x0_given = 1
        info = SolveInfo()
        fn = lib().air_solve_noalloc if noalloc else lib().air_solve
        st = check(fn(self.h, _p(rhs), _p(x), C.byref(prm), _stream(), C.byref(info)),
                   "air_solve_noalloc" if noalloc else "air_solve", allow=(AH_OK, AH_ENOCONV))
        return x, _info(info, st)

    def solve_adjoint(self, g, out=None, **kw):
        """``S^T lam = g`` with the transposed cycle."""
        prm = solve_params(**kw)
        n = self.system.n
        g = _vec(g, n, "g")
        lam = _vec(out, n, "out", out=True) if out is not None else torch.empty(n, dtype=torch.float64,
                                                                                 device="cuda")
        info = SolveInfo()
        st = check(lib().air_solve_adjoint(self.h, _p(g), _p(lam), C.byref(prm), _stream(),
                                           C.byref(info)), "air_solve_adjoint", allow=(AH_OK, AH_ENOCONV))
        return lam, _info(info, st)

    def vcycle(self, r, precision=0, transpose=False):
        r = _vec(r, self.system.n, "r")
        z = torch.empty_like(r)
        check(lib().ah_vcycle_apply(self.h, _p(r), _p(z), int(precision), int(bool(transpose)),
                                    _stream()), "ah_vcycle_apply")
        return z

    def flow_levels(self):
        """Level of every level-0 facet block in the flow order of the ordered
        relaxations (``relax`` 2 or 3), the number of rounds and of cycle
        breaks."""
        nb, rounds, breaks = C.c_int64(), C.c_int(), C.c_int()
        check(lib().ah_hier_flow_levels(self.h, None, C.byref(nb), C.byref(rounds), C.byref(breaks)),
              "flow_levels")
        lev = torch.empty(nb.value, dtype=torch.int32)
        if nb.value:
            check(lib().ah_hier_flow_levels(self.h, C.c_void_p(lev.data_ptr()), None, None, None), "flow_levels")
        return lev.numpy(), rounds.value, breaks.value

    def level(self, l):
        n, nnz, nnzr = C.c_int64(), C.c_int64(), C.c_int64()
        check(lib().ah_hier_level_sizes(self.h, l, C.byref(n), C.byref(nnz), C.byref(nnzr)), "level_sizes")
        n, nnz, nnzr = n.value, nnz.value, nnzr.value
        coarse = l + 1 < self.info["levels"]
        e = lambda k, dt: torch.empty(max(k, 1), dtype=dt, device="cuda")
        out = {"rowptr": e(n + 1, torch.int64), "col": e(nnz, torch.int32), "val": e(nnz, torch.float64)}
        if coarse:
            nc = self.info["n"][l + 1]
            out.update({"cf": e(n, torch.int8), "pcol": e(n, torch.int32), "Rptr": e(nc + 1, torch.int64),
                        "Rcol": e(nnzr, torch.int32), "Rval": e(nnzr, torch.float64)})
        g = out.get
        check(lib().ah_hier_level_export(self.h, l, _p(g("rowptr")), _p(g("col")), _p(g("val")), _p(g("cf")),
                                         _p(g("pcol")), _p(g("Rptr")), _p(g("Rcol")), _p(g("Rval")), _stream()),
              "level_export")
        torch.cuda.synchronize()
        out["col"], out["val"] = out["col"][:nnz], out["val"][:nnz]
        if coarse:
            out["cf"], out["pcol"] = out["cf"][:n], out["pcol"][:n]
            out["Rcol"], out["Rval"] = out["Rcol"][:nnzr], out["Rval"][:nnzr]
        out["n"], out["nnz"] = n, nnz
        return out


def _info(info, st):
    return {"iters": info.iters, "converged": bool(info.converged), "relres": info.relres,
            "true_relres": info.true_relres, "t_solve_ms": info.t_solve_ms, "status": st}


def _points(X):
    if not torch.is_tensor(X) or X.device.type != "cuda" or X.dim() < 2:
        raise ValueError("X: expected a device tensor of points [..., dim_st]")
    D = X.shape[-1]
    if D not in (2, 3):
        raise ValueError("X: points of dimension 2 or 3 expected, got %d" % D)
    return X.to(torch.float64).contiguous(), D, X.numel() // D


def _centers(centers, D):
    cen = _dev(centers)
    if cen.dim() != 2 or cen.shape[1] != D:
        raise ValueError("centers: expected [K][%d], got %s" % (D, tuple(cen.shape)))
    return cen


def source_gauss(X, centers, width, c):
    """``f(X) = sum_k c_k exp(-|X - X_k|^2 / (2 width^2))`` (device)."""
    X, D, npts = _points(X)
    cen = _centers(centers, D)
    cc = _vec(_dev(c), cen.shape[0], "c")
    f = torch.empty(X.shape[:-1], dtype=torch.float64, device="cuda")
    check(lib().ah_source_gauss(D, npts, _p(X), cen.shape[0], _p(cen), float(width), _p(cc), _p(f), _stream()),
          "ah_source_gauss")
    return f


def source_gauss_T(X, centers, width, y):
    """``dc_k = sum_points y(X) phi_k(X)`` (device)."""
    X, D, npts = _points(X)
    cen = _centers(centers, D)
    y = _vec(y, npts, "y")
    dc = torch.empty(cen.shape[0], dtype=torch.float64, device="cuda")
    check(lib().ah_source_gauss_T(D, npts, _p(X), cen.shape[0], _p(cen), float(width), _p(y),
                                  _p(dc), _stream()), "ah_source_gauss_T")
    return dc


def _require_converged(info, what):
    if not info["converged"]:
        raise AirHdgError(AH_ENOCONV, what, "no convergence in %d iterations, relative residual %.3e"
                          % (info["iters"], info["true_relres"]))


class GaussSource(torch.autograd.Function):
    """``f_q = sum_k c_k phi_k(X)`` with Gaussian bumps
    ``phi_k(X) = exp(-|X - X_k|^2 / (2 width^2))`` at the points ``X``
    (e.g. the element quadrature points); the backward pass contracts
    ``dL/df_q`` with the same bumps (``ah_source_gauss_T``).  Differentiable
    in the amplitudes ``c`` only."""

    @staticmethod
    def forward(ctx, c, X, centers, width):
        ctx.X, ctx.centers, ctx.width = X, centers, width
        return source_gauss(X, centers, width, c.detach())

    @staticmethod
    def backward(ctx, gf):
        return source_gauss_T(ctx.X, ctx.centers, ctx.width, gf.reshape(-1)), None, None, None


class AIRSolve(torch.autograd.Function):
    """``Lambda = S^-1 rhs``; the backward pass solves ``S^T lam = dL/dLambda``
    with the transposed hierarchy (P^T restriction, R^T interpolation).  The
    hierarchy must be built with ``adjoint=1`` (and ``fp32_cycle=1`` for
    ``precision=1``).  Raises ``AirHdgError`` when either solve does not
    converge."""

    @staticmethod
    def forward(ctx, rhs, hier, tol=1e-8, precision=0, maxit=1000, adjoint_maxit=None):
        x, info = hier.solve(rhs.detach(), tol=tol, precision=precision, maxit=maxit)
        _require_converged(info, "AIRSolve forward")
        ctx.hier, ctx.tol, ctx.precision = hier, tol, precision
        ctx.maxit = maxit if adjoint_maxit is None else adjoint_maxit
        ctx.info = info
        return x

    @staticmethod
    def backward(ctx, g):
        lam, info = ctx.hier.solve_adjoint(g, tol=ctx.tol, precision=ctx.precision, maxit=ctx.maxit)
        _require_converged(info, "AIRSolve adjoint")
        return lam, None, None, None, None, None


class HDGSolve(torch.autograd.Function):
    """``Lambda(f_q, nu)``: assembly, AIR setup and solve in the forward pass;
    the backward pass returns ``dJ/df_q`` (at the element quadrature points)
    and ``dJ/dnu`` from one adjoint solve and the element adjoint.  Raises
    ``AirHdgError`` when the forward or the adjoint solve does not
    converge."""

    @staticmethod
    def forward(ctx, f_q, nu, mesh, p, a_vert, g_q, tol=1e-12, precision=0, air_kw=None):
        sysm = System(mesh, p, float(nu), a_vert, f_q.detach(), g_q)
        hier = Hierarchy(sysm, adjoint=1, fp32_cycle=1 if precision else 0, **(air_kw or {}))
        lam, info = hier.solve(tol=tol, precision=precision)
        _require_converged(info, "HDGSolve forward")
        ctx.sysm, ctx.hier, ctx.tol, ctx.precision = sysm, hier, tol, precision
        ctx.info = info
        ctx.save_for_backward(lam)
        ctx.nu_is_tensor = torch.is_tensor(nu)
        return lam

    @staticmethod
    def backward(ctx, g):
        (lam,) = ctx.saved_tensors
        adj, info = ctx.hier.solve_adjoint(g, tol=ctx.tol, precision=ctx.precision)
        _require_converged(info, "HDGSolve adjoint")
        ctx.adj_info = info
        dq, dnu = ctx.sysm.grad(lam, adj)
        gnu = torch.tensor(dnu, dtype=torch.float64) if ctx.nu_is_tensor else None
        return dq, gnu, None, None, None, None, None, None, None
