"""Flexible GMRES with right preconditioning (oracle).

The paper accelerates AIR with BiCGSTAB and notes that GMRES performed
equally well in most cases but can stall at restarts (Section 4.1, remark on
GMRES).  This build uses FGMRES(m): modified Gram-Schmidt Arnoldi, Givens
rotations, convergence when the estimated residual ``|g_{j+1}|`` is at most
``tol ||b||``, then a true-residual check that restarts from the current
iterate if it fails.  Happy breakdown when ``h_{j+1,j} <= 1e-14 ||w||``.
Iterations = preconditioner applications.
"""
import numpy as np


def fgmres(A, b, M, tol=1e-8, restart=100, maxit=1000, x0=None):
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else x0.astype(np.float64).copy()
    bnorm = np.linalg.norm(b)
    hist = []
    its = 0
    if bnorm == 0.0:
        return np.zeros(n), {"iters": 0, "converged": True, "relres": 0.0, "hist": hist}
    while True:
        r = b - A @ x
        beta = np.linalg.norm(r)
        hist.append(beta / bnorm)
        if beta <= tol * bnorm:
            return x, {"iters": its, "converged": True, "relres": beta / bnorm, "hist": hist}
        if its >= maxit:
            return x, {"iters": its, "converged": False, "relres": beta / bnorm, "hist": hist}
        m = restart
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        Hs = np.zeros((m + 1, m))
        cs = np.zeros(m); sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = M(V[j])
            w = A @ Z[j]
            its += 1
            wn0 = np.linalg.norm(w)
            for i in range(j + 1):
                Hs[i, j] = V[i] @ w
                w = w - Hs[i, j] * V[i]
            Hs[j + 1, j] = np.linalg.norm(w)
            for i in range(j):
                t = cs[i] * Hs[i, j] + sn[i] * Hs[i + 1, j]
                Hs[i + 1, j] = -sn[i] * Hs[i, j] + cs[i] * Hs[i + 1, j]
                Hs[i, j] = t
            den = np.hypot(Hs[j, j], Hs[j + 1, j])
            breakdown = Hs[j + 1, j] <= 1e-14 * wn0
            hj1 = Hs[j + 1, j]
            if den == 0.0:
                cs[j], sn[j] = 1.0, 0.0
            else:
                cs[j], sn[j] = Hs[j, j] / den, hj1 / den
            Hs[j, j] = cs[j] * Hs[j, j] + sn[j] * hj1
            Hs[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= tol * bnorm or breakdown or its >= maxit:
                break
            V[j + 1] = w / hj1
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - Hs[i, i + 1:k] @ y[i + 1:k]) / Hs[i, i]
        x = x + Z[:k].T @ y


def bicgstab(A, b, M, tol=1e-8, maxit=1000, x0=None):
    """BiCGSTAB with right preconditioning (van der Vorst's method), the
    Krylov accelerator the paper pairs with AIR (Section 4).

    Each step applies the preconditioner twice: p_hat = M p, v = A p_hat,
    alpha = rho / (r_hat, v), s = r - alpha v; s_hat = M s, t = A s_hat,
    omega = (t, s) / (t, t), x += alpha p_hat + omega s_hat,
    r = s - omega t.  Convergence when the recursively updated residual
    (s after the first half, r after the second) satisfies
    ||.|| <= tol ||b||; it is confirmed by the true residual, and the method
    restarts from the current iterate (r_hat = r) if that check fails or
    rho vanishes.  Iterations = BiCGSTAB steps (a step that converges on s
    counts as one)."""
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else x0.astype(np.float64).copy()
    bnorm = np.linalg.norm(b)
    hist = []
    its = 0
    if bnorm == 0.0:
        return np.zeros(n), {"iters": 0, "converged": True, "relres": 0.0, "hist": hist}
    while True:
        r = b - A @ x
        rel = np.linalg.norm(r) / bnorm
        hist.append(rel)
        if rel <= tol:
            return x, {"iters": its, "converged": True, "relres": rel, "hist": hist}
        if its >= maxit:
            return x, {"iters": its, "converged": False, "relres": rel, "hist": hist}
        rh = r.copy()
        rho_old = alpha = omega = 1.0
        p = np.zeros(n)
        v = np.zeros(n)
        while its < maxit:
            rho = rh @ r
            if rho == 0.0:
                break                       # restart with r_hat = r
            beta = (rho / rho_old) * (alpha / omega)
            p = r + beta * (p - omega * v)
            ph = M(p)
            v = A @ ph
            its += 1
            rv = rh @ v
            if rv == 0.0:
                break
            alpha = rho / rv
            s = r - alpha * v
            if np.linalg.norm(s) <= tol * bnorm:
                x = x + alpha * ph
                break
            sh = M(s)
            t = A @ sh
            tt = t @ t
            omega = (t @ s) / tt if tt > 0.0 else 0.0
            x = x + alpha * ph + omega * sh
            r = s - omega * t
            rho_old = rho
            if np.linalg.norm(r) <= tol * bnorm or omega == 0.0:
                break
