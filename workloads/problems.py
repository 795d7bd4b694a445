"""Problem data of each workload: velocity ``a``, diffusion ``nu``, source ``f``,
exact solution ``u`` (where known), Dirichlet data ``g_D`` and Neumann data.

All functions take space-time points ``X[..., D]`` (column 0 = t) as numpy
arrays or torch tensors and return the same kind.  Neumann data follows the
boundary condition of Section 2.1: on the initial plane (inflow, ``n_t=-1``,
spatial normal zero) the condition reduces to ``u = g``, so ``g = u(t0, x)``;
on the final plane (outflow) ``g = 0``.
"""
import math
import numpy as np


def _ns(X):
    if type(X).__module__.startswith("torch"):
        import torch
        return torch
    return np


class Problem:
    d = 1
    nu = 0.0
    has_exact = True

    def a(self, X):
        raise NotImplementedError

    def f(self, X):
        xp = _ns(X)
        return xp.zeros_like(X[..., 0])

    def u(self, X):
        raise NotImplementedError

    def g_dirichlet(self, X):
        return self.u(X)

    def g_neumann(self, X, on_bottom):
        """``on_bottom`` selects the inflow plane (True) or outflow plane."""
        xp = _ns(X)
        if on_bottom:
            return self.u(X)
        return xp.zeros_like(X[..., 0])

    def a_vertices(self, vert):
        """Velocity at mesh vertices ``[nv][d]``; every velocity field here is
        affine in x, so its vertex interpolant is exact."""
        return self.a(vert)


class C1Advection1D(Problem):
    """1+1-D: ``a=1``, ``u = sin(2 pi (x-t)) e^{-t}``, ``f = (4 pi^2 nu - 1) u``."""

    def __init__(self, nu=1e-4):
        self.d = 1
        self.nu = nu

    def a(self, X):
        xp = _ns(X)
        return xp.ones_like(X[..., 1:2])

    def u(self, X):
        xp = _ns(X)
        t, x = X[..., 0], X[..., 1]
        return xp.sin(2 * math.pi * (x - t)) * xp.exp(-t)

    def f(self, X):
        return (4 * math.pi ** 2 * self.nu - 1.0) * self.u(X)


class PolynomialProblem(Problem):
    """Space-time polynomial ``u`` of total degree ``deg`` with an affine
    velocity; ``f = u_t + div(a u) - nu lap u`` exactly.  Used for the
    polynomial-reproduction (consistency) check."""

    def __init__(self, d, deg, nu, seed=0, a_const=None, a_lin=None):
        rng = np.random.default_rng(seed)
        self.d = d
        self.nu = nu
        self.deg = deg
        D = d + 1
        exps = []
        import itertools
        for e in itertools.product(range(deg + 1), repeat=D):
            if sum(e) <= deg:
                exps.append(e)
        self.exps = np.array(exps)
        self.coef = rng.standard_normal(len(exps))
        self.a_const = np.asarray(a_const if a_const is not None else rng.uniform(0.5, 1.0, d))
        self.a_lin = np.asarray(a_lin if a_lin is not None else 0.2 * rng.standard_normal((d, D)))

    def _mono(self, X, e, dk=None, dk2=None):
        xp = _ns(X)
        out = xp.ones_like(X[..., 0])
        ee = list(e)
        c = 1.0
        for k in (dk, dk2):
            if k is None:
                continue
            if ee[k] == 0:
                return xp.zeros_like(X[..., 0])
            c *= ee[k]
            ee[k] -= 1
        for k, p in enumerate(ee):
            if p:
                out = out * X[..., k] ** p
        return c * out

    def u(self, X):
        return sum(c * self._mono(X, e) for c, e in zip(self.coef, self.exps))

    def a(self, X):
        xp = _ns(X)
        cols = []
        for i in range(self.d):
            v = self.a_const[i] + sum(self.a_lin[i, k] * X[..., k] for k in range(self.d + 1))
            cols.append(v)
        return xp.stack(cols, axis=-1)

    def f(self, X):
        # conservative operator d_t u + div(a u) - nu lap u (the bilinear form's
        # volume term -u a_hat.grad_hat v is its weak form); equal to the
        # advective form when div a = 0, as for every other workload
        a = self.a(X)
        diva = sum(self.a_lin[i, i + 1] for i in range(self.d))
        out = sum(c * self._mono(X, e, 0) for c, e in zip(self.coef, self.exps))
        out = out + diva * self.u(X)
        for i in range(self.d):
            du = sum(c * self._mono(X, e, i + 1) for c, e in zip(self.coef, self.exps))
            out = out + a[..., i] * du
            lap = sum(c * self._mono(X, e, i + 1, i + 1) for c, e in zip(self.coef, self.exps))
            out = out - self.nu * lap
        return out


class RotatingGaussian(Problem):
    """Rotating, diffusing Gaussian (Section 4.1 family).

    ``a = w (-(x2-c2), x1-c1)``; with ``xt = R(-w t)(x-c) + c``,
    ``u = s^2/(s^2+2 nu t) exp(-|xt-x0|^2 / (2 s^2 + 4 nu t))`` and ``f = 0``.
    The paper's pulse is ``w=4``, ``c=0``, ``x0=(-0.2,0.1)``, ``s=0.1``; the
    slab workload is ``w=1``, ``c=(0.5,0.5)``, ``x0=(0.3,0.5)``, ``s=0.05``.
    """

    def __init__(self, nu, omega=1.0, center=(0.5, 0.5), x0=(0.3, 0.5), sigma=0.05):
        self.d = 2
        self.nu = nu
        self.omega = omega
        self.center = center
        self.x0 = x0
        self.sigma = sigma

    def a(self, X):
        xp = _ns(X)
        return xp.stack([-self.omega * (X[..., 2] - self.center[1]),
                         self.omega * (X[..., 1] - self.center[0])], axis=-1)

    def u(self, X):
        xp = _ns(X)
        t = X[..., 0]
        y1 = X[..., 1] - self.center[0]
        y2 = X[..., 2] - self.center[1]
        c, s = xp.cos(self.omega * t), xp.sin(self.omega * t)
        xt1 = y1 * c + y2 * s + self.center[0]
        xt2 = -y1 * s + y2 * c + self.center[1]
        s2 = self.sigma ** 2
        r2 = (xt1 - self.x0[0]) ** 2 + (xt2 - self.x0[1]) ** 2
        return s2 / (s2 + 2 * self.nu * t) * xp.exp(-r2 / (2 * s2 + 4 * self.nu * t))


def paper_pulse(nu):
    """The rotating pulse of Section 4.1 (``a = (-4 x2, 4 x1)``)."""
    return RotatingGaussian(nu, omega=4.0, center=(0.0, 0.0), x0=(-0.2, 0.1), sigma=0.1)


def slab_hill(nu=1e-4):
    """The slab workload: Gaussian hill at (0.3,0.5), width 0.05, rotating about
    (0.5,0.5) at unit angular speed."""
    return RotatingGaussian(nu, omega=1.0, center=(0.5, 0.5), x0=(0.3, 0.5), sigma=0.05)


class SmoothPlusFront(Problem):
    """2+1-D all-at-once workload: constant ``a``, smooth mode plus a
    transported tanh front of width ``w``:
    ``u = sin(pi x1) sin(pi x2) cos(2 pi t) + 1/2 tanh((s.x - |a| t - 0.2)/w)``
    with ``s = a/|a|``; the front is transported exactly, so it contributes
    only ``-nu lap`` to ``f``."""

    def __init__(self, nu, a=(1.0, 0.5), width=1e-2):
        self.d = 2
        self.nu = nu
        self.av = a
        self.width = width
        na = math.hypot(a[0], a[1])
        self.na = na
        self.s = (a[0] / na, a[1] / na)

    def a(self, X):
        xp = _ns(X)
        return xp.stack([xp.full_like(X[..., 1], self.av[0]),
                         xp.full_like(X[..., 1], self.av[1])], axis=-1)

    def _z(self, X):
        return (self.s[0] * X[..., 1] + self.s[1] * X[..., 2] - self.na * X[..., 0] - 0.2) / self.width

    def u(self, X):
        xp = _ns(X)
        t, x1, x2 = X[..., 0], X[..., 1], X[..., 2]
        sm = xp.sin(math.pi * x1) * xp.sin(math.pi * x2) * xp.cos(2 * math.pi * t)
        return sm + 0.5 * xp.tanh(self._z(X))

    def f(self, X):
        xp = _ns(X)
        t, x1, x2 = X[..., 0], X[..., 1], X[..., 2]
        pi = math.pi
        s1, s2 = xp.sin(pi * x1), xp.sin(pi * x2)
        c1, c2 = xp.cos(pi * x1), xp.cos(pi * x2)
        ct, st = xp.cos(2 * pi * t), xp.sin(2 * pi * t)
        smooth = (-2 * pi * s1 * s2 * st
                  + pi * (self.av[0] * c1 * s2 + self.av[1] * s1 * c2) * ct
                  + 2 * pi ** 2 * self.nu * s1 * s2 * ct)
        z = self._z(X)
        th = xp.tanh(z)
        sech2 = 1.0 - th * th
        g2 = -(1.0 / self.width ** 2) * sech2 * th      # second derivative of tanh(z)/2 in s.x
        return smooth - self.nu * g2


class GaussianSources(Problem):
    """Differentiation workload: ``a = (1, 0)``, zero boundary/initial data,
    ``f = sum_k c_k exp(-|X - X_k|^2 / (2 w^2))`` in space-time."""
    has_exact = False

    def __init__(self, nu, centers, coeffs, width=0.1, a=(1.0, 0.0)):
        self.d = 2
        self.nu = nu
        self.centers = np.asarray(centers, dtype=np.float64)
        self.coeffs = np.asarray(coeffs, dtype=np.float64)
        self.width = width
        self.av = a

    def a(self, X):
        xp = _ns(X)
        return xp.stack([xp.full_like(X[..., 1], self.av[0]),
                         xp.full_like(X[..., 1], self.av[1])], axis=-1)

    def basis(self, X):
        """``phi_k(X)`` for every source, shape ``X.shape[:-1] + (K,)``."""
        xp = _ns(X)
        C = self.centers
        if xp is not np:
            import torch
            C = torch.as_tensor(C, dtype=X.dtype, device=X.device)
        r2 = ((X[..., None, :] - C) ** 2).sum(-1)
        return xp.exp(-r2 / (2 * self.width ** 2))

    def f(self, X):
        xp = _ns(X)
        c = self.coeffs
        if xp is not np:
            import torch
            c = torch.as_tensor(c, dtype=X.dtype, device=X.device)
        return self.basis(X) @ c

    def u(self, X):
        raise NotImplementedError

    def g_dirichlet(self, X):
        xp = _ns(X)
        return xp.zeros_like(X[..., 0])

    def g_neumann(self, X, on_bottom):
        xp = _ns(X)
        return xp.zeros_like(X[..., 0])


def c5_sources(n_src=256, seed_centers=1, seed_target=0, seed_eval=2):
    """Seeded source centres (uniform in [0.1,0.9]^3), target and evaluation
    amplitudes (standard normal), numpy PCG64."""
    centers = np.random.default_rng(seed_centers).uniform(0.1, 0.9, (n_src, 3))
    c_target = np.random.default_rng(seed_target).standard_normal(n_src)
    c_eval = np.random.default_rng(seed_eval).standard_normal(n_src)
    return centers, c_target, c_eval


class MovingInternalLayer(Problem):
    """Moving internal layer (Section 4.2) on the space-time unit cube:
    ``nu = 0``, ``f = 0``, ``a = (x2, -x1)``; ``u = 1`` where ``|x| < 1`` and
    ``atan2(x2, x1) > pi/2 - t``, else 0.  The characteristics are circles
    about the origin run clockwise, so the front enters through ``x1 = 0``
    (value 1 for ``x2 < 1``) and sweeps the square; the initial data is 0.
    The spatial boundary data is this exact solution."""

    def __init__(self):
        self.d = 2
        self.nu = 0.0

    def a(self, X):
        xp = _ns(X)
        return xp.stack([X[..., 2], -X[..., 1]], axis=-1)

    def u(self, X):
        xp = _ns(X)
        t, x1, x2 = X[..., 0], X[..., 1], X[..., 2]
        inside = (x1 * x1 + x2 * x2 < 1.0) & (xp.arctan2(x2, x1) > math.pi / 2 - t)
        return xp.where(inside, xp.ones_like(t), xp.zeros_like(t))


class SwirlFlow(Problem):
    """A velocity that is not affine in x, for the assembly with the velocity
    at the quadrature points: 1+1-D ``a = 1 + 0.5 sin(2 pi x) cos(t)``,
    2+1-D ``a = (1 + 0.3 sin(pi x2) cos(t), 0.5 + 0.3 sin(pi x1))``.  Boundary
    and initial data from ``u = sin(pi x1) e^-t`` (times ``sin(pi x2) + 1`` in
    2+1-D), ``f = 0``; no exact solution."""
    has_exact = False

    def __init__(self, d, nu):
        self.d = d
        self.nu = nu

    def a(self, X):
        xp = _ns(X)
        t = X[..., 0]
        if self.d == 1:
            return (1.0 + 0.5 * xp.sin(2 * math.pi * X[..., 1]) * xp.cos(t))[..., None]
        return xp.stack([1.0 + 0.3 * xp.sin(math.pi * X[..., 2]) * xp.cos(t),
                         0.5 + 0.3 * xp.sin(math.pi * X[..., 1])], axis=-1)

    def a_vertices(self, vert):
        return self.a(vert)

    def u(self, X):
        xp = _ns(X)
        v = xp.sin(math.pi * X[..., 1]) * xp.exp(-X[..., 0])
        if self.d == 2:
            v = v * (xp.sin(math.pi * X[..., 2]) + 1.0)
        return v
