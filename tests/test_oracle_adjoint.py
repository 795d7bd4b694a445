"""Pins of the oracle's adjoint gradients: central finite differences and a
dense transposed solve (no GPU)."""
import numpy as np
import pytest

from oracle import adjoint, air
from oracle.drivers import setup_problem, direct_solve, problem_g
from workloads import kuhn_cube_mesh, map_vertices_c5
from workloads.problems import GaussianSources, c5_sources


@pytest.fixture(scope="module")
def c5_tiny():
    v, c = kuhn_cube_mesh(2)
    v = map_vertices_c5(v)
    centers, ct, ce = c5_sources(6)
    return v, c, centers, ct, ce


def _solve(v, c, centers, coef, nu):
    prob = GaussianSources(nu, centers, coef)
    s = setup_problem(v, c, prob, 2)
    return s, direct_solve(s), prob


def test_gradients_vs_fd_and_dense(c5_tiny):
    v, c, centers, ct, ce = c5_tiny
    nu = 1e-3
    _, lam_t, _ = _solve(v, c, centers, ct, nu)
    s, lam, prob = _solve(v, c, centers, ce, nu)
    g_fn = problem_g(prob, s.mesh, s.kinds, 0.0, 1.0)
    J, dc, dnu, _ = adjoint.misfit_and_grads(s, lam, lam_t, prob.a, prob.f, g_fn, prob.basis)
    Jd, dcd, dnud, _ = adjoint.misfit_and_grads(s, lam, lam_t, prob.a, prob.f, g_fn, prob.basis,
                                                dense=True)
    assert np.allclose(dc, dcd, rtol=1e-10, atol=1e-12)
    assert abs(dnu - dnud) <= 1e-9 * abs(dnud)
    h = 1e-6
    for k in range(len(ce)):
        e = np.zeros(len(ce)); e[k] = h
        Jp = 0.5 * np.sum((_solve(v, c, centers, ce + e, nu)[1] - lam_t) ** 2)
        Jm = 0.5 * np.sum((_solve(v, c, centers, ce - e, nu)[1] - lam_t) ** 2)
        assert abs((Jp - Jm) / (2 * h) - dc[k]) <= 1e-6 * max(1.0, abs(dc[k]))
    Jp = 0.5 * np.sum((_solve(v, c, centers, ce, nu + h)[1] - lam_t) ** 2)
    Jm = 0.5 * np.sum((_solve(v, c, centers, ce, nu - h)[1] - lam_t) ** 2)
    assert abs((Jp - Jm) / (2 * h) - dnu) <= 1e-6 * max(1.0, abs(dnu))


def test_adjoint_air_solve_matches_dense(c5_tiny):
    v, c, centers, ct, ce = c5_tiny
    s, lam, prob = _solve(v, c, centers, ce, 1e-3)
    g = np.random.default_rng(4).standard_normal(s.n)
    H = air.setup(s.Shat, max_coarse=40)
    la, info = adjoint.adjoint_solve(s, H, g, tol=1e-13)
    ld = adjoint.adjoint_dense(s, g)
    assert info["converged"]
    assert np.linalg.norm(la - ld) <= 1e-10 * np.linalg.norm(ld)
