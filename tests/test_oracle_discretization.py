"""Pins of the oracle's discretization against what the mathematics and the
paper fix (no GPU)."""
import math
import itertools
import os

import numpy as np
import pytest

from oracle.quad import simplex_rule, bary
from oracle.basis import lattice, lagrange, lagrange_ref_grad
from oracle.hdg import Mesh, assemble, reconstruct, l2_error, dense_full_solve
from oracle.drivers import (setup_problem, direct_solve, solve_all_at_once, solve_slabs)
from workloads import (square_tri_mesh, slab_prism_tet_mesh, kuhn_cube_mesh,
                       pulse_slab_mesh, boundary_kinds)
from workloads.problems import (PolynomialProblem, C1Advection1D, paper_pulse,
                                SmoothPlusFront, slab_hill, MovingInternalLayer)

HERE = os.path.dirname(__file__)


@pytest.mark.parametrize("D", [1, 2, 3])
@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_quadrature_exact_on_simplex_monomials(D, n):
    # closed form: int_T xi^alpha = alpha! / (|alpha| + D)!  on the unit simplex
    xi, w = simplex_rule(D, n)
    for alpha in itertools.product(range(2 * n), repeat=D):
        k = sum(alpha)
        if k > 2 * n - 1:
            continue
        exact = np.prod([math.factorial(a) for a in alpha]) / math.factorial(k + D)
        got = np.sum(w * np.prod(xi ** np.array(alpha), axis=1))
        assert abs(got - exact) <= 1e-14 * max(1.0, exact), (alpha, got, exact)


@pytest.mark.parametrize("D", [1, 2, 3])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_lagrange_basis_nodal_and_partition(D, p):
    nodes = lattice(D, p) / p
    v, _ = lagrange(D, p, bary(nodes))
    assert np.allclose(v, np.eye(nodes.shape[0]), atol=1e-13)
    rng = np.random.default_rng(0)
    pts = rng.dirichlet(np.ones(D + 1), size=20)
    v, g = lagrange_ref_grad(D, p, pts)
    assert np.allclose(v.sum(-1), 1.0, atol=1e-13)
    assert np.allclose(g.sum(-2), 0.0, atol=1e-11)
    # derivative check by central differences in xi_1
    h = 1e-6
    xi = pts[:, 1:]
    e = np.zeros(D); e[0] = h
    vp, _ = lagrange(D, p, bary(xi + e))
    vm, _ = lagrange(D, p, bary(xi - e))
    assert np.allclose((vp - vm) / (2 * h), g[..., 0], atol=1e-7)


def test_facet_count_kuhn_and_dof_count():
    # Kuhn cube mesh: 12 n^3 + 6 n^2 facets (tets' triangles); DOFs = b * facets
    for n in (2, 3, 4):
        v, c = kuhn_cube_mesh(n)
        m = Mesh(v, c)
        assert m.nf == 12 * n ** 3 + 6 * n ** 2
        assert m.ne == 6 * n ** 3
    v, c = slab_prism_tet_mesh(8, 1 / 8)
    assert Mesh(v, c).ne == 384          # Table 1, 8 slabs: 384 elements per slab


@pytest.mark.parametrize("nu", [0.0, 1e-2])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_polynomial_reproduction_1p1(nu, p):
    prob = PolynomialProblem(1, p, nu, seed=1)
    v, c = square_tri_mesh(3)
    s, lam, U, _ = solve_all_at_once(v, c, prob, p)
    assert l2_error(s, U, prob.u) < 1e-12


@pytest.mark.parametrize("mesh", ["kuhn", "slab"])
@pytest.mark.parametrize("nu", [0.0, 1e-2])
@pytest.mark.parametrize("p", [1, 2])
def test_polynomial_reproduction_2p1(mesh, nu, p):
    prob = PolynomialProblem(2, p, nu, seed=2)
    v, c = kuhn_cube_mesh(2) if mesh == "kuhn" else slab_prism_tet_mesh(2, 0.3)
    s, lam, U, _ = solve_all_at_once(v, c, prob, p)
    assert l2_error(s, U, prob.u) < 1e-12
    # the trace equals u on every free facet: check at facet nodes
    from oracle.hdg import full_trace
    lamf = full_trace(s, lam).reshape(s.mesh.nf, s.b)
    nodes = lattice(2, p) / p
    mu = bary(nodes)
    V = s.mesh.vert[s.mesh.facet_vert]                        # [nf][3][3]
    X = np.einsum("qs,fsc->fqc", mu, V)
    assert np.abs(lamf - prob.u(X)).max() < 1e-11


def test_condensation_matches_dense_full_system():
    prob = PolynomialProblem(2, 3, 1e-2, seed=5)     # degree p+1: not reproduced
    v, c = kuhn_cube_mesh(2)
    s = setup_problem(v, c, prob, 2)
    lam = direct_solve(s)
    U = reconstruct(s, lam)
    Ud, lamd = dense_full_solve(s)
    assert np.abs(lam - lamd).max() < 1e-11 * np.abs(lamd).max()
    assert np.abs(U - Ud).max() < 1e-11 * np.abs(Ud).max()


@pytest.mark.parametrize("p", [1, 2])
def test_convergence_order_c1(p):
    # manufactured u = sin(2 pi (x - t)) e^-t: error O(h^(p+1))
    prob = C1Advection1D(1e-4)
    errs = []
    for n in (8, 16, 32):
        v, c = square_tri_mesh(n)
        s, lam, U, _ = solve_all_at_once(v, c, prob, p)
        errs.append(l2_error(s, U, prob.u))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - (p + 1)) < 0.25), rates


def _table1():
    rows = {}
    for line in open(os.path.join(HERE, "golden", "table1_slab_by_slab.txt")):
        if line.startswith("#") or not line.strip():
            continue
        nu, N, ne, e1, e2, e3 = line.split()
        rows[(float(nu), int(N))] = (int(ne), float(e1), float(e2), float(e3))
    return rows


@pytest.mark.parametrize("nu", [1e-2, 1e-6])
@pytest.mark.parametrize("p", [1, 2])
def test_table1_slab_rows(nu, p):
    # Table 1: the paper's slab meshes are not available (orientation of the
    # prism split unknown), so magnitudes are pinned within a factor 3 and the
    # observed rate between 8 and 16 slabs within 0.8 of the paper's (the
    # coarsest rows are pre-asymptotic).
    tab = _table1()
    prob = paper_pulse(nu)
    errs = []
    for N in (8, 16):
        assert tab[(nu, N)][0] == 6 * N * N
        e, _, _ = solve_slabs(lambda k: pulse_slab_mesh(N, k), N, prob, p)
        errs.append(e)
    ref = [tab[(nu, N)][p] for N in (8, 16)]
    for e, r in zip(errs, ref):
        assert r / 3 < e < 3 * r, (errs, ref)
    rate = math.log2(errs[0] / errs[1])
    rref = math.log2(ref[0] / ref[1])
    assert abs(rate - rref) < 0.8, (rate, rref)


def test_pure_advection_transported_profile_rate():
    # nu = 0: a smooth profile transported along a = (1, 0.5) converges at p+1
    class Transport(SmoothPlusFront):
        def u(self, X):
            z = X[..., 1] - self.av[0] * X[..., 0]
            y = X[..., 2] - self.av[1] * X[..., 0]
            return np.sin(np.pi * z) * np.cos(np.pi * y)

        def f(self, X):
            return np.zeros_like(X[..., 0])
    prob = Transport(0.0)
    errs = []
    for n in (3, 6):
        v, c = kuhn_cube_mesh(n)
        s, lam, U, _ = solve_all_at_once(v, c, prob, 1)
        errs.append(l2_error(s, U, prob.u))
    assert 1.6 < math.log2(errs[0] / errs[1]) < 2.6, errs


def test_moving_internal_layer_converges():
    # Section 4.2, uniform meshes: nu = 0, a = (x2, -x1), a discontinuous
    # front entering through x1 = 0.  The L2 error of a discontinuous
    # solution falls like h^(1/2); with the velocity or the inflow data
    # wrong the discrete solution does not approach u (reversed rotation
    # leaves the error at 0.50 on both meshes).
    prob = MovingInternalLayer()
    errs = []
    for n in (4, 8):
        v, c = kuhn_cube_mesh(n)
        s, lam, U, _ = solve_all_at_once(v, c, prob, 1)
        errs.append(l2_error(s, U, prob.u))
    assert errs[1] < 0.16, errs
    assert 0.25 < math.log2(errs[0] / errs[1]) < 1.0, errs


def test_lemma31_acyclic_facet_graph_pure_advection():
    # Lemma 3.1: with nu = 0 and a constant velocity the scaled matrix is block
    # lower triangular in a topological order of its facet graph, and one
    # ordered block forward sweep reproduces the direct solve.
    prob = SmoothPlusFront(0.0)
    v, c = kuhn_cube_mesh(3)
    s = setup_problem(v, c, prob, 1)
    b = s.b
    A = s.Shat.tocoo()
    nb = s.n // b
    bi, bj = A.row // b, A.col // b
    keep = (bi != bj) & (np.abs(A.data) > 1e-13)
    edges = set(zip(bi[keep], bj[keep]))          # block row i depends on block j
    indeg = np.zeros(nb, dtype=int)
    succ = [[] for _ in range(nb)]
    for i, j in edges:
        succ[j].append(i)
        indeg[i] += 1
    order = [k for k in range(nb) if indeg[k] == 0]
    head = 0
    while head < len(order):
        k = order[head]; head += 1
        for i in succ[k]:
            indeg[i] -= 1
            if indeg[i] == 0:
                order.append(i)
    assert len(order) == nb, "facet graph has a cycle"
    x = np.zeros(s.n)
    Sd = s.Shat.tocsr()
    for k in order:
        rows = slice(k * b, (k + 1) * b)
        r = s.Hhat[rows] - Sd[rows] @ x
        x[rows] += r           # diagonal blocks are the identity
    ref = direct_solve(s)
    assert np.linalg.norm(s.S @ x - s.H) <= 1e-11 * np.linalg.norm(s.H)
    assert np.abs(x - ref).max() <= 1e-10 * np.abs(ref).max()
