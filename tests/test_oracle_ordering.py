"""Pins of the oracle's flow order and ordered Gauss-Seidel relaxation
(Lemma 3.1, Section 3.3; the relaxation schedule of Section 4).  No GPU."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import air, krylov
from oracle.drivers import setup_problem
from workloads import kuhn_cube_mesh, slab_prism_tet_mesh, square_tri_mesh
from workloads.problems import SmoothPlusFront, slab_hill, C1Advection1D


@pytest.fixture(scope="module")
def kuhn_nu0():
    # pure advection with a constant velocity: the element graph is acyclic
    v, c = kuhn_cube_mesh(4)
    return setup_problem(v, c, SmoothPlusFront(0.0), 1)


@pytest.fixture(scope="module")
def slab_diff():
    v, c = slab_prism_tet_mesh(4, 1 / 16)
    return setup_problem(v, c, slab_hill(1e-2), 1)


def _block_dense_weights(A, b):
    """Block weights by plain loops over a dense copy (independent of
    air.block_weights)."""
    Ad = A.toarray()
    nb = Ad.shape[0] // b
    W = np.zeros((nb, nb))
    for I in range(nb):
        for J in range(nb):
            if I != J:
                W[I, J] = np.abs(Ad[I * b:(I + 1) * b, J * b:(J + 1) * b]).max()
    return W


def _longest_path_levels(W, ratio=1.5):
    """Level = length of the longest chain of predecessors, by memoised
    recursion over the dominance relation (DAG case)."""
    nb = W.shape[0]
    preds = [[J for J in range(nb) if J != I and W[I, J] > ratio * W[J, I]] for I in range(nb)]
    memo = {}

    def lev(I, depth=0):
        assert depth <= nb, "cycle"
        if I not in memo:
            memo[I] = 1 + max((lev(J, depth + 1) for J in preds[I]), default=-1)
        return memo[I]
    return np.array([lev(I) for I in range(nb)])


def test_lemma_3_1_block_lower_triangular(kuhn_nu0):
    """Pure advection on an acyclic element graph: the scaled facet matrix
    is block lower triangular in the flow order (Lemma 3.1)."""
    A, b = kuhn_nu0.Shat, kuhn_nu0.b
    lev, rounds, breaks = air.flow_levels(A, b)
    assert breaks == 0
    C = A.tocoo()
    I, J = C.row // b, C.col // b
    nz = (I != J) & (C.data != 0)
    assert np.all(lev[J[nz]] < lev[I[nz]])
    assert rounds == lev.max() + 1


def test_levels_are_longest_paths(kuhn_nu0):
    A, b = kuhn_nu0.Shat, kuhn_nu0.b
    lev, _, breaks = air.flow_levels(A, b)
    assert breaks == 0
    ref = _longest_path_levels(_block_dense_weights(A, b))
    np.testing.assert_array_equal(lev, ref)


def test_cycle_break_rule():
    """Hand-worked example, b = 1: 3 -> 0 -> 1 -> 2 -> 0 (a cycle through 0).
    Round 0 takes 3; then nothing is ready and 0, 1, 2 each wait for one
    predecessor, so 0 (smallest index) is placed alone; then 1, then 2."""
    n = 4
    A = np.eye(n)
    for i, j in ((1, 0), (2, 1), (0, 2), (0, 3)):   # dominant couplings: j precedes i
        A[i, j] = 0.5
        A[j, i] = 0.1
    lev, rounds, breaks = air.flow_levels(sp.csr_matrix(A), 1)
    np.testing.assert_array_equal(lev, [1, 2, 3, 0])
    assert (rounds, breaks) == (4, 1)


def test_balanced_pairs_stay_unordered():
    A = np.eye(4)
    A[0, 2], A[2, 0] = 0.3, 0.25     # within the ratio 1.5: no order between 0 and 2
    A[1, 0] = 0.2                    # 0 precedes 1 (A[0, 1] = 0)
    A[3, 1], A[1, 3] = 0.5, 0.25     # ratio 2: 1 precedes 3
    lev, rounds, breaks = air.flow_levels(sp.csr_matrix(A), 1)
    np.testing.assert_array_equal(lev, [0, 1, 0, 2])
    assert (rounds, breaks) == (3, 0)
    lev, _, _ = air.flow_levels(sp.csr_matrix(A), 1, ratio=1.1)   # now 2 precedes 0
    np.testing.assert_array_equal(lev, [1, 2, 0, 3])


def _level_gs(A, b_, x, rows, row_level):
    """Gauss-Seidel over levels, Jacobi inside a level, one row at a time:
    a row reads the values of its own level as they were when the level
    began and the current values of every other row."""
    Ad = A.toarray()
    x = x.copy()
    for k in np.unique(row_level):
        snap = x.copy()
        same = np.zeros(len(x), dtype=bool)
        same[rows[row_level == k]] = True
        for i in rows[row_level == k]:
            xt = np.where(same, snap, x)
            x[i] = snap[i] + (b_[i] - Ad[i] @ xt) / Ad[i, i]
    return x


def _sequential_gs(A, b_, x, rows_in_order):
    """Textbook forward Gauss-Seidel, one row at a time."""
    Ad = A.toarray()
    x = x.copy()
    for i in rows_in_order:
        x[i] += (b_[i] - Ad[i] @ x) / Ad[i, i]
    return x


@pytest.mark.parametrize("which", ["all", "F"])
@pytest.mark.parametrize("ratio", [1.5, 1.0])
def test_ordered_sweep_by_rows(slab_diff, which, ratio):
    A, b = slab_diff.Shat, slab_diff.b
    H = air.setup(A, relax="ordered_fa", block=b, order_ratio=ratio)
    L0 = H.levels[0]
    sw = L0.gs_all if which == "all" else L0.gs_F
    X = sw.X
    rng = np.random.default_rng(3)
    rhs = rng.standard_normal(A.shape[0])
    x0 = rng.standard_normal(A.shape[0])
    ref = _level_gs(A, rhs, x0, X, L0.blev[X // b])
    got = sw.apply(A, rhs, x0)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_ordered_sweep_without_level_couplings_is_gauss_seidel(kuhn_nu0):
    """Pure advection: no two blocks of a level are coupled, so the sweep is
    the textbook sequential sweep in level order."""
    A, b = kuhn_nu0.Shat, kuhn_nu0.b
    H = air.setup(A, relax="ordered", block=b)
    L0 = H.levels[0]
    n = A.shape[0]
    rng = np.random.default_rng(8)
    rhs, x0 = rng.standard_normal((2, n))
    X = np.arange(n)
    ref = _sequential_gs(A, rhs, x0, X[np.lexsort((X, L0.blev[X // b]))])
    np.testing.assert_allclose(L0.gs_all.apply(A, rhs, x0), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_ordered_sweep_is_exact_for_pure_advection(kuhn_nu0):
    """With the matrix block lower triangular in the flow order, one ordered
    sweep from zero is the exact solve, and FGMRES stops after one step."""
    A, b = kuhn_nu0.Shat, kuhn_nu0.b
    H = air.setup(A, relax="ordered", block=b)
    x = H.levels[0].gs_all.apply(A, kuhn_nu0.Hhat, np.zeros(A.shape[0]))
    ref = spla.spsolve(A.tocsc(), kuhn_nu0.Hhat)
    np.testing.assert_allclose(x, ref, rtol=0, atol=1e-11 * np.abs(ref).max())
    x, info = krylov.fgmres(A, kuhn_nu0.Hhat, lambda r: air.vcycle(H, r), tol=1e-8)
    assert info["iters"] == 1


@pytest.mark.parametrize("relax", ["ordered", "ordered_fa"])
def test_transposed_cycle_is_adjoint(slab_diff, relax):
    A, b = slab_diff.Shat, slab_diff.b
    H = air.setup(A, relax=relax, block=b)
    rng = np.random.default_rng(5)
    u, v = rng.standard_normal((2, A.shape[0]))
    lhs = v @ air.vcycle(H, u)
    rhs = u @ air.vcycle_T(H, v)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + abs(rhs))


def test_ordered_relaxation_converges_with_diffusion(slab_diff):
    A, b = slab_diff.Shat, slab_diff.b
    ref = spla.spsolve(A.tocsc(), slab_diff.Hhat)
    for relax in ("ordered", "ordered_fa"):
        H = air.setup(A, relax=relax, block=b)
        x, info = krylov.fgmres(A, slab_diff.Hhat, lambda r: air.vcycle(H, r), tol=1e-10)
        assert info["converged"]
        np.testing.assert_allclose(x, ref, rtol=0, atol=1e-8 * np.abs(ref).max())


def test_ordered_needs_scaled_blocks():
    v, c = square_tri_mesh(6)
    s = setup_problem(v, c, C1Advection1D(1e-2), 1, block_scale=False)
    with pytest.raises(ValueError):
        air.setup(s.Shat, relax="ordered", block=s.b)
