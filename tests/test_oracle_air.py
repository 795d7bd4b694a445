"""Pins of the oracle's AIR setup, cycles and Krylov solver (no GPU)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import air, krylov
from oracle.drivers import setup_problem, direct_solve, air_fgmres_solve
from workloads import square_tri_mesh, slab_prism_tet_mesh, kuhn_cube_mesh
from workloads.problems import C1Advection1D, slab_hill, SmoothPlusFront


@pytest.fixture(scope="module")
def c1_sys():
    v, c = square_tri_mesh(16)
    return setup_problem(v, c, C1Advection1D(1e-4), 1)


@pytest.fixture(scope="module")
def slab_sys():
    v, c = slab_prism_tet_mesh(6, 1 / 6)
    return setup_problem(v, c, slab_hill(1e-3), 2)


def _dense_strength(Ad, theta):
    n = Ad.shape[0]
    S = np.zeros((n, n), dtype=bool)
    for i in range(n):
        off = [abs(Ad[i, k]) for k in range(n) if k != i]
        m = max(off) if off else 0.0
        for j in range(n):
            if j != i and m > 0 and abs(Ad[i, j]) >= theta * m * (1 - 1e-12) and Ad[i, j] != 0:
                S[i, j] = True
    return S


def test_strength_brute_force(c1_sys):
    A = c1_sys.Shat[:200, :200].tocsr()
    A.sort_indices()
    st = air.strength(A, 0.25)
    Sd = np.zeros(A.shape, dtype=bool)
    r = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    Sd[r[st], A.indices[st]] = True
    assert np.array_equal(Sd, _dense_strength(A.toarray(), 0.25))


def test_hash44_is_injective():
    h = air.hash44(np.arange(200000), 3)
    assert np.unique(h).size == 200000
    assert int(h.max()) < (1 << 44)


def _pmis_loops(n, S_rows, level):
    """PMIS written with plain loops over points (tiny inputs only)."""
    infl = [0] * n
    for i in range(n):
        for j in S_rows[i]:
            infl[j] += 1
    key = [infl[i] * (1 << 44) + int(air.hash44(i, level)) for i in range(n)]
    nbrs = [set() for _ in range(n)]
    for i in range(n):
        for j in S_rows[i]:
            nbrs[i].add(j)
            nbrs[j].add(i)
    state = ["F" if infl[i] == 0 else "U" for i in range(n)]
    while "U" in state:
        newc = [i for i in range(n) if state[i] == "U"
                and all(key[i] > key[j] for j in nbrs[i] if state[j] == "U")]
        for i in newc:
            state[i] = "C"
        for j in range(n):
            if state[j] == "U" and any(state[i] == "C" for i in S_rows[j]):
                state[j] = "F"
    return np.array([1 if s == "C" else 0 for s in state])


@pytest.mark.parametrize("which", ["c1", "slab"])
def test_pmis_matches_loop_definition_and_invariants(which, c1_sys, slab_sys):
    s = c1_sys if which == "c1" else slab_sys
    A = s.Shat[:600, :600].tocsr() if which == "slab" else s.Shat
    A.sort_indices()
    st = air.strength(A, 0.25)
    cf = air.pmis(A, st, 2)
    r = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    si, sj = r[st], A.indices[st]
    S_rows = [[] for _ in range(A.shape[0])]
    for i, j in zip(si, sj):
        S_rows[i].append(j)
    assert np.array_equal(cf, _pmis_loops(A.shape[0], S_rows, 2))
    # every F point that something depends on has a strong C dependency
    infl = np.bincount(sj, minlength=A.shape[0])
    hasC = np.zeros(A.shape[0], dtype=bool)
    hasC[si[cf[sj] == 1]] = True
    assert np.all(hasC[(cf == 0) & (infl > 0)])
    # no point that depends on nothing strongly and influences nothing is C
    assert np.all(cf[infl == 0] == 0)


def test_one_point_interpolation_preserves_constants(slab_sys):
    A = slab_sys.Shat
    st = air.strength(A, 0.25)
    cf = air.pmis(A, st, 0)
    cidx = np.cumsum(cf) - 1
    P = air.one_point_P(A, st, cf, cidx)
    rs = np.asarray(P.sum(1)).ravel()
    r = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    hasC = np.zeros(A.shape[0], dtype=bool)
    hasC[r[st & (cf[A.indices] == 1)]] = True
    assert np.all(rs[(cf == 1) | hasC] == 1.0)
    assert np.all(rs[(cf == 0) & ~hasC] == 0.0)
    # the chosen C neighbour is a strongest one
    Ad = A.tocsr()
    for i in np.nonzero((cf == 0) & hasC)[0][:200]:
        j = np.nonzero(cf == 1)[0][P[i].indices[0]]
        lo, hi = Ad.indptr[i], Ad.indptr[i + 1]
        cand = [abs(Ad.data[k]) for k in range(lo, hi) if st[k] and cf[Ad.indices[k]] == 1]
        assert abs(Ad[i, j]) >= max(cand) * (1 - 1e-12)


@pytest.mark.parametrize("which", ["c1", "slab"])
def test_lair_rows_annihilate_f_neighbourhood(which, c1_sys, slab_sys):
    s = c1_sys if which == "c1" else slab_sys
    A = s.Shat
    st = air.strength(A, 0.25)
    cf = air.pmis(A, st, 0)
    cidx = np.cumsum(cf) - 1
    R, nfall = air.lair_R(A, st, cf, cidx)
    RA = (R @ A).tocsr()
    Cpts = np.nonzero(cf == 1)[0]
    Ad = A.tocsr()
    checked = 0
    for ci, i in enumerate(Cpts):
        assert R[ci, i] == 1.0
        lo, hi = Ad.indptr[i], Ad.indptr[i + 1]
        Ni = [Ad.indices[k] for k in range(lo, hi) if st[k] and cf[Ad.indices[k]] == 0]
        if not Ni or R[ci].nnz == 1:
            continue
        rownorm = np.abs(Ad[i].data).max()
        for j in Ni:
            assert abs(RA[ci, j]) <= 1e-12 * max(rownorm, 1.0)
        checked += 1
    assert checked > 0


def _bfs_f_neighbourhood(A, st, cf, i, distance):
    """Points reachable from i through at most ``distance`` strong entries
    whose column is an F point, by breadth-first search on the dense mask."""
    D = A.toarray()
    n = D.shape[0]
    S = np.zeros((n, n), dtype=bool)
    r = np.repeat(np.arange(n), np.diff(A.indptr))
    S[r[st], A.indices[st]] = True
    seen, front = set(), {i}
    for _ in range(distance):
        nxt = set()
        for u in front:
            nxt |= {int(j) for j in np.nonzero(S[u])[0] if cf[j] == 0}
        nxt -= seen | {i}
        seen |= nxt
        front = nxt
    return sorted(seen)


@pytest.mark.parametrize("which", ["c1", "slab"])
def test_lair_distance_two(which, c1_sys, slab_sys):
    # Section 4 names distance-one lAIR; distance two widens N_i to the
    # F points two strong steps (through F points) from the C point.  Its
    # neighbourhoods equal a breadth-first search on the strength mask, and
    # every row still annihilates (R A)[i, N_i].
    s = c1_sys if which == "c1" else slab_sys
    A = s.Shat.tocsr()
    st = air.strength(A, 0.25)
    cf = air.pmis(A, st, 0)
    cidx = np.cumsum(cf) - 1
    nb1 = air.lair_neighbourhoods(A, st, cf, 1)
    nb2 = air.lair_neighbourhoods(A, st, cf, 2)
    Cpts = np.nonzero(cf == 1)[0]
    rng = np.random.default_rng(5)
    for i in rng.choice(Cpts, size=min(40, len(Cpts)), replace=False):
        assert list(nb2[int(i)]) == _bfs_f_neighbourhood(A, st, cf, int(i), 2)
        assert list(nb1[int(i)]) == _bfs_f_neighbourhood(A, st, cf, int(i), 1)
        assert set(nb1[int(i)]) <= set(nb2[int(i)])
    assert sum(len(v) for v in nb2.values()) > sum(len(v) for v in nb1.values())
    R, nfall = air.lair_R(A, st, cf, cidx, distance=2)
    RA = (R @ A).tocsr()
    checked = 0
    for ci, i in enumerate(Cpts):
        N = nb2[int(i)]
        if len(N) == 0 or R[ci].nnz == 1:
            continue
        rownorm = np.abs(A[i].data).max()
        assert np.all(np.abs(RA[ci, N].toarray()) <= 1e-11 * max(rownorm, 1.0))
        checked += 1
    assert checked > 0


def test_separate_restriction_threshold():
    # theta_R != theta_C: the splitting follows theta_C, the neighbourhoods
    # theta_R (a larger tolerance gives fewer strong F neighbours)
    v, c = kuhn_cube_mesh(4)
    s = setup_problem(v, c, SmoothPlusFront(1e-3), 1)
    H1 = air.setup(s.Shat, theta=0.2)
    H2 = air.setup(s.Shat, theta=0.2, theta_r=0.5)
    assert np.array_equal(H1.levels[0].cf, H2.levels[0].cf)
    assert H2.levels[0].R.nnz < H1.levels[0].R.nnz


def test_batched_lu_matches_library_solve():
    rng = np.random.default_rng(3)
    M = rng.standard_normal((50, 7, 7))
    rhs = rng.standard_normal((50, 7))
    x, bad = air.batched_lu_solve(M, rhs)
    assert not bad.any()
    assert np.allclose(x, np.linalg.solve(M, rhs[..., None])[..., 0], atol=1e-12)
    M[0] = 0.0
    _, bad = air.batched_lu_solve(M, rhs)
    assert bad[0] and not bad[1:].any()


def test_ideal_restriction_two_grid_exact():
    # Section 3: with R_ideal = [-A_cf A_ff^-1, I] and any P = [W; I],
    # R A P = A_cc - A_cf A_ff^-1 A_fc and coarse correction followed by an exact
    # F solve removes all error.
    rng = np.random.default_rng(7)
    n, nc = 12, 5
    A = rng.standard_normal((n, n)) + 6 * np.eye(n)
    f = np.arange(n - nc); c = np.arange(n - nc, n)
    Aff, Afc, Acf, Acc = A[np.ix_(f, f)], A[np.ix_(f, c)], A[np.ix_(c, f)], A[np.ix_(c, c)]
    R = np.hstack([-Acf @ np.linalg.inv(Aff), np.eye(nc)])
    W = rng.standard_normal((n - nc, nc))
    P = np.vstack([W, np.eye(nc)])
    schur = Acc - Acf @ np.linalg.solve(Aff, Afc)
    assert np.allclose(R @ A @ P, schur, atol=1e-12)
    b = rng.standard_normal(n)
    x = P @ np.linalg.solve(R @ A @ P, R @ b)
    r = b - A @ x
    x[f] += np.linalg.solve(Aff, r[f])
    assert np.allclose(x, np.linalg.solve(A, b), atol=1e-11)


def test_vcycle_linear_and_transpose_identity(slab_sys):
    H = air.setup(slab_sys.Shat, max_coarse=50)
    assert H.nlev >= 3
    rng = np.random.default_rng(11)
    n = slab_sys.n
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    Bx, By = air.vcycle(H, x), air.vcycle(H, y)
    assert np.allclose(air.vcycle(H, 2 * x - 3 * y), 2 * Bx - 3 * By, atol=1e-10 * np.abs(Bx).max())
    lhs = Bx @ y
    rhs = x @ air.vcycle_T(H, y)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(y) * np.linalg.norm(Bx) / np.linalg.norm(x) * 10


def test_fgmres_exact_preconditioner_one_iteration(c1_sys):
    A = c1_sys.Shat
    Ad = A.toarray()
    lu = np.linalg.inv(Ad)
    x, info = krylov.fgmres(A, c1_sys.Hhat, lambda r: lu @ r, tol=1e-12)
    assert info["iters"] == 1
    assert np.allclose(x, np.linalg.solve(Ad, c1_sys.Hhat), atol=1e-10)


def test_fgmres_restart_path_reaches_solution(c1_sys):
    A = c1_sys.Shat
    x, info = krylov.fgmres(A, c1_sys.Hhat, lambda r: r, tol=1e-10, restart=5, maxit=5000)
    assert info["converged"]
    ref = direct_solve(c1_sys)
    assert np.abs(x - ref).max() <= 1e-7 * np.abs(ref).max()


@pytest.mark.parametrize("which", ["c1", "slab"])
def test_air_fgmres_matches_direct(which, c1_sys, slab_sys):
    s = c1_sys if which == "c1" else slab_sys
    x, info = air_fgmres_solve(s, tol=1e-12)
    assert info["converged"] and info["iters"] < 30
    ref = direct_solve(s)
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)


def test_pure_advection_air_converges():
    prob = SmoothPlusFront(0.0)
    v, c = kuhn_cube_mesh(6)
    s = setup_problem(v, c, prob, 1)
    x, info = air_fgmres_solve(s, tol=1e-10)
    assert info["converged"] and info["iters"] <= 15


def test_bicgstab_exact_preconditioner_one_step(c1_sys):
    """With M = A^-1 the first half-step gives s = 0 (BiCGSTAB definition)."""
    A = c1_sys.Shat
    Ad = A.toarray()
    inv = np.linalg.inv(Ad)
    x, info = krylov.bicgstab(A, c1_sys.Hhat, lambda r: inv @ r, tol=1e-12)
    assert info["converged"] and info["iters"] == 1
    assert np.allclose(x, np.linalg.solve(Ad, c1_sys.Hhat), atol=1e-10)


def test_bicgstab_unpreconditioned_matches_scipy():
    """Without preconditioning the iteration is the textbook one; scipy's
    implementation of the same method takes the same number of steps
    (within one, for the placement of the convergence test) to the same
    solution."""
    from scipy.sparse.linalg import bicgstab as sp_bicgstab
    rng = np.random.default_rng(4)
    n = 60
    A = sp.csr_matrix(np.eye(n) * 4 + rng.standard_normal((n, n)) * 0.3)
    b = rng.standard_normal(n)
    x, info = krylov.bicgstab(A, b, lambda r: r, tol=1e-10, maxit=500)
    count = [0]
    xs, flag = sp_bicgstab(A, b, rtol=1e-10, atol=0.0, maxiter=500, callback=lambda xk: count.__setitem__(0, count[0] + 1))
    assert flag == 0 and info["converged"]
    assert abs(info["iters"] - count[0]) <= 1, (info["iters"], count[0])
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)


@pytest.mark.parametrize("which", ["c1", "slab"])
def test_air_bicgstab_matches_direct(which, c1_sys, slab_sys):
    from oracle.drivers import air_bicgstab_solve
    s = c1_sys if which == "c1" else slab_sys
    x, info = air_bicgstab_solve(s, tol=1e-12)
    ref = direct_solve(s)
    assert info["converged"]
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)
    _, i8f = air_fgmres_solve(s, tol=1e-8)
    _, i8b = air_bicgstab_solve(s, tol=1e-8)
    # two preconditioner applications per BiCGSTAB step
    assert i8b["iters"] <= i8f["iters"] + 2


def test_no_block_inverse_same_solution_more_iterations():
    """Without the facet-block scaling the system is S itself; its solution
    is the same Lambda, and AIR converges far worse on it (Section 4.1)."""
    v, c = slab_prism_tet_mesh(6, 1 / 6)
    prob = slab_hill(1e-3)
    s1 = setup_problem(v, c, prob, 2)
    s0 = setup_problem(v, c, prob, 2, block_scale=False)
    assert np.array_equal(np.eye(s0.b)[None].repeat(s0.Dinv.shape[0], 0), s0.Dinv)
    assert abs(s0.Shat - s1.S).max() == 0.0
    l1, l0 = direct_solve(s1), direct_solve(s0)
    assert np.linalg.norm(l1 - l0) <= 1e-12 * np.linalg.norm(l1)
    x0, i0 = air_fgmres_solve(s0, tol=1e-8, maxit=200)
    x1, i1 = air_fgmres_solve(s1, tol=1e-8)
    # with Jacobi relaxation the unscaled system stalls (relres ~0.7 after
    # 200 iterations); the scaled one converges in about a dozen
    assert i1["converged"] and i1["iters"] < 20
    assert not i0["converged"] or i0["iters"] > 3 * i1["iters"]


def _dense_cycle_matrix(H, l, sets_order, omega=1.0, transpose=False):
    """The V-cycle of Section 3 written out as one dense matrix: with
    ``E_k = I - M_k A`` and ``M_k = omega I_X D^-1 I_X^T`` the sweep on the
    set X_k, a post-relaxed cycle with zero initial guess is
    ``B = M_3 + E_3 M_2 + E_3 E_2 M_1 + E_3 E_2 E_1 P B_c R`` (sweeps 1, 2, 3
    in application order), and the coarsest level is ``A_L^-1``."""
    lev = H.levels[l]
    A = lev.A.toarray()
    n = A.shape[0]
    if l == H.nlev - 1:
        return np.linalg.inv(A)
    Bc = _dense_cycle_matrix(H, l + 1, sets_order, omega)
    d = np.diag(A)
    F = np.nonzero(lev.cf == 0)[0]
    C = np.nonzero(lev.cf == 1)[0]
    Ms = []
    for name in sets_order:
        X = F if name == "F" else C
        X = X[np.abs(d[X]) >= 1e-30]
        M = np.zeros((n, n))
        M[X, X] = omega / d[X]
        Ms.append(M)
    Id = np.eye(n)
    B = lev.P.toarray() @ Bc @ lev.R.toarray()
    for M in Ms:                          # B <- M + (I - M A) B, sweep by sweep
        B = M + (Id - M @ A) @ B
    return B.T if transpose else B


@pytest.mark.parametrize("relax, order", [("FFC", "FFC"), ("F", "F")])
def test_vcycle_equals_dense_cycle_formula(relax, order):
    """Pin of the cycle schedule: the oracle's V-cycle and its transpose equal
    the dense matrix of the coarse-grid correction followed by the post
    sweeps (F, F, C or F), to rounding, on a 3-level hierarchy; the wrong
    schedules (C first, or the C sweep dropped) are far from it."""
    v, c = square_tri_mesh(6)
    s = setup_problem(v, c, C1Advection1D(1e-3), 2)
    H = air.setup(s.Shat, max_coarse=40, relax=relax)
    assert H.nlev >= 3
    B = _dense_cycle_matrix(H, 0, order)
    rng = np.random.default_rng(21)
    X = rng.standard_normal((s.n, 4))
    nb = np.linalg.norm(B, 2)
    for k in range(X.shape[1]):
        x = X[:, k]
        assert np.linalg.norm(air.vcycle(H, x) - B @ x) <= 1e-13 * nb * np.linalg.norm(x)
        assert np.linalg.norm(air.vcycle_T(H, x) - B.T @ x) <= 1e-13 * nb * np.linalg.norm(x)
    if relax == "FFC":
        for wrong in ("CFF", "FF", "FCF"):
            Bw = _dense_cycle_matrix(H, 0, wrong)
            assert np.linalg.norm(Bw - B, 2) > 1e-6 * nb, wrong


def test_fp32_cycle_emulation():
    """The FP32 emulation of the cycle is the FP64 cycle up to FP32 rounding:
    its output is FP32, it agrees with the dense FP64 cycle matrix to about
    the FP32 unit roundoff, and not to FP64 accuracy (it really rounds)."""
    v, c = square_tri_mesh(6)
    s = setup_problem(v, c, C1Advection1D(1e-3), 2)
    H = air.setup(s.Shat, max_coarse=40)
    B = _dense_cycle_matrix(H, 0, "FFC")
    x = np.random.default_rng(22).standard_normal(s.n)
    ref, refT = B @ x, B.T @ x
    for z, zr in ((air.vcycle(H, x, dtype=np.float32), ref), (air.vcycle_T(H, x, dtype=np.float32), refT)):
        assert z.dtype == np.float32
        e = np.linalg.norm(z - zr) / np.linalg.norm(zr)
        assert 1e-9 < e < 1e-5, e


def _rs_brute(n, S_rows):
    """Ruge-Stueben first pass with a plain scan for the next C point (tiny
    inputs only): the same rules as the oracle's, without its heap."""
    ST = [[] for _ in range(n)]
    for i in range(n):
        for j in S_rows[i]:
            ST[j].append(i)
    lam = [len(ST[i]) for i in range(n)]
    state = [0 if lam[i] else -1 for i in range(n)]
    while any(s == 0 for s in state):
        best = None
        for i in range(n):
            if state[i] == 0 and (best is None or lam[i] > lam[best]):
                best = i
        i = best
        state[i] = 1
        for j in ST[i]:
            if state[j] == 0:
                state[j] = -1
                for k in S_rows[j]:
                    if state[k] == 0:
                        lam[k] += 1
        for k in S_rows[i]:
            if state[k] == 0:
                lam[k] -= 1
                if lam[k] == 0:
                    state[k] = -1
    return np.array([1 if s == 1 else 0 for s in state], dtype=np.int8)


@pytest.mark.parametrize("which", ["c1", "slab"])
def test_rs_first_pass_matches_scan_definition(which, c1_sys, slab_sys):
    s = c1_sys if which == "c1" else slab_sys
    A = s.Shat[:600, :600].tocsr()
    A.sort_indices()
    st = air.strength(A, 0.25)
    r = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    S_rows = [[] for _ in range(A.shape[0])]
    for a, b in zip(r[st], A.indices[st]):
        S_rows[a].append(int(b))
    cf = air.rs_first_pass(A, st)
    assert np.array_equal(cf, _rs_brute(A.shape[0], S_rows))
    # every F point that something depends on has a strong C dependency,
    # unless its own measure fell to zero
    assert 0 < cf.sum() < A.shape[0]


def test_rs_coarsening_hierarchy_solves(slab_sys):
    H = air.setup(slab_sys.Shat, max_coarse=50, coarsening="rs")
    assert H.nlev >= 3
    x, info = krylov.fgmres(slab_sys.Shat, slab_sys.Hhat, lambda r: air.vcycle(H, r), tol=1e-10)
    assert info["converged"] and info["iters"] < 40
    ref = direct_solve(slab_sys)
    assert np.linalg.norm(x - ref) <= 1e-8 * np.linalg.norm(ref)


@pytest.mark.parametrize("which", ["c1", "slab"])
def test_block_air_level_pins(which, c1_sys, slab_sys):
    """Block AIR on the facet blocks: the C/F splitting is constant on each
    block and is PMIS (its loop definition) on the strong block graph, whose
    weights are the blocks' largest magnitudes; every F block that something
    depends on has a strong C block; P is the block one-point interpolation times the identity of
    the block (each row of an F block takes weight 1 at the same row of its
    strongest C block); and every restriction row annihilates the rows of its
    block's strong F neighbourhood."""
    s = c1_sys if which == "c1" else slab_sys
    A = sp.csr_matrix(s.Shat)
    A.sort_indices()
    b = s.b
    cf, P, R, nf = air.block_air_level(A, b, 0.25, None, 0)
    nb = A.shape[0] // b
    cfb = cf.reshape(nb, b)
    assert np.all(cfb == cfb[:, :1])
    cfb = cfb[:, 0]
    W = air.block_graph(A, b)
    # the block weights are the largest magnitudes of the blocks' entries
    Ad = A.toarray()
    for I, J in [(int(i), int(W.indices[k])) for i in range(0, nb, max(1, nb // 25))
                 for k in range(W.indptr[i], W.indptr[i + 1])]:
        assert W[I, J] == np.abs(Ad[I * b:(I + 1) * b, J * b:(J + 1) * b]).max()
    sb = air.strength(W, 0.25)
    rW = np.repeat(np.arange(nb), np.diff(W.indptr))
    si, sj = rW[sb], W.indices[sb]
    S_rows = [[] for _ in range(nb)]
    for i, j in zip(si, sj):
        S_rows[i].append(j)
    assert np.array_equal(cfb, _pmis_loops(nb, S_rows, 0))
    infl = np.bincount(sj, minlength=nb)
    for I in np.nonzero((cfb == 0) & (infl > 0))[0]:
        assert np.any(cfb[sj[si == I]] == 1), I
    # P: weight 1 at the same row m of one C block, for every row of an F block
    Pd = P.tocsr()
    cidx = np.cumsum(cf) - 1
    for I in range(nb):
        cols = [Pd.indices[Pd.indptr[I * b + m]:Pd.indptr[I * b + m + 1]] for m in range(b)]
        if cfb[I] == 1:
            assert all(list(c) == [cidx[I * b + m]] for m, c in enumerate(cols))
        elif len(cols[0]):
            J = int(np.nonzero(cf == 1)[0][cols[0][0]]) // b
            assert all(list(c) == [cidx[J * b + m]] for m, c in enumerate(cols))
            assert np.allclose(Pd.data[Pd.indptr[I * b]:Pd.indptr[I * b + b]], 1.0)
    # lAIR: (R A)[row, rows of the strong F blocks] = 0
    RA = (R @ A).tocsr()
    Cb = np.nonzero(cfb == 1)[0]
    for I in Cb[:200]:
        lo, hi = W.indptr[I], W.indptr[I + 1]
        N = W.indices[lo:hi][sb[lo:hi] & (cfb[W.indices[lo:hi]] == 0)]
        if len(N) == 0:
            continue
        rN = (N[:, None] * b + np.arange(b)).ravel()
        for m in range(b):
            r = cidx[I * b + m]
            row = RA[r].toarray().ravel()
            assert np.abs(row[rN]).max() <= 1e-12 * np.abs(A[I * b + m].toarray()).max()
            assert R[r, I * b + m] == 1.0


def test_block_air_hierarchy_solves(slab_sys):
    H = air.setup(slab_sys.Shat, max_coarse=50, block_air=True, block=slab_sys.b)
    assert H.nlev >= 3
    x, info = krylov.fgmres(slab_sys.Shat, slab_sys.Hhat, lambda r: air.vcycle(H, r), tol=1e-10)
    assert info["converged"] and info["iters"] < 40
    ref = direct_solve(slab_sys)
    assert np.linalg.norm(x - ref) <= 1e-8 * np.linalg.norm(ref)
    # the transposed cycle is still the adjoint of the cycle
    rng = np.random.default_rng(23)
    u, v = rng.standard_normal(slab_sys.n), rng.standard_normal(slab_sys.n)
    lhs, rhs = air.vcycle(H, u) @ v, u @ air.vcycle_T(H, v)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
