"""lAIR algebraic multigrid (oracle).

Passages followed: two-grid correction ``x <- x + P (R A P)^-1 R r`` and the
C/F block form, ideal restriction ``R_ideal = [-A_cf A_ff^-1, I]`` with any
``P = [W; I]`` (Section 3); the solver settings of Section 4: distance-one
restriction neighbourhoods from a strength tolerance, one-point
interpolation, no pre-relaxation, post-relaxation on F points then all
points, AIR applied to the matrix scaled by the inverse facet blocks.

Readings where the paper is silent or where this build deviates (listed in
the design notes):
  * strength: ``j in S_i`` iff ``j != i`` and
    ``|a_ij| >= theta max_{k != i} |a_ik| (1 - 1e-12)``; a row whose
    off-diagonal entries are all zero has no strong connections;
  * coarsening: PMIS on the symmetrised strength graph, point weights compared
    as the integer key ``influence_count * 2^44 + hash44(i, level)`` (a
    bijective 44-bit mix, so keys never tie); points nothing depends on
    strongly start as F; coarse index = rank of the C point; or, as an
    option, the sequential Ruge-Stueben first pass (largest measure first,
    ties to the smallest index), the single-process form of the Falgout
    coarsening the paper uses;
  * lAIR restriction row of C point i: ``N_i`` = strong F neighbours (sorted)
    for distance one; for distance two also the strong F neighbours of those
    (paths through F points only); the strength tolerance of R may differ
    from that of the coarsening (Section 4 uses 0.3 and 0.2);
    ``A[N_i,N_i]^T z = -A[i,N_i]^T`` by LU with partial pivoting,
    ``R[i,i] = 1``, ``R[i,N_i] = z``; injection when ``N_i`` is empty or a pivot
    satisfies ``|pivot| <= 1e-14 max |A[N_i,N_i]|``;
  * one-point interpolation: an F point takes weight 1 at its strongest
    strong C neighbour (ties within relative 1e-12 -> smallest index), or
    a zero row when it has none;
  * relaxation: Jacobi (omega = 1) sweeps on F, F, C ("FFC") or one F sweep
    ("F") instead of Gauss-Seidel; or, on level 0 only, forward Gauss-Seidel
    over the levels of the flow order of Lemma 3.1 (Section 3.3), Jacobi
    inside a level: over all points ("ordered", the exact solve of the
    advective part) or on F points then on all points ("ordered_fa", the
    schedule of Section 4); a pair of facet blocks is ordered only when one
    coupling exceeds ``order_ratio`` (1.5) times the other; coarser levels
    keep F, F, C Jacobi; no filtering of R, P or R A P;
  * hierarchy stops when the coarse grid has at most ``max_coarse`` points,
    when ``max_levels`` is reached, or when coarsening stalls
    (``n_c == 0`` or ``n_c > 0.9 n``); coarsest level: dense LU.
"""
import numpy as np
import scipy.sparse as sp
import scipy.linalg as sla

MASK44 = (1 << 44) - 1


def hash44(i, level):
    """Bijective 44-bit mix of the point index (per level)."""
    m = np.uint64(MASK44)
    with np.errstate(over="ignore"):          # products are taken mod 2^64, then mod 2^44
        x = (np.asarray(i, dtype=np.uint64) + np.uint64((level + 1) * 0x9E3779B97F4A7C15 & MASK44)) & m
        x = x ^ (x >> np.uint64(21))
        x = (x * np.uint64(0xBF58476D1CE4E5B9 & MASK44)) & m
        x = x ^ (x >> np.uint64(19))
        x = (x * np.uint64(0x94D049BB133111EB & MASK44)) & m
        x = x ^ (x >> np.uint64(22))
    return x


def _rows(A):
    return np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))


def strength(A, theta):
    """Boolean mask over the stored entries of CSR ``A``: strong connections."""
    n = A.shape[0]
    r = _rows(A)
    absv = np.abs(A.data)
    off = A.indices != r
    offabs = np.where(off, absv, 0.0)
    rmax = np.zeros(n)
    np.maximum.at(rmax, r, offabs)
    return off & (rmax[r] > 0) & (absv >= theta * rmax[r] * (1.0 - 1e-12))


def pmis(A, strong, level):
    """PMIS C/F splitting: returns ``cf`` with 1 = C, 0 = F."""
    n = A.shape[0]
    r = _rows(A)
    si, sj = r[strong], A.indices[strong]           # i depends strongly on j
    lam = np.bincount(sj, minlength=n)              # how many points depend on j
    key = (lam.astype(np.uint64) << np.uint64(44)) | hash44(np.arange(n), level)
    state = np.zeros(n, dtype=np.int8)               # 0 undecided, 1 C, -1 F
    state[lam == 0] = -1
    # symmetrised graph edges (both directions)
    gi = np.concatenate([si, sj])
    gj = np.concatenate([sj, si])
    while np.any(state == 0):
        und = state == 0
        e = und[gi] & und[gj]
        nbmax = np.zeros(n, dtype=np.uint64)
        np.maximum.at(nbmax, gi[e], key[gj[e]])
        newc = und & (key > nbmax)
        state[newc] = 1
        isc = state == 1
        dep = np.zeros(n, dtype=bool)
        hit = isc[sj] & (state[si] == 0)
        dep[si[hit]] = True
        state[dep & (state == 0)] = -1
    return (state == 1).astype(np.int8)


def rs_first_pass(A, strong):
    """Ruge-Stueben first-pass coarsening (the single-process form of the
    Falgout coarsening of Section 4): returns ``cf`` with 1 = C, 0 = F.

    With ``S_i`` the strong dependencies of i and ``S_i^T`` the points that
    depend strongly on i, the measure of an undecided point is the number of
    undecided points of ``S_i^T``.  Points with measure 0 at the start (nothing
    depends on them) are F.  Then, while points are undecided: the undecided
    point of largest measure (ties: smallest index) becomes C; the undecided
    points of ``S_i^T`` become F, and each undecided point that a new F point
    depends on gains one in measure; each undecided point of ``S_i`` loses
    one, and an undecided point whose measure reaches 0 becomes F."""
    import heapq
    n = A.shape[0]
    r = _rows(A)
    si, sj = r[strong], A.indices[strong]            # i depends strongly on j
    S = [[] for _ in range(n)]
    ST = [[] for _ in range(n)]
    for a, b in zip(si.tolist(), sj.tolist()):
        S[a].append(b)
        ST[b].append(a)
    lam = [len(ST[i]) for i in range(n)]
    state = [0] * n                                  # 0 undecided, 1 C, -1 F
    heap = []
    for i in range(n):
        if lam[i] == 0:
            state[i] = -1
        else:
            heap.append((-lam[i], i))
    heapq.heapify(heap)
    while heap:
        m, i = heapq.heappop(heap)
        if state[i] != 0 or -m != lam[i]:
            continue                                 # stale entry
        state[i] = 1
        for j in ST[i]:
            if state[j] == 0:
                state[j] = -1
                for k in S[j]:
                    if state[k] == 0:
                        lam[k] += 1
                        heapq.heappush(heap, (-lam[k], k))
        for k in S[i]:
            if state[k] == 0:
                lam[k] -= 1
                if lam[k] == 0:
                    state[k] = -1
                else:
                    heapq.heappush(heap, (-lam[k], k))
    return (np.array(state) == 1).astype(np.int8)


def one_point_P(A, strong, cf, cidx):
    n = A.shape[0]
    nc = int(cf.sum())
    r = _rows(A)
    absv = np.abs(A.data)
    elig = strong & (cf[A.indices] == 1) & (cf[r] == 0)
    rmax = np.zeros(n)
    np.maximum.at(rmax, r[elig], absv[elig])
    cand = elig & (absv >= rmax[r] * (1.0 - 1e-12))
    pos = np.nonzero(cand)[0]
    first = {}
    for k in pos:                       # CSR order: smallest column first within a row
        i = r[k]
        if i not in first:
            first[i] = A.indices[k]
    rows = list(np.nonzero(cf == 1)[0])
    cols = [cidx[i] for i in rows]
    for i, j in first.items():
        rows.append(i)
        cols.append(cidx[j])
    P = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, nc))
    P.sort_indices()
    return P


def batched_lu_solve(M, rhs):
    """Gaussian elimination with partial pivoting on a batch ``M[k][m][m]``,
    ``rhs[k][m]``.  Returns solutions and a flag for systems with a pivot
    ``|pivot| <= 1e-14 max |M|``."""
    M = M.copy()
    x = rhs.copy()
    k, m, _ = M.shape
    scale = np.abs(M).reshape(k, -1).max(axis=1) if m else np.zeros(k)
    bad = np.zeros(k, dtype=bool)
    ar = np.arange(k)
    for c in range(m):
        piv = c + np.argmax(np.abs(M[:, c:, c]), axis=1)
        # swap rows c and piv
        rowc = M[ar, c].copy(); M[ar, c] = M[ar, piv]; M[ar, piv] = rowc
        xc = x[ar, c].copy(); x[ar, c] = x[ar, piv]; x[ar, piv] = xc
        pv = M[:, c, c]
        bad |= np.abs(pv) <= 1e-14 * scale
        pv_safe = np.where(bad, 1.0, pv)
        f = M[:, c + 1:, c] / pv_safe[:, None]
        M[:, c + 1:, :] -= f[:, :, None] * M[:, None, c, :]
        x[:, c + 1:] -= f * x[:, c:c + 1]
    for c in range(m - 1, -1, -1):
        pv = np.where(bad, 1.0, M[:, c, c])
        x[:, c] = (x[:, c] - np.einsum("kj,kj->k", M[:, c, c + 1:], x[:, c + 1:])) / pv
    return x, bad


def lair_neighbourhoods(A, strong, cf, distance=1):
    """``N_i`` of every C point, sorted: the F points reachable from i by at
    most ``distance`` strong connections that pass through F points only
    (distance one: the strong F neighbours of i)."""
    sF = strong & (cf[A.indices] == 0)
    nb = {}
    for i in np.nonzero(cf == 1)[0]:
        lo, hi = A.indptr[i], A.indptr[i + 1]
        front = set(A.indices[lo:hi][sF[lo:hi]].tolist())
        N = set(front)
        for _ in range(distance - 1):
            nxt = set()
            for j in front:
                lj, hj = A.indptr[j], A.indptr[j + 1]
                nxt.update(A.indices[lj:hj][sF[lj:hj]].tolist())
            nxt -= N
            N |= nxt
            front = nxt
        nb[int(i)] = np.array(sorted(N), dtype=np.int64)
    return nb


def lair_R(A, strong, cf, cidx, distance=1):
    """lAIR restriction: ``(R A)[i, j] = 0`` for ``j in N_i``, with ``N_i``
    from ``lair_neighbourhoods``."""
    n = A.shape[0]
    nc = int(cf.sum())
    Cpts = np.nonzero(cf == 1)[0]
    nbh = lair_neighbourhoods(A, strong, cf, distance)
    cnt = np.zeros(n, dtype=np.int64)
    for i, N in nbh.items():
        cnt[i] = len(N)
    rows, cols, vals = [], [], []
    nfall = 0
    for m in np.unique(cnt[Cpts]):
        pts = Cpts[cnt[Cpts] == m]
        if m == 0:
            rows.append(cidx[pts]); cols.append(pts); vals.append(np.ones(len(pts)))
            nfall += len(pts)
            continue
        N = np.zeros((len(pts), m), dtype=np.int64)
        for t, i in enumerate(pts):
            N[t] = nbh[int(i)]
        rr = np.repeat(N, m, axis=1).ravel()
        cc = np.tile(N, (1, m)).ravel()
        Mloc = np.asarray(A[rr, cc]).reshape(len(pts), m, m)
        ai = np.asarray(A[np.repeat(pts, m), N.ravel()]).reshape(len(pts), m)
        z, bad = batched_lu_solve(np.transpose(Mloc, (0, 2, 1)), -ai)
        good = ~bad
        nfall += int(bad.sum())
        rows.append(cidx[pts]); cols.append(pts); vals.append(np.ones(len(pts)))
        rows.append(np.repeat(cidx[pts[good]], m)); cols.append(N[good].ravel())
        vals.append(z[good].ravel())
    R = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nc, n))
    R.sort_indices()
    return R, nfall


def block_weights(A, b):
    """Off-diagonal blocks of the level-0 matrix (facet blocks of size ``b``):
    sorted keys ``I * nb + J`` (``I != J``) of the blocks holding a stored
    entry, and ``w_IJ = max |a_ij|`` over each block."""
    C = A.tocoo()
    nb = A.shape[0] // b
    I = C.row // b
    J = C.col // b
    off = I != J
    key = I[off].astype(np.int64) * nb + J[off]
    uk, inv = np.unique(key, return_inverse=True)
    w = np.zeros(len(uk))
    np.maximum.at(w, inv, np.abs(C.data[off]))
    return uk, w


def block_graph(A, b):
    """Block graph of the level-0 matrix in facet blocks of size ``b``: CSR
    ``W`` (nb x nb) with ``W[I, J] = w_IJ = max |a_ij|`` over each off-diagonal
    block that holds a stored entry."""
    uk, w = block_weights(A, b)
    nb = A.shape[0] // b
    W = sp.csr_matrix((w, (uk // nb, uk % nb)), shape=(nb, nb))
    W.sort_indices()
    return W


def block_air_level(A, b, theta, theta_r, level):
    """Block AIR on a level with facet-block structure (the block variant of
    the Section 3 construction; facet blocks of size ``b`` are the unknowns):
    strength, PMIS and one-point interpolation on the block graph
    (``w_IJ``), the C/F splitting and P expanded to the rows of each block
    (``P = P_blocks (x) I_b``), and the lAIR rows of each C block from one
    local system over the rows of its strong F blocks,
    ``A[N, N]^T Z = -A[I, N]^T`` with ``b`` right-hand sides, ``R[I, I] = I_b``.
    Returns ``cf, P, R, n_fallback`` (scalar)."""
    W = block_graph(A, b)
    sb = strength(W, theta)
    cfb = pmis(W, sb, level)
    cidxb = np.cumsum(cfb) - 1
    Pb = one_point_P(W, sb, cfb, cidxb)
    P = sp.kron(Pb, sp.identity(b, format="csr")).tocsr()
    P.eliminate_zeros()                               # kron keeps the zeros of the identity blocks
    P.sort_indices()
    cf = np.repeat(cfb, b).astype(np.int8)
    cidx = np.cumsum(cf) - 1
    nc = int(cf.sum())
    sbr = sb if theta_r is None or theta_r == theta else strength(W, theta_r)
    nbh = {}
    for I in np.nonzero(cfb == 1)[0]:
        lo, hi = W.indptr[I], W.indptr[I + 1]
        J = W.indices[lo:hi][sbr[lo:hi] & (cfb[W.indices[lo:hi]] == 0)]
        nbh[int(I)] = np.sort(J)
    rows, cols, vals = [], [], []
    nfall = 0
    Cb = np.nonzero(cfb == 1)[0]
    cnt = np.array([len(nbh[int(I)]) for I in Cb], dtype=np.int64)
    for m in np.unique(cnt):
        blocks = Cb[cnt == m]
        own = (blocks[:, None] * b + np.arange(b)).ravel()          # the C rows
        if m == 0:
            rows.append(cidx[own]); cols.append(own); vals.append(np.ones(len(own)))
            nfall += len(own)
            continue
        N = np.stack([nbh[int(I)] for I in blocks])                  # [k][m] blocks
        rN = (N[:, :, None] * b + np.arange(b)).reshape(len(blocks), m * b)   # sorted rows
        q = m * b
        Mloc = np.asarray(A[np.repeat(rN, q, axis=1).ravel(), np.tile(rN, (1, q)).ravel()]).reshape(len(blocks), q, q)
        MT = np.transpose(Mloc, (0, 2, 1))
        for r in range(b):
            ci = blocks * b + r
            ai = np.asarray(A[np.repeat(ci, q), rN.ravel()]).reshape(len(blocks), q)
            z, bad = batched_lu_solve(MT, -ai)
            good = ~bad
            nfall += int(bad.sum())
            rows.append(cidx[ci]); cols.append(ci); vals.append(np.ones(len(ci)))
            rows.append(np.repeat(cidx[ci[good]], q)); cols.append(rN[good].ravel())
            vals.append(z[good].ravel())
    R = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nc, A.shape[0]))
    R.sort_indices()
    return cf, P, R, nfall


def flow_levels(A, b, ratio=1.5):
    """Flow order of the facet blocks (Lemma 3.1, Section 3.3).

    A coupled pair of blocks ``I != J`` is oriented along its dominant
    coupling when that dominance is clear: ``J`` precedes ``I`` when
    ``w_IJ > ratio * w_JI``.  For pure advection on an acyclic element graph
    the upwind flux couples each pair one way only (``w_JI = 0``), so every
    coupled pair is oriented and this is the upwind order of the lemma;
    pairs whose two couplings are within the ratio (diffusion-dominated
    facets) stay unordered.  Levels by Kahn rounds over the oriented pairs:
    round k takes every block whose predecessors are all placed; when
    blocks remain but none is ready (a cycle), the remaining block with the
    fewest unplaced predecessors (then the smallest index) forms the round
    alone.  Returns ``(level[nb], rounds, cycle_breaks)``."""
    nb = A.shape[0] // b
    uk, w = block_weights(A, b)
    I, J = uk // nb, uk % nb
    if len(uk):
        rk = J * nb + I
        pos = np.minimum(np.searchsorted(uk, rk), len(uk) - 1)
        w_rev = np.where(uk[pos] == rk, w[pos], 0.0)
    else:
        w_rev = w
    pred = w > ratio * w_rev
    # successor lists: edge J -> I for every predecessor J of I
    succ = sp.csr_matrix((np.ones(int(pred.sum())), (J[pred], I[pred])), shape=(nb, nb))
    indeg = np.bincount(I[pred], minlength=nb).astype(np.int64)
    level = np.full(nb, -1, dtype=np.int64)
    done = np.zeros(nb, dtype=bool)
    frontier = np.nonzero(indeg == 0)[0]
    k = 0
    breaks = 0
    placed = 0
    while placed < nb:
        if len(frontier) == 0:
            cand = np.nonzero(~done)[0]
            frontier = cand[[int(np.argmin(indeg[cand]))]]
            breaks += 1
        level[frontier] = k
        done[frontier] = True
        placed += len(frontier)
        dec = np.asarray(succ[frontier].sum(axis=0)).ravel().astype(np.int64)
        indeg -= dec
        frontier = np.nonzero((dec > 0) & (indeg == 0) & ~done)[0]
        k += 1
    return level, k, breaks


class OrderedSweep:
    """Forward Gauss-Seidel over the levels of the flow order on the rows
    ``X``, Jacobi inside a level: the splitting matrix ``M`` holds the
    diagonal and every entry ``(i, j)``, ``i, j in X``, whose block ``J``
    lies on an earlier level than block ``I``.  One sweep is
    ``x_X <- x_X + M^-1 (b - A x)_X``; the transposed sweep is
    ``y_X <- y_X + M^-T (g - A^T y)_X``.  When no two blocks of a level are
    coupled this is the sequential Gauss-Seidel sweep in level order."""

    def __init__(self, A, b, blev, X):
        self.X = X
        rl = blev[X // b]
        order = np.lexsort((X, rl))
        self.perm = order                      # position in X of the k-th row of the order
        AX = A[X][:, X].tocoo()
        li = rl[AX.row]
        lj = rl[AX.col]
        if np.any((AX.row != AX.col) & (X[AX.row] // b == X[AX.col] // b) & (AX.data != 0)):
            raise ValueError("ordered relaxation needs identity diagonal blocks (the scaled system)")
        keep = (AX.row == AX.col) | (lj < li)
        inv = np.empty_like(order)
        inv[order] = np.arange(len(order))
        M = sp.csr_matrix((AX.data[keep], (inv[AX.row[keep]], inv[AX.col[keep]])), shape=(len(X), len(X)))
        M.sort_indices()
        self.M = M
        self.MT = M.T.tocsr()

    def _solve(self, r, transpose):
        from scipy.sparse.linalg import spsolve_triangular
        if len(r) == 0:
            return r
        rp = r[self.perm]
        y = spsolve_triangular(self.MT if transpose else self.M, rp, lower=not transpose)
        out = np.empty_like(y)
        out[self.perm] = y
        return out

    def apply(self, A, b, x):
        r = b - A @ x
        x = x.copy()
        x[self.X] += self._solve(r[self.X], False)
        return x

    def apply_T(self, AT, g, y):
        r = g - AT @ y
        y = y.copy()
        y[self.X] += self._solve(r[self.X], True)
        return y


class Level:
    pass


class Hierarchy:
    pass


def setup(A0, theta=0.25, max_coarse=64, max_levels=25, relax="FFC", omega=1.0,
          stall=0.9, max_dense=8192, theta_r=None, distance=1, block=1, order_ratio=1.5, coarsening="pmis",
          block_air=False):
    """Build the lAIR hierarchy on the scaled matrix (treated as scalar).
    ``theta`` is the strength tolerance of the coarsening (and of P);
    ``theta_r`` that of the restriction neighbourhoods (default: theta);
    ``distance`` the neighbourhood distance of lAIR (1 or 2); ``relax`` one
    of "FFC", "F", "ordered", "ordered_fa"; ``block`` the facet block size
    of level 0 (the unit of the flow order); ``order_ratio`` the dominance
    ratio that orients a pair of blocks in the flow order; ``coarsening``
    "pmis" or "rs" (Ruge-Stueben first pass); ``block_air``: level 0 is
    coarsened by block AIR on its facet blocks of size ``block``
    (``block_air_level``, distance one), the coarser levels by scalar AIR."""
    if relax not in ("FFC", "F", "ordered", "ordered_fa"):
        raise ValueError("unknown relaxation %r" % (relax,))
    if coarsening not in ("pmis", "rs"):
        raise ValueError("unknown coarsening %r" % (coarsening,))
    H = Hierarchy()
    H.levels = []
    H.relax, H.omega = relax, omega
    H.n_fallback = 0
    A = sp.csr_matrix(A0)
    A.sort_indices()
    l = 0
    while True:
        n = A.shape[0]
        lev = Level()
        lev.A = A
        lev.diag = A.diagonal()
        H.levels.append(lev)
        if n <= max_coarse or l == max_levels - 1:
            break
        if l == 0 and block_air:
            if block < 2 or distance != 1 or coarsening != "pmis":
                raise ValueError("block AIR needs facet blocks, distance one and PMIS")
            cf, Pb, Rb, nf = block_air_level(A, block, theta, theta_r, l)
            nc = int(cf.sum())
            if nc == 0 or nc > stall * n:
                break
            lev.cf, lev.P, lev.R = cf, Pb, Rb
            H.n_fallback += nf
        else:
            strong = strength(A, theta)
            cf = pmis(A, strong, l) if coarsening == "pmis" else rs_first_pass(A, strong)
            nc = int(cf.sum())
            if nc == 0 or nc > stall * n:
                break
            cidx = np.cumsum(cf) - 1
            lev.cf = cf
            lev.strong = strong
            lev.P = one_point_P(A, strong, cf, cidx)
            strong_r = strong if theta_r is None or theta_r == theta else strength(A, theta_r)
            lev.R, nf = lair_R(A, strong_r, cf, cidx, distance)
            H.n_fallback += nf
        if l == 0 and relax in ("ordered", "ordered_fa"):
            lev.blev, lev.rounds, lev.breaks = flow_levels(A, block, order_ratio)
            lev.gs_all = OrderedSweep(A, block, lev.blev, np.arange(n))
            lev.gs_F = OrderedSweep(A, block, lev.blev, np.nonzero(cf == 0)[0])
        Ac = (lev.R @ A @ lev.P).tocsr()
        Ac.sort_indices()
        A = Ac
        l += 1
    last = H.levels[-1]
    if last.A.shape[0] > max_dense:
        raise RuntimeError("coarsest level too large for a dense solve")
    last.lu = sla.lu_factor(last.A.toarray()) if last.A.shape[0] else None
    H.nlev = len(H.levels)
    return H


def _sweep_sets(H, lev, transpose):
    F = np.nonzero(lev.cf == 0)[0]
    C = np.nonzero(lev.cf == 1)[0]
    sets = [F] if H.relax == "F" else [F, F, C]
    return sets[::-1] if transpose else sets


def _ordered_sweeps(H, lev, transpose):
    """Level-0 sweeps of the ordered relaxations, in application order."""
    sw = [lev.gs_F, lev.gs_all] if H.relax == "ordered_fa" else [lev.gs_all]
    return sw[::-1] if transpose else sw


def _coarse_solve(last, b, trans=0):
    """Coarsest level: dense LU in FP64 whatever the cycle's precision (the
    input is widened to FP64 and the result rounded back to its type)."""
    if last.lu is None:
        return np.zeros(0, dtype=b.dtype)
    return sla.lu_solve(last.lu, b.astype(np.float64), trans=trans).astype(b.dtype)


def _level_ops(lev, dtype):
    """``A``, ``R``, ``P``, diagonal and ``A^T`` of a level with their values
    rounded to ``dtype`` (FP64: the level's own matrices)."""
    cache = lev.__dict__.setdefault("_ops", {})
    key = np.dtype(dtype).name
    if key not in cache:
        A = lev.A.astype(dtype)
        R = lev.R.astype(dtype) if hasattr(lev, "R") else None
        P = lev.P.astype(dtype) if hasattr(lev, "P") else None
        cache[key] = (A, R, P, lev.diag.astype(dtype), A.T.tocsr())
    return cache[key]


def vcycle(H, b, l=0, dtype=np.float64):
    """One V-cycle with zero initial guess (Section 3 coarse-grid correction,
    post-relaxation only).  ``dtype=np.float32`` runs the cycle with every
    operator rounded to FP32 and FP32 arithmetic throughout (products
    accumulate in FP32), except the FP64 coarsest solve: the reduced-precision
    cycle of the precision form (F, F, C or F sweeps only)."""
    lev = H.levels[l]
    b = np.asarray(b).astype(dtype, copy=False)
    if l == H.nlev - 1:
        return _coarse_solve(lev, b)
    A, R, P, d, _ = _level_ops(lev, dtype)
    ec = vcycle(H, R @ b, l + 1, dtype)
    x = P @ ec
    if hasattr(lev, "gs_all"):
        if np.dtype(dtype) != np.float64:
            raise NotImplementedError("ordered sweeps are emulated in FP64 only")
        for sw in _ordered_sweeps(H, lev, False):
            x = sw.apply(lev.A, b, x)
        return x
    om = np.asarray(H.omega, dtype=dtype)
    for X in _sweep_sets(H, lev, False):
        X = X[np.abs(lev.diag[X]) >= 1e-30]
        r = b - A @ x
        x[X] += om * r[X] / d[X]
    return x


def vcycle_T(H, g, l=0, dtype=np.float64):
    """Transpose of :func:`vcycle`: sweeps C, F, F with ``A^T``, then restriction
    by ``P^T`` and interpolation by ``R^T``; coarsest ``LU^T`` solve.
    ``dtype`` as in :func:`vcycle`."""
    lev = H.levels[l]
    g = np.asarray(g).astype(dtype, copy=False)
    if l == H.nlev - 1:
        return _coarse_solve(lev, g, trans=1)
    A, R, P, d, AT = _level_ops(lev, dtype)
    y = np.zeros_like(g)
    if hasattr(lev, "gs_all"):
        if np.dtype(dtype) != np.float64:
            raise NotImplementedError("ordered sweeps are emulated in FP64 only")
        for sw in _ordered_sweeps(H, lev, True):
            y = sw.apply_T(AT, g, y)
    else:
        om = np.asarray(H.omega, dtype=dtype)
        for X in _sweep_sets(H, lev, True):
            X = X[np.abs(lev.diag[X]) >= 1e-30]
            r = g - AT @ y
            y[X] += om * r[X] / d[X]
    y = y + R.T @ vcycle_T(H, P.T @ (g - AT @ y), l + 1, dtype)
    return y


def stats(H):
    """Level sizes, nonzeros and operator complexity."""
    ns = [lev.A.shape[0] for lev in H.levels]
    nnz = [lev.A.nnz for lev in H.levels]
    return {"n": ns, "nnz": nnz, "op_complexity": sum(nnz) / nnz[0]}
