"""Structured space-time simplex meshes (inputs only).

Every generator returns ``(vert, cell)``: ``vert`` is float64 ``[nv][D]`` with
column 0 the time coordinate, ``cell`` is int32 ``[ne][D+1]``.  The cell
vertex order is part of the input (it fixes each element's reference map).

The splits avoid facets on which the space-time advection vanishes
identically (a singular facet block at zero diffusion): see the notes on
each generator.  Meshes of the paper's own experiments (unstructured and
adaptive space-time meshes, Sections 4.1-4.2) are not available; these
structured meshes stand in for them with the same element counts.
"""
import numpy as np


def square_tri_mesh(n, t0=0.0, t1=1.0, x0=0.0, x1=1.0):
    """(1+1)-D space-time square split into ``n*n`` quads, two triangles each.

    Vertex ``(t_j, x_i)`` has id ``j*(n+1)+i``.  Each quad is split along the
    diagonal joining ``(t_j, x_{i+1})`` and ``(t_{j+1}, x_i)``; the other
    diagonal is parallel to the space-time velocity (1, 1) of unit
    advection and would be a characteristic facet.
    """
    t = np.linspace(t0, t1, n + 1)
    x = np.linspace(x0, x1, n + 1)
    T, X = np.meshgrid(t, x, indexing="ij")
    vert = np.stack([T.ravel(), X.ravel()], axis=1).astype(np.float64)
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    j = j.ravel(); i = i.ravel()
    v00 = j * (n + 1) + i
    v01 = j * (n + 1) + i + 1          # (t_j, x_{i+1})
    v10 = (j + 1) * (n + 1) + i        # (t_{j+1}, x_i)
    v11 = (j + 1) * (n + 1) + i + 1
    tri_a = np.stack([v00, v01, v10], axis=1)
    tri_b = np.stack([v01, v11, v10], axis=1)
    cell = np.stack([tri_a, tri_b], axis=1).reshape(-1, 3)
    return vert, cell.astype(np.int32)


def _unit_square_triangles(n, lo=0.0, hi=1.0):
    """Spatial n*n grid on [lo,hi]^2 split along the (i,j)-(i+1,j+1) diagonal."""
    s = np.linspace(lo, hi, n + 1)
    X2, X1 = np.meshgrid(s, s, indexing="ij")     # vertex (x1_i, x2_j) id j*(n+1)+i
    xy = np.stack([X1.ravel(), X2.ravel()], axis=1)
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    j = j.ravel(); i = i.ravel()
    p00 = j * (n + 1) + i
    p10 = j * (n + 1) + i + 1
    p01 = (j + 1) * (n + 1) + i
    p11 = (j + 1) * (n + 1) + i + 1
    t1 = np.stack([p00, p10, p11], axis=1)
    t2 = np.stack([p00, p11, p01], axis=1)
    tri = np.stack([t1, t2], axis=1).reshape(-1, 3)
    return xy, tri


def _extrude_prisms(xy, tri, tb, tt):
    """Extrude a spatial triangulation into one slab of prisms, 3 tets each.

    Bottom vertices keep their spatial ids, top vertices are offset by the
    spatial vertex count.  A prism over the bottom triangle ``a<b<c`` is cut
    into ``(a,b,c,c')``, ``(a,b,b',c')``, ``(a,a',b',c')``: every quad side is
    then cut along the diagonal from its lower-id bottom vertex to its
    higher-id top vertex, so neighbouring prisms agree.
    """
    nv2 = xy.shape[0]
    vert = np.concatenate([
        np.concatenate([np.full((nv2, 1), tb), xy], axis=1),
        np.concatenate([np.full((nv2, 1), tt), xy], axis=1)], axis=0)
    s = np.sort(tri, axis=1)
    a, b, c = s[:, 0], s[:, 1], s[:, 2]
    ap, bp, cp = a + nv2, b + nv2, c + nv2
    tets = np.stack([np.stack([a, b, c, cp], 1),
                     np.stack([a, b, bp, cp], 1),
                     np.stack([a, ap, bp, cp], 1)], axis=1).reshape(-1, 4)
    return vert.astype(np.float64), tets.astype(np.int32)


def slab_prism_tet_mesh(n, dt, t0=0.0):
    """One space-time slab ``[t0, t0+dt] x [0,1]^2``: ``n*n`` quads -> ``2n^2``
    triangles -> prisms -> ``6 n^2`` tets (the slab-by-slab mesh family of
    Section 4.1, Table 1: 384 tets per slab at n=8 ... 24,576 at n=64)."""
    xy, tri = _unit_square_triangles(n)
    return _extrude_prisms(xy, tri, t0, t0 + dt)


def stacked_prism_tet_mesh(n, nt, T=1.0):
    """All-at-once mesh of ``nt`` stacked slabs over ``[0,T] x [0,1]^2``: layer
    ``k`` is ``slab_prism_tet_mesh(n, T/nt, k T/nt)`` with its vertices
    renumbered ``k * nv2 + spatial id``, so elements ``[6 n^2 k, 6 n^2 (k+1))``
    are the tets of slab ``k`` in the same order and orientation."""
    xy, tri = _unit_square_triangles(n)
    nv2 = xy.shape[0]
    ts = np.linspace(0.0, T, nt + 1)
    vert = np.concatenate([np.concatenate([np.full((nv2, 1), t), xy], axis=1) for t in ts], axis=0)
    s = np.sort(tri, axis=1)
    cells = []
    for k in range(nt):
        a, b, c = s[:, 0] + k * nv2, s[:, 1] + k * nv2, s[:, 2] + k * nv2
        ap, bp, cp = a + nv2, b + nv2, c + nv2
        cells.append(np.stack([np.stack([a, b, c, cp], 1),
                               np.stack([a, b, bp, cp], 1),
                               np.stack([a, ap, bp, cp], 1)], axis=1).reshape(-1, 4))
    return vert.astype(np.float64), np.concatenate(cells, axis=0).astype(np.int32)


def kuhn_cube_mesh(n, reflect_x1=True, t_extent=1.0):
    """All-at-once space-time cube ``[0,T] x [0,1]^2``: ``n^3`` cubes, 6 tets each.

    Vertex ``(t_k, x1_j, x2_i)`` has id ``(k*(n+1)+j)*(n+1)+i``.  Each cube is
    split into the tets ``{y_s1 <= y_s2 <= y_s3}`` over the six orderings of its
    local coordinates ``y``; with ``reflect_x1`` the local coordinates are
    ``(t, 1-x1, x2)``, which keeps the diagonal planes of the split off the
    characteristics of velocities with equal t and x1 components.
    """
    n1 = n + 1
    g = np.linspace(0.0, 1.0, n1)
    K, J, I = np.meshgrid(g * t_extent, g, g, indexing="ij")
    vert = np.stack([K.ravel(), J.ravel(), I.ravel()], axis=1).astype(np.float64)
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    k = k.ravel(); j = j.ravel(); i = i.ravel()

    def vid(dk, dj, di):
        return ((k + dk) * n1 + (j + dj)) * n1 + (i + di)

    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    tets = []
    for s in perms:
        # region y_{s[0]} <= y_{s[1]} <= y_{s[2]}: path 0 -> e_{s2} -> e_{s2}+e_{s1} -> 1
        y = [np.zeros(3, dtype=int)]
        cur = np.zeros(3, dtype=int)
        for ax in (s[2], s[1], s[0]):
            cur = cur.copy(); cur[ax] = 1
            y.append(cur)
        vs = []
        for yy in y:
            dk, dj, di = int(yy[0]), int(yy[1]), int(yy[2])
            if reflect_x1:
                dj = 1 - dj
            vs.append(vid(dk, dj, di))
        tets.append(np.stack(vs, axis=1))
    cell = np.stack(tets, axis=1).reshape(-1, 4)
    return vert, cell.astype(np.int32)


def map_vertices_c5(vert, amp=0.1):
    """Time-dependent domain map ``x <- x + amp sin(pi t) sin(pi x1) sin(pi x2)``
    applied to both spatial components (straight-sided tets after mapping)."""
    v = vert.copy()
    t, x1, x2 = vert[:, 0], vert[:, 1], vert[:, 2]
    s = amp * np.sin(np.pi * t) * np.sin(np.pi * x1) * np.sin(np.pi * x2)
    v[:, 1] = x1 + s
    v[:, 2] = x2 + s
    return v


def pulse_slab_mesh(N, k, amp=0.1, T=1.0):
    """Slab ``k`` of ``N`` for the rotating pulse on a moving domain (Section 4.1).

    The uniform space-time mesh on ``[0,T] x [-1/2,1/2]^2`` (``N*N`` quads per
    slab, ``dt = T/N``) is deformed by
    ``x_i = x_i^u + amp (1/2 - x_i^u) sin(2 pi (1/2 - x_i^* + t))`` with
    ``x^* = (x_2^u, x_1^u)``.
    """
    xy, tri = _unit_square_triangles(N, -0.5, 0.5)
    dt = T / N
    vert, cell = _extrude_prisms(xy, tri, k * dt, (k + 1) * dt)
    t = vert[:, 0]
    xu1, xu2 = vert[:, 1].copy(), vert[:, 2].copy()
    vert[:, 1] = xu1 + amp * (0.5 - xu1) * np.sin(2 * np.pi * (0.5 - xu2 + t))
    vert[:, 2] = xu2 + amp * (0.5 - xu2) * np.sin(2 * np.pi * (0.5 - xu1 + t))
    return vert, cell


def boundary_kinds(vert, facet_vert, is_boundary, t_min=None, t_max=None, tol=1e-12):
    """Boundary rule of all workloads: 0 interior, 1 Dirichlet, 2 Neumann.

    Facets lying in the initial or final time plane are Neumann (inflow data
    at ``t_min``, outflow at ``t_max``); every other boundary facet is
    Dirichlet.  ``facet_vert`` is ``[nf][D]`` vertex ids, ``is_boundary`` a
    boolean mask.
    """
    t = vert[:, 0]
    if t_min is None:
        t_min = float(t.min())
    if t_max is None:
        t_max = float(t.max())
    tf = t[facet_vert]
    on_bot = np.all(np.abs(tf - t_min) <= tol, axis=1)
    on_top = np.all(np.abs(tf - t_max) <= tol, axis=1)
    kind = np.zeros(facet_vert.shape[0], dtype=np.int8)
    kind[is_boundary] = 1
    kind[is_boundary & (on_bot | on_top)] = 2
    return kind
