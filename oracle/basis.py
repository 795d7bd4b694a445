"""Equispaced Lagrange bases on simplices (oracle).

Nodes of degree ``p`` on a ``D``-simplex are the lattice points
``xi = (i_1, ..., i_D)/p`` with ``sum i <= p``, ordered with ``i_1`` fastest,
then ``i_2``, ...; the barycentric multi-index of a node is
``gamma = (p - sum i, i_1, ..., i_D)``.  The basis function of node ``gamma``
is the product formula

    phi_gamma(lam) = prod_k prod_{m < gamma_k} (p lam_k - m) / (m + 1),

which is 1 at its node and 0 at every other lattice node.

Facet basis (the space M_h of Section 2.3): the same construction on the
(D-1)-simplex whose vertices are the facet's global vertex ids in increasing
order.  The element basis of the oracle is the same construction on the
element's reference simplex (vertex order of the cell); the system matrix S
does not depend on the element basis.
"""
import numpy as np


def lattice(D, p):
    """Multi-indices ``i[nn][D]`` of the degree-p lattice, i_1 fastest."""
    import itertools
    if D == 0:
        return np.zeros((1, 0), dtype=int)
    res = [t for t in itertools.product(range(p + 1), repeat=D) if sum(t) <= p]
    res.sort(key=lambda t: tuple(reversed(t)))     # i_D slowest ... i_1 fastest
    return np.array(res, dtype=int)


def ndofs(D, p):
    return lattice(D, p).shape[0]


def _L(g, p, s):
    """prod_{m<g} (p s - m)/(m+1) and its derivative in s."""
    val = np.ones_like(s)
    der = np.zeros_like(s)
    for m in range(g):
        fac = (p * s - m) / (m + 1)
        der = der * fac + val * (p / (m + 1))
        val = val * fac
    return val, der


def lagrange(D, p, lam):
    """Values ``[..., nn]`` and barycentric derivatives ``[..., nn, D+1]``.

    ``lam[..., D+1]`` are barycentric coordinates (lam_0 = 1 - sum xi)."""
    idx = lattice(D, p)
    gam = np.concatenate([p - idx.sum(1, keepdims=True), idx], axis=1)   # [nn][D+1]
    nn = gam.shape[0]
    shp = lam.shape[:-1]
    vals = np.ones(shp + (nn,))
    dl = np.zeros(shp + (nn, D + 1))
    Ls = [[_L(gam[a, k], p, lam[..., k]) for k in range(D + 1)] for a in range(nn)]
    for a in range(nn):
        v = np.ones(shp)
        for k in range(D + 1):
            v = v * Ls[a][k][0]
        vals[..., a] = v
        for k in range(D + 1):
            d = Ls[a][k][1]
            for k2 in range(D + 1):
                if k2 != k:
                    d = d * Ls[a][k2][0]
            dl[..., a, k] = d
    return vals, dl


def lagrange_ref_grad(D, p, lam):
    """Values and reference gradients ``d/dxi_a = d/dlam_a - d/dlam_0``."""
    v, dl = lagrange(D, p, lam)
    g = dl[..., 1:] - dl[..., :1]
    return v, g
