"""Quadrature on the reference simplex (oracle).

The paper does not fix a rule.  Reading used here (and by the HIP path, which
computes its own nodes): conical-product (collapsed coordinate) rules with
``n`` Gauss-Jacobi points per direction, exact for total degree ``2n-1``.

Reference simplex ``T_D = {xi >= 0, sum xi <= 1}``.  Collapsed coordinates
``s in [0,1]^D``:
  D=1: xi1 = s1
  D=2: xi1 = s1 (1-s2),             xi2 = s2,           Jacobian (1-s2)
  D=3: xi1 = s1 (1-s2)(1-s3),       xi2 = s2 (1-s3),    xi3 = s3,
       Jacobian (1-s2)(1-s3)^2
Direction k carries the Gauss-Jacobi weight ``(1-s)^(k-1)`` on [0,1].
Weights sum to ``|T_D| = 1/D!``.  Point index: s1 varies fastest.
"""
import numpy as np
from scipy.special import roots_jacobi


def gauss_jacobi_01(n, alpha):
    """n-point Gauss rule on [0,1] for the weight (1-s)^alpha (library nodes)."""
    y, w = roots_jacobi(n, alpha, 0.0)
    s = 0.5 * (1.0 + y)
    return s, w / 2.0 ** (alpha + 1)


def simplex_rule(D, n):
    """Points ``xi[nq][D]`` and weights ``w[nq]`` on the reference simplex."""
    if D == 0:
        return np.zeros((1, 0)), np.ones(1)
    rules = [gauss_jacobi_01(n, k) for k in range(D)]
    if D == 1:
        s1, w1 = rules[0]
        return s1[:, None].copy(), w1.copy()
    if D == 2:
        (s1, w1), (s2, w2) = rules
        S2, S1 = np.meshgrid(s2, s1, indexing="ij")
        W2, W1 = np.meshgrid(w2, w1, indexing="ij")
        xi = np.stack([S1 * (1 - S2), S2], axis=-1).reshape(-1, 2)
        return xi, (W1 * W2).ravel()
    if D == 3:
        (s1, w1), (s2, w2), (s3, w3) = rules
        S3, S2, S1 = np.meshgrid(s3, s2, s1, indexing="ij")
        W3, W2, W1 = np.meshgrid(w3, w2, w1, indexing="ij")
        xi = np.stack([S1 * (1 - S2) * (1 - S3), S2 * (1 - S3), S3], axis=-1).reshape(-1, 3)
        return xi, (W1 * W2 * W3).ravel()
    raise ValueError("D must be 0..3")


def bary(xi):
    """Barycentric coordinates ``(1 - sum xi, xi_1, ..., xi_D)``."""
    return np.concatenate([1.0 - xi.sum(-1, keepdims=True), xi], axis=-1)
