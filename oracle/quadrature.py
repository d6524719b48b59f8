"""Quadrature rules for the Galerkin double integrals (oracle).

The paper does not state its quadrature. The rule adopted here: every panel
pair uses the 8 x 8 tensor Gauss-Legendre rule,
except that on self and adjacent panel pairs the Laplace singular parts
  -(1/2 pi) log|x - y|          (single layer / Maue hypersingular form)
  (1/2 pi) (x - y).n_y/|x - y|^2 (double layer, adjacent pairs)
are integrated to full double precision, and only the smooth remainders use
the 8 x 8 rule.

Self pair: closed form. With xi, eta in [0,1], psi_0 = 1 - xi, psi_1 = xi,
  int int psi_a(xi) psi_b(eta) log|xi - eta| = J_ab,
  J_00 = J_11 = -7/16, J_01 = J_10 = -5/16
(from I_00 = -3/2, I_10 = -3/4 and I_11 = int int xi eta log|xi-eta| = -7/16,
the last by the substitution eta = xi - d on the half-square xi > eta), so on a
panel of length h: int_p int_p psi_a psi_b log|x-y| = h^2 (log(h)/4 + J_ab).

Adjacent pair: Duffy's split of the unit square at the shared corner into two
triangles, rho integrated in closed form (polynomial times log rho), the
remaining angle variable t by Gauss-Legendre (the integrand is analytic in t
for a non-degenerate corner).
"""
from __future__ import annotations

import functools

import numpy as np

TWO_PI = 2.0 * np.pi

SELF_LOG_J = np.array([[-7.0 / 16.0, -5.0 / 16.0],
                       [-5.0 / 16.0, -7.0 / 16.0]])


@functools.lru_cache(maxsize=None)
def gauss_legendre_01(n: int):
    """n-point Gauss-Legendre nodes and weights on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def shape_values(xi: np.ndarray) -> np.ndarray:
    """psi_alpha(xi) for alpha = 0, 1; shape (2, len(xi))."""
    return np.stack([1.0 - xi, xi])


def self_log(h: float) -> np.ndarray:
    """int_p int_p psi_a(x) psi_b(y) log|x - y| ds_x ds_y on one panel of length h."""
    return h * h * (0.25 * np.log(h) + SELF_LOG_J)


def _corner_coeffs(end_x: bool, end_y: bool):
    """Linear shape functions as c0 + c1 s, where s is the fraction of panel
    length measured from the shared node. end_x: the shared node is the end
    (xi = 1) of the x-panel; end_y likewise for the y-panel."""
    # psi_0 = 1 - xi, psi_1 = xi; at the end node xi = 1 - s, at the start xi = s
    def lin(end):
        if end:
            return np.array([[0.0, 1.0], [1.0, -1.0]])   # psi_0 = s, psi_1 = 1 - s
        return np.array([[1.0, -1.0], [0.0, 1.0]])       # psi_0 = 1 - s, psi_1 = s
    return lin(end_x), lin(end_y)


def adjacent_singular(hp: float, hq: float, a: np.ndarray, b: np.ndarray,
                      nq: np.ndarray, end_x: bool, end_y: bool, nt: int = 32):
    """Singular parts for two panels sharing one node.

    The x-panel has length hp and leaves the shared node c in direction a; the
    y-panel has length hq and leaves c in direction b; nq is the y-panel normal.
    With x = c + hp s1 a, y = c + hq s2 b:
      R^2 = hp^2 s1^2 + hq^2 s2^2 - 2 hp hq s1 s2 (a.b),
      (x - y).nq = hp s1 (a.nq)   (b is orthogonal to nq).
    Returns (Lg, Dl), both 2 x 2 over (alpha, beta):
      Lg = int int psi_a psi_b log|x - y| ds_x ds_y
      Dl = int int psi_a psi_b (1/2pi) (x - y).nq / |x - y|^2 ds_x ds_y
    """
    cx, cy = _corner_coeffs(end_x, end_y)
    t, wt = gauss_legendre_01(nt)
    ab = float(a @ b)
    anq = float(a @ nq)
    f1sq = hp * hp + hq * hq * t * t - 2.0 * hp * hq * t * ab   # s1 = rho, s2 = rho t
    f2sq = hp * hp * t * t + hq * hq - 2.0 * hp * hq * t * ab   # s2 = rho, s1 = rho t
    lf1 = 0.5 * np.log(f1sq)
    lf2 = 0.5 * np.log(f2sq)
    Lg = np.zeros((2, 2))
    Dl = np.zeros((2, 2))
    for al in range(2):
        a0, a1 = cx[al]
        for be in range(2):
            b0, b1 = cy[be]
            # triangle 1: psi_a(rho) psi_b(rho t) = sum_m c_m rho^m
            c1 = [a0 * b0 + 0 * t, a1 * b0 + a0 * b1 * t, a1 * b1 * t]
            # triangle 2: psi_a(rho t) psi_b(rho)
            c2 = [a0 * b0 + 0 * t, a1 * b0 * t + a0 * b1, a1 * b1 * t]
            # int_0^1 rho^(m+1) (log rho + log f) d rho = -1/(m+2)^2 + log f/(m+2)
            g1 = sum(c1[m] * (-1.0 / (m + 2) ** 2 + lf1 / (m + 2)) for m in range(3))
            g2 = sum(c2[m] * (-1.0 / (m + 2) ** 2 + lf2 / (m + 2)) for m in range(3))
            Lg[al, be] = hp * hq * float(wt @ (g1 + g2))
            # double layer: rho-Jacobian and 1/R^2 leave int_0^1 rho^m = 1/(m+1)
            d1 = sum(c1[m] / (m + 1) for m in range(3)) * (hp * anq / f1sq)
            d2 = sum(c2[m] / (m + 1) for m in range(3)) * (hp * anq * t / f2sq)
            Dl[al, be] = hp * hq / TWO_PI * float(wt @ (d1 + d2))
    return Lg, Dl
