"""Green's function of the 2D Helmholtz equation (oracle; test infrastructure).

Paper, Notation and Background: g2(r, r') = (i/4) H0^(1)(k |r - r'|); the double
layer D uses the normal derivative with respect to the source point r'.

Bessel functions come from scipy.special (j0, y0, j1, y1, k0); the HIP library
has its own evaluator. H_n^(1) = J_n + i Y_n.

The Yukawa kernel of the Yukawa-Calderon TE-CFIE (paper, Filters Based Fast
Direct Solver, 2D case: the Calderon preconditioner localised) is g2 at the
imaginary wavenumber i kappa: (i/4) H0^(1)(i kappa R) = (1/2 pi) K0(kappa R).
"""
from __future__ import annotations

import numpy as np
from scipy import special as _sp

EULER_GAMMA = float(np.euler_gamma)
TWO_PI = 2.0 * np.pi


def hankel1_01(x):
    """(H0^(1)(x), H1^(1)(x)) for real x > 0."""
    x = np.asarray(x, dtype=np.float64)
    return _sp.j0(x) + 1j * _sp.y0(x), _sp.j1(x) + 1j * _sp.y1(x)


def green(k: float, R):
    """g(R) = (i/4) H0^(1)(kR)."""
    R = np.asarray(R, dtype=np.float64)
    return 0.25j * (_sp.j0(k * R) + 1j * _sp.y0(k * R))


def green_reg_at_zero(k: float) -> complex:
    """lim_{R->0} g(R) + log(R)/(2 pi) = i/4 - (log(k/2) + gamma_E)/(2 pi).

    From the small-argument form Y0(z) = (2/pi)(log(z/2) + gamma_E) J0(z) + O(z^2)."""
    return 0.25j - (np.log(0.5 * k) + EULER_GAMMA) / TWO_PI


def green_reg(k: float, R):
    """Regular part of g after removing the Laplace log singularity:
    g_reg(R) = g(R) + log(R)/(2 pi), continuous at R = 0."""
    R = np.asarray(R, dtype=np.float64)
    out = np.empty(R.shape, dtype=np.complex128)
    z = R == 0.0
    nz = ~z
    out[nz] = green(k, R[nz]) + np.log(R[nz]) / TWO_PI
    out[z] = green_reg_at_zero(k)
    return out


def dgreen_coef(k: float, R):
    """c(R) with  d g / d n_y (x, y) = c(R) * ((x - y) . n_y).

    grad_y g = (ik/4) H1^(1)(kR) (x - y)/R, hence c = (ik/4) H1^(1)(kR) / R."""
    R = np.asarray(R, dtype=np.float64)
    return 0.25j * k * (_sp.j1(k * R) + 1j * _sp.y1(k * R)) / R


def dgreen_laplace_coef(R):
    """Small-R limit of dgreen_coef: the Laplace double-layer 1/(2 pi R^2)."""
    R = np.asarray(R, dtype=np.float64)
    return 1.0 / (TWO_PI * R * R)


def yukawa(kappa: float, R):
    """(1/2 pi) K0(kappa R) for R > 0."""
    R = np.asarray(R, dtype=np.float64)
    return _sp.k0(kappa * R) / TWO_PI


def yukawa_reg_at_zero(kappa: float) -> float:
    """lim_{R->0} (1/2 pi)(K0(kappa R) + log R) = -(log(kappa/2) + gamma_E)/(2 pi),
    from K0(z) = -(log(z/2) + gamma_E) I0(z) + O(z^2 log z)."""
    return -(np.log(0.5 * kappa) + EULER_GAMMA) / TWO_PI


def yukawa_reg(kappa: float, R):
    """Regular part (1/2 pi)(K0(kappa R) + log R), continuous at R = 0."""
    R = np.asarray(R, dtype=np.float64)
    out = np.empty(R.shape, dtype=np.float64)
    z = R == 0.0
    nz = ~z
    out[nz] = yukawa(kappa, R[nz]) + np.log(R[nz]) / TWO_PI
    out[z] = yukawa_reg_at_zero(kappa)
    return out
