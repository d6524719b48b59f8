"""Normalised Calderon TE-EFIE, TE-MFIE and TE-CFIE (oracle).

Paper, Notation and Background (discretised normalised Calderon TE-EFIE and
TE-MFIE) and Filters Based Fast Direct Solver, 2D case. Unknown y = G^{1/2} j
(the paper writes j_2 for the normalised unknown; j = G^{-1/2} y is reported).

Readings taken where the printed text is garbled or silent:
  * EFIE: Z_e = G^{-1/2} S G^{-1} N G^{-1/2} -> I/4 + compact. The printed
    (ik)^{-1} factor is dropped from Z_2 because C_2 = Z_2 - I/4 must be
    compact; the physical constants sit in the right-hand side, built from
    f = <phi, du_inc/dn>: v_e = -G^{-1/2} S G^{-1} f  (so that N j = -f).
  * MFIE: Z_h = I/2 - G^{-1/2} D G^{-1/2}, v_h = -G^{-1/2} h; its compact part
    is C_h = -G^{-1/2} D G^{-1/2} (the filtered MFIE is I/2 + P C_h).
  * CFIE: Z_e + alpha Z_h, v_e + alpha v_h, beta = (1 + 2 alpha)/4.
  * Yukawa-Calderon CFIE ("ycfie", paper, Filters Based Fast Direct Solver, 2D
    case, the filtered Yukawa-Calderon TE-CFIE): the CFIE with the single layer
    of the Calderon product and of v_e taken at the imaginary wavenumber i k
    (kernel (1/2 pi) K0(k R), the "localised" preconditioner):
    Z_e = G^{-1/2} S_y G^{-1} N G^{-1/2}, v_e = -G^{-1/2} S_y G^{-1} f; the
    compact part is again Z_e - I/4 + alpha C_h, beta = (1 + 2 alpha)/4. The
    paper names the preconditioner but not its wavenumber; i k is the reading
    taken here.
G^{+-1/2} and G^{-1} are formed from a dense symmetric eigendecomposition of
G (exact to rounding).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .assembly import periodic_dense

FORMS = ("efie", "mfie", "cfie", "ycfie")


def gram_powers(diag: np.ndarray, off: np.ndarray):
    """(G^{1/2}, G^{-1/2}, G^{-1}) as dense matrices."""
    G = periodic_dense(diag, off)
    lam, V = sla.eigh(G)
    if lam[0] <= 0.0:
        raise ValueError("Gram matrix not positive definite")
    Gh = (V * np.sqrt(lam)) @ V.T
    Gmh = (V / np.sqrt(lam)) @ V.T
    Gi = (V / lam) @ V.T
    return Gh, Gmh, Gi


def beta_of(form: str, alpha: float = 1.0) -> float:
    if form == "efie":
        return 0.25
    if form == "mfie":
        return 0.5
    if form in ("cfie", "ycfie"):
        return (1.0 + 2.0 * alpha) / 4.0
    raise ValueError(form)


def compact_part(form: str, S, Nm, D, Gmh, Gi, alpha: float = 1.0, Sy=None):
    """C = Z - beta I for the chosen formulation; returns (C, beta). Sy: the
    Yukawa single layer (required for "ycfie")."""
    n = S.shape[0]
    I = np.eye(n)
    Ce = Ch = None
    if form in ("efie", "cfie", "ycfie"):
        Sc = Sy if form == "ycfie" else S
        Ce = Gmh @ (Sc @ (Gi @ (Nm @ Gmh))) - 0.25 * I
    if form in ("mfie", "cfie", "ycfie"):
        Ch = -(Gmh @ (D @ Gmh))
    if form == "efie":
        C = Ce
    elif form == "mfie":
        C = Ch
    else:
        C = Ce + alpha * Ch
    return C, beta_of(form, alpha)


def rhs_vector(form: str, S, Gmh, Gi, f, h, alpha: float = 1.0, Sy=None):
    """v for columns f, h (N x nrhs)."""
    v = 0
    if form in ("efie", "cfie", "ycfie"):
        v = -(Gmh @ ((Sy if form == "ycfie" else S) @ (Gi @ f)))
    if form in ("mfie", "cfie", "ycfie"):
        vh = -(Gmh @ h)
        v = vh if form == "mfie" else v + alpha * vh
    return v


def system_matrix(form: str, S, Nm, D, Gmh, Gi, alpha: float = 1.0, Sy=None):
    """Z = beta I + C (unfiltered)."""
    C, beta = compact_part(form, S, Nm, D, Gmh, Gi, alpha, Sy)
    return C + beta * np.eye(S.shape[0])
