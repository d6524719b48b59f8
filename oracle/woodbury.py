"""Woodbury direct inverse and iterative refinement (oracle).

Paper, Inversion of the structured matrices: each filtered equation has the
form (beta I + C) y = v with C = U V^T of rank r, and
    (beta I + U V^T)^{-1} = beta^{-1} I - beta^{-2} U (I_r + beta^{-1} V^T U)^{-1} V^T.
Here W plays the role of V^T (a plain transpose; no conjugation is involved).

Iterative refinement is not in the paper: it drives the compressed solve to
the solution of the uncompressed filtered system (beta I + P C) y = v, using
the Woodbury solve as the preconditioner and an FP64 residual.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

SINGULAR_RTOL = 64.0 * np.finfo(np.float64).eps


class SingularCore(RuntimeError):
    pass


def factor(U: np.ndarray, W: np.ndarray, beta: float):
    """LU (partial pivoting) of K = I_r + beta^{-1} W U."""
    r = U.shape[1]
    K = np.eye(r, dtype=np.complex128) + (W @ U) / beta
    if r == 0:
        return None
    lu, piv = sla.lu_factor(K)
    nk = np.abs(K).max()
    if np.abs(np.diag(lu)).min() < SINGULAR_RTOL * nk:
        raise SingularCore("Woodbury core is numerically singular")
    return lu, piv


def solve(U, W, beta: float, lu, v: np.ndarray) -> np.ndarray:
    """y = beta^{-1} v - beta^{-2} U K^{-1} (W v) for columns v."""
    y = v / beta
    if lu is not None:
        y = y - (U @ sla.lu_solve(lu, W @ v)) / (beta * beta)
    return y


def refine(apply_A, U, W, beta, lu, v, y, tol: float, max_iters: int):
    """y <- y + M^{-1}(v - A y) until max_r ||v_r - A y_r|| / ||v_r|| <= tol.

    Returns (y, residual history)."""
    vn = np.linalg.norm(v, axis=0)
    vn[vn == 0.0] = 1.0
    hist = []
    for _ in range(max_iters + 1):
        res = v - apply_A(y)
        rel = float(np.max(np.linalg.norm(res, axis=0) / vn))
        hist.append(rel)
        if rel <= tol or len(hist) > max_iters:
            break
        y = y + solve(U, W, beta, lu, res)
    return y, hist
