"""Randomised low-rank compression of the filtered compact part (oracle).

Paper, Inversion of the structured matrices: the filtered compact part C is
written C = U V^T by a skeleton-detecting algorithm (the cited randomised
algorithm of Liberty et al. among them). The oracle takes the randomised
range finder with power (subspace) iterations in the form of Halko,
Martinsson & Tropp (SIAM Review 2011, randomised subspace iteration), with
Householder QR (LAPACK via SciPy):
    Y = A Omega,  Q = qr(Y)
    repeat q times:  Q' = qr(A^H Q),  Q = qr(A Q')
    B = Q^H A,  B = U~ Sigma V~^H (SVD)
and truncates to r: U = Q U~_r Sigma_r, W = V~_r^H so that A ~ U W.

Truncation (this build's reading; the paper only names a tolerance eps):
    r = min(rank_cap, #{sigma_i > max(eps, 1e-13) sigma_1}),
then r is lowered while sigma_r < (1 + 1e-6) sigma_{r+1}, so that a pair of
(numerically) equal singular values is never split.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

ZERO_RTOL = 1e-13
TIE_RTOL = 1e-6


def qr_q(Y: np.ndarray) -> np.ndarray:
    return sla.qr(Y, mode="economic")[0]


def range_finder(A: np.ndarray, Omega: np.ndarray, power_iters: int):
    Q = qr_q(A @ Omega)
    for _ in range(power_iters):
        Qp = qr_q(A.conj().T @ Q)
        Q = qr_q(A @ Qp)
    return Q


def truncation_rank(s: np.ndarray, rank_cap: int, tol: float) -> int:
    if s.size == 0 or s[0] == 0.0:
        return 0
    thr = max(tol, ZERO_RTOL) * s[0]
    r = min(rank_cap, int(np.count_nonzero(s > thr)))
    while 0 < r < s.size and s[r - 1] < (1.0 + TIE_RTOL) * s[r]:
        r -= 1
    return r


def compress(A: np.ndarray, Omega: np.ndarray, power_iters: int, rank_cap: int,
             tol: float):
    """Returns (U (N x r), W (r x N), singular values of B)."""
    Q = range_finder(A, Omega, power_iters)
    B = Q.conj().T @ A
    Ub, s, Vh = sla.svd(B, full_matrices=False)
    r = truncation_rank(s, rank_cap, tol)
    U = (Q @ Ub[:, :r]) * s[None, :r]
    W = Vh[:r]
    return U, W, s
