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

Truncation (the reading taken here; the paper only names a tolerance eps):
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


# ----------------------------------------------------------------------------- cross approximation
# Paper, Inversion of the structured matrices: the skeleton C = U V^T may come
# from either cited skeleton-detecting algorithm; besides the randomised one
# above, the adaptive cross approximation of Bebendorf (Hierarchical Matrices,
# 2008, ACA with partial pivoting). It builds C ~ S_k = sum_l a_l b_l^T from
# single rows and columns of the residual C - S_{k-1}:
#   row i_k of the residual; j_k = its largest entry outside the used columns,
#   pivot p = that entry; b_k = row / p; a_k = column j_k of the residual;
#   ||S_k||_F^2 = ||S_{k-1}||_F^2 + 2 Re sum_{l<k} (a_l^H a_k)(b_l^H b_k) + ||a_k||^2 ||b_k||^2;
#   stop once ||a_k|| ||b_k|| <= eps ||S_k||_F (or k = rank_cap);
#   i_{k+1} = the largest entry of a_k outside the used rows.
# The first row is row 0. A residual row that vanishes (largest entry 0) marks
# the row used and moves on to the lowest unused row, without a step.

def aca(A: np.ndarray, rank_cap: int, tol: float):
    """Returns (U (m x r), V (n x r), rows, cols, cross norms ||a_k|| ||b_k||) with
    A ~ U V^T. Reads A only by rows and columns."""
    m, n = A.shape
    us, vs, rows, cols, norms = [], [], [], [], []
    used_r = np.zeros(m, dtype=bool)
    used_c = np.zeros(n, dtype=bool)
    s2 = 0.0
    i = 0
    while len(us) < min(rank_cap, m, n):
        row = A[i, :].copy()
        for a, b in zip(us, vs):
            row -= a[i] * b
        used_r[i] = True
        mag = np.where(used_c, -1.0, np.abs(row))
        j = int(np.argmax(mag))
        if mag[j] <= 0.0:
            free = np.flatnonzero(~used_r)
            if free.size == 0:
                break
            i = int(free[0])
            continue
        b = row / row[j]
        a = A[:, j].copy()
        for ap, bp in zip(us, vs):
            a -= bp[j] * ap
        used_c[j] = True
        cross = 2.0 * sum((np.vdot(ap, a) * np.vdot(bp, b)).real for ap, bp in zip(us, vs))
        na, nb = np.linalg.norm(a), np.linalg.norm(b)
        s2 += cross + (na * nb) ** 2
        us.append(a)
        vs.append(b)
        rows.append(i)
        cols.append(j)
        norms.append(na * nb)
        if na * nb <= tol * np.sqrt(max(s2, 0.0)):
            break
        mag = np.where(used_r, -1.0, np.abs(a))
        i = int(np.argmax(mag))
        if used_r[i]:
            break
    if not us:
        return np.zeros((m, 0), A.dtype), np.zeros((n, 0), A.dtype), rows, cols, np.zeros(0)
    return np.stack(us, axis=1), np.stack(vs, axis=1), rows, cols, np.array(norms)
