"""Laplacian filter P^L_n (oracle).

Paper, Laplacian Filters, 2D case (filtered Laplacian and eq. LapFilter):
P^L_n = L_n^+ L_n = V S_{L,n}^+ S_{L,n} V^T, where S_{L,n} keeps the n singular
values with index i > N - n in descending order, i.e. the n smallest. For
non-homogeneous meshes L is replaced by the orthonormalised Laplacian
L~ = G^{-1/2} L G^{-1/2}.

Readings of points the paper leaves open:
  * keep_nullspace=True (default): P projects onto the eigenvectors of the n
    smallest eigenvalues of L~ *including* the constant (null) mode. The
    literal S^+ S would drop that mode (keep_nullspace=False gives it: modes
    1..n-1); the constant mode then disappears from P C altogether, which
    is an O(1) error at low frequency, where it dominates the solution.
  * cluster guard: if the cut falls inside a cluster of eigenvalues
    (relative gap <= cluster_rtol) n grows until it closes the cluster.
The eigenvectors come from a dense symmetric eigensolver (no FFT, which is
exact only for equal-length panels).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .assembly import gram, laplacian, periodic_dense
from .formulation import gram_powers
from .geometry import Mesh


def orthonormal_laplacian(m: Mesh, Gmh=None):
    Ld, Lo = laplacian(m)
    if Gmh is None:
        _, Gmh, _ = gram_powers(*gram(m))
    Lt = Gmh @ periodic_dense(Ld, Lo) @ Gmh
    return 0.5 * (Lt + Lt.T)


def choose_cut(lam: np.ndarray, start: int, n_modes: int, cluster_rtol: float) -> int:
    """Number of kept modes after the cluster guard."""
    n = n_modes
    total = lam.shape[0] - start
    while n < total:
        lo, hi = lam[start + n - 1], lam[start + n]
        if hi - lo > cluster_rtol * max(abs(lo), abs(hi)):
            break
        n += 1
    return n


def laplacian_filter(m: Mesh, n_modes: int, keep_nullspace: bool = True,
                     cluster_rtol: float = 1e-6, Gmh=None):
    """Returns (V_n (N x n_eff, orthonormal columns), eigenvalues, n_eff).

    With keep_nullspace=False the null mode is dropped (rank n_modes - 1)."""
    if not 1 <= n_modes <= m.n:
        raise ValueError("n_modes out of range")
    lam, V = sla.eigh(orthonormal_laplacian(m, Gmh))
    start = 0 if keep_nullspace else 1
    want = n_modes if keep_nullspace else n_modes - 1
    if want == 0:
        return V[:, :0], lam[:0], 0
    n = choose_cut(lam, start, want, cluster_rtol)
    return V[:, start:start + n], lam[start:start + n], n


def projector(Vn: np.ndarray) -> np.ndarray:
    return Vn @ Vn.T
