"""End-to-end filtered fast direct solve and its exact references (oracle).

Pipeline (paper: Filters Based Fast Direct Solver, 2D case, and Inversion of
the structured matrices):
  1. mesh, Galerkin S, N, D, Gram G, Laplacian L            (assembly)
  2. compact part C of the chosen normalised formulation   (formulation)
  3. Laplacian filter P = V_n V_n^T                          (filters)
  4. A_c = P C compressed to U W                             (compress)
  5. Woodbury factor / solve of (beta I + U W) y = v          (woodbury)
  6. FP64 refinement against beta I + P C, j = G^{-1/2} y
Exact references: y_fil = (beta I + P C)^{-1} v (dense LU) and
y_full = Z^{-1} v (unfiltered, dense LU).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

from . import assembly, compress, filters, formulation, geometry, rng, woodbury


@dataclasses.dataclass
class Problem:
    nodes: np.ndarray
    k: float
    form: str = "efie"
    alpha: float = 1.0
    n_modes: int = 21
    keep_nullspace: bool = True
    cluster_rtol: float = 1e-6
    rank_cap: int = 32
    oversample: int = 0
    power_iters: int = 0
    tol: float = 0.0
    seed: int = 0
    refine_tol: float = 1e-12
    max_refine: int = 10


@dataclasses.dataclass
class Operators:
    mesh: geometry.Mesh
    S: np.ndarray
    N: np.ndarray
    D: np.ndarray
    G: tuple
    L: tuple
    Gh: np.ndarray
    Gmh: np.ndarray
    Gi: np.ndarray
    C: np.ndarray
    beta: float
    Vn: np.ndarray
    lam: np.ndarray
    n_eff: int
    Ac: np.ndarray
    Sy: np.ndarray | None = None    # Yukawa single layer ("ycfie" only)


def build_operators(pb: Problem) -> Operators:
    m = geometry.mesh(pb.nodes)
    S, Nm, D = assembly.assemble(m, pb.k)
    G = assembly.gram(m)
    L = assembly.laplacian(m)
    Gh, Gmh, Gi = formulation.gram_powers(*G)
    Sy = assembly.assemble_yukawa(m, pb.k) if pb.form == "ycfie" else None
    C, beta = formulation.compact_part(pb.form, S, Nm, D, Gmh, Gi, pb.alpha, Sy)
    Vn, lam, n_eff = filters.laplacian_filter(m, pb.n_modes, pb.keep_nullspace,
                                              pb.cluster_rtol, Gmh)
    Ac = Vn @ (Vn.T @ C)
    return Operators(m, S, Nm, D, G, L, Gh, Gmh, Gi, C, beta, Vn, lam, n_eff, Ac, Sy)


@dataclasses.dataclass
class Solution:
    y: np.ndarray           # refined normalised unknown (N x nrhs)
    y_fast: np.ndarray      # Woodbury solve before refinement
    j: np.ndarray           # current coefficients G^{-1/2} y
    v: np.ndarray           # right-hand sides
    U: np.ndarray
    W: np.ndarray
    sigma: np.ndarray
    rank: int
    history: list


def solve(pb: Problem, ops: Operators, angles, amps) -> Solution:
    n = ops.mesh.n
    ell = pb.rank_cap + pb.oversample
    Om = rng.sketch(pb.seed, n, ell)
    U, W, s = compress.compress(ops.Ac, Om, pb.power_iters, pb.rank_cap, pb.tol)
    lu = woodbury.factor(U, W, ops.beta)
    f, h = assembly.rhs_planewave(ops.mesh, pb.k, angles, amps)
    v = formulation.rhs_vector(pb.form, ops.S, ops.Gmh, ops.Gi, f.T, h.T, pb.alpha, ops.Sy)
    y0 = woodbury.solve(U, W, ops.beta, lu, v)

    def apply_A(y):
        return ops.beta * y + ops.Ac @ y

    y, hist = woodbury.refine(apply_A, U, W, ops.beta, lu, v, y0,
                              pb.refine_tol, pb.max_refine)
    return Solution(y, y0, ops.Gmh @ y, v, U, W, s, U.shape[1], hist)


def y_filtered(ops: Operators, v: np.ndarray) -> np.ndarray:
    A = ops.beta * np.eye(ops.mesh.n) + ops.Ac
    return sla.solve(A, v)


def y_unfiltered(ops: Operators, v: np.ndarray) -> np.ndarray:
    A = ops.beta * np.eye(ops.mesh.n) + ops.C
    return sla.solve(A, v)


def relerr(y: np.ndarray, ref: np.ndarray) -> float:
    """max over right-hand sides of ||y - ref||_2 / ||ref||_2."""
    num = np.linalg.norm(y - ref, axis=0)
    den = np.linalg.norm(ref, axis=0)
    den[den == 0.0] = 1.0
    return float(np.max(num / den))
