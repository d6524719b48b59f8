#!/usr/bin/env python3
"""Writes the full-size parity fixtures tests/golden/fullsize_<case>.npz from the
CPU oracle alone (no GPU code is imported or run).

Each fixture holds, for one configuration of the benchmark sizes, what the
oracle computes in FP64 (paper: Laplacian Filters, 2D case, eq. LapFilter;
Filters Based Fast Direct Solver, 2D case; Inversion of the structured
matrices):
  n_eff, lam        kept modes after the cluster guard and their eigenvalues
                    (the pencil L v = lambda G v, i.e. the orthonormalised
                    Laplacian G^{-1/2} L G^{-1/2});
  lam_max, gap      largest eigenvalue and the gap at the cut (they scale the
                    subspace tolerance of the projector);
  X, PX             four seeded probe vectors and P X, P = V_n V_n^T;
  angles, amps      the plane waves of the stored right-hand sides;
  y_fil, j_fil      the filtered uncompressed solution y = (beta I + P C)^{-1} v
                    (dense LU) and j = G^{-1/2} y, one row per right-hand side;
and, for a truncating case, the skeleton of the same SplitMix64 sketch:
  sigma             singular values of the projected block,
  rank              the truncation rank,
  UWX               U W X for the probes X (as complex),
  y_fast            the Woodbury solve with that skeleton, before refinement.

Usage: python tests/golden/make_fullsize.py [case ...]   (default: all cases)
Runtime on 8 cores: minutes per case at N = 4096, about half an hour at N = 8192.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np
import scipy.linalg as sla

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import assembly, compress, filters, formulation, rng, solver, woodbury  # noqa: E402
from paper_2210_08580_amd import workloads as wl  # noqa: E402

PROBE_SEED = 4242

# name: (workload, N or None, form, n_modes, keep_nullspace, stored RHS, compression or None)
# compression: (rank_cap, oversample, power_iters, tol, seed)
CASES = {
    # the C2 star, both formulations, lossless skeleton
    "star4096_efie": ("star4096", None, "efie", 255, True, 8, None),
    "star4096_mfie": ("star4096", None, "mfie", 255, True, 8, None),
    # the throughput workload at full size
    "star8192_efie": ("star8192", None, "efie", 255, True, 8, None),
    # 255 kept modes with a truncating skeleton (r = 128 < n_eff): the sketched branch
    "star2048_trunc": ("star4096", 2048, "efie", 255, True, 8, (128, 10, 2, 1e-8, 7)),
    # a 5-fold symmetric mesh (N = 5 * 512) whose Laplacian pairs are exactly
    # degenerate, without the null mode: modes 1..255 of the pencil end with the
    # first of the pair of Fourier mode 128, so the cluster guard must grow the
    # cut to 256 kept modes
    "star2560_split": ("star4096", 2560, "efie", 256, False, 0, None),
}


def probes(n: int) -> np.ndarray:
    return np.random.default_rng(PROBE_SEED).standard_normal((n, 4))


def make(case: str) -> str:
    wname, n, form, nm, keep, nrhs, comp = CASES[case]
    w = wl.workload(wname, n=n, form=form)
    t0 = time.perf_counter()
    pb = solver.Problem(w.nodes, w.k, form=form, n_modes=nm, keep_nullspace=keep)
    ops = solver.build_operators(pb)
    print(f"{case}: operators {time.perf_counter() - t0:.0f} s, n_eff {ops.n_eff}", flush=True)
    lam_all = sla.eigvalsh(filters.orthonormal_laplacian(ops.mesh, ops.Gmh))
    s0 = 0 if keep else 1
    cut = s0 + ops.n_eff
    gap = lam_all[cut] - lam_all[cut - 1] if cut < lam_all.size else 0.0
    X = probes(ops.mesh.n)
    out = {"n": ops.mesh.n, "k": w.k, "form": form, "n_modes": nm, "keep_nullspace": int(keep),
           "n_eff": ops.n_eff, "lam": ops.lam, "lam_max": lam_all[-1], "gap": gap,
           "lam_next": lam_all[cut:cut + 4], "X": X, "PX": ops.Vn @ (ops.Vn.T @ X)}
    if nrhs:
        ang, amps = w.angles[:nrhs], w.amps[:nrhs]
        f, h = assembly.rhs_planewave(ops.mesh, w.k, ang, amps)
        v = formulation.rhs_vector(form, ops.S, ops.Gmh, ops.Gi, f.T, h.T)
        yf = solver.y_filtered(ops, v)
        out.update(angles=ang, amps=amps, y_fil=yf.T.copy(), j_fil=(ops.Gmh @ yf).T.copy())
        if comp is not None:
            cap, p, q, tol, seed = comp
            U, W, s = compress.compress(ops.Ac, rng.sketch(seed, ops.mesh.n, cap + p), q, cap, tol)
            lu = woodbury.factor(U, W, ops.beta)
            y0 = woodbury.solve(U, W, ops.beta, lu, v)
            out.update(rank_cap=cap, oversample=p, power_iters=q, tol=tol, seed=seed, sigma=s,
                       rank=U.shape[1], UWX=U @ (W @ X.astype(np.complex128)), y_fast=y0.T.copy(),
                       ac_max=np.abs(ops.Ac).max())
    path = os.path.join(HERE, f"fullsize_{case}.npz")
    np.savez_compressed(path, **out)
    print(f"{case}: wrote {path} ({time.perf_counter() - t0:.0f} s)", flush=True)
    return path


if __name__ == "__main__":
    for c in (sys.argv[1:] or list(CASES)):
        make(c)
