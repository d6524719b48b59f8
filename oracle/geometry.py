"""Straight-panel mesh of a closed curve and the P1 hat basis (oracle).

Paper, Notation and Background: the current is expanded in piecewise-linear
Lagrange interpolants phi_i on a mesh of segments of the closed curve. On a
closed curve there is one hat function per node, so #unknowns = #nodes = N.

Panel p runs from node p to node p+1 (mod N), with length h_p, unit tangent
tau_p and outward normal n_p = (tau_y, -tau_x) (nodes counter-clockwise).
On panel p the local parameter xi in [0, 1] gives the two local shape
functions psi_0 = 1 - xi (node p) and psi_1 = xi (node p+1);
d psi_0/ds = -1/h_p and d psi_1/ds = +1/h_p.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Mesh:
    nodes: np.ndarray   # (N, 2)
    h: np.ndarray       # (N,)   panel lengths
    tau: np.ndarray     # (N, 2) unit tangents
    nrm: np.ndarray     # (N, 2) outward unit normals

    @property
    def n(self) -> int:
        return int(self.nodes.shape[0])

    def points(self, xi: np.ndarray) -> np.ndarray:
        """Points x_p(xi) = node_p + xi h_p tau_p, shape (N, len(xi), 2)."""
        return (self.nodes[:, None, :]
                + xi[None, :, None] * (self.h[:, None, None] * self.tau[:, None, :]))


def mesh(nodes: np.ndarray) -> Mesh:
    nodes = np.asarray(nodes, dtype=np.float64)
    if nodes.ndim != 2 or nodes.shape[1] != 2 or nodes.shape[0] < 4:
        raise ValueError("nodes must have shape (N, 2) with N >= 4")
    d = np.roll(nodes, -1, axis=0) - nodes
    h = np.hypot(d[:, 0], d[:, 1])
    if np.any(h == 0.0) or not np.all(np.isfinite(h)):
        raise ValueError("zero-length or non-finite panel")
    tau = d / h[:, None]
    nrm = np.stack([tau[:, 1], -tau[:, 0]], axis=1)
    return Mesh(nodes, h, tau, nrm)


def signed_area(nodes: np.ndarray) -> float:
    """Shoelace area; positive for counter-clockwise node order."""
    x, y = nodes[:, 0], nodes[:, 1]
    return 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))


# ----------------------------------------------------------------------------- equal-chord meshes
# Paper, Laplacian Filters, Two-Dimensional Case: the filter is defined through
# the SVD of L~ = G^{-1/2} L G^{-1/2}, which on a homogeneously discretised curve
# (all panels of one length) is the plain L up to a scalar and is diagonalised
# by the DFT, so that the filter needs no eigensolver. A homogeneous mesh of a
# closed curve is a polygon inscribed in the curve with n equal chords.
#
# Curves here are trigonometric polynomials in Cartesian form,
#   x(t) = sum_m ax[m] cos(m t) + bx[m] sin(m t),  y(t) likewise with ay, by,
# t in [0, 2 pi), counter-clockwise.

def trig_point(trig, t):
    """(x(t), y(t)) of the trigonometric-polynomial curve, t scalar or array."""
    ax, bx, ay, by = (np.asarray(v, dtype=np.float64) for v in trig)
    m = np.arange(ax.size, dtype=np.float64)
    tt = np.asarray(t, dtype=np.float64)
    c = np.cos(np.multiply.outer(tt, m))
    s = np.sin(np.multiply.outer(tt, m))
    return np.stack([c @ ax + s @ bx, c @ ay + s @ by], axis=-1)


def equal_chord_params(trig, n: int):
    """Parameters 0 = t_0 < t_1 < ... < t_{n-1} < 2 pi of n points of the curve whose
    n chords |r(t_{i+1}) - r(t_i)| (cyclic, t_n = 2 pi) are all equal.

    Each t_{i+1} is the first parameter after t_i at chord distance c from r(t_i)
    (bracketed by steps shorter than c / max|r'|, then Brent's method); c is the
    root of the closing defect F(c) = |r(2 pi) - r(t_{n-1}(c))| - c, which falls
    with c (a walk that passes t = 2 pi early counts as F = -c). Returns (t, c)."""
    from scipy.optimize import brentq

    if n < 4:
        raise ValueError("n >= 4")
    ts = np.linspace(0.0, 2.0 * np.pi, 20001)
    pts = trig_point(trig, ts)
    seg = np.hypot(*(np.diff(pts, axis=0).T))
    length = float(seg.sum())
    vmax = float(seg.max()) / (ts[1] - ts[0])
    two_pi = 2.0 * np.pi

    def walk(c):
        t = np.empty(n)
        t[0] = 0.0
        dt = 0.25 * c / vmax
        for i in range(1, n):
            p0 = trig_point(trig, t[i - 1])

            def g(s):
                return float(np.hypot(*(trig_point(trig, s) - p0))) - c

            a = t[i - 1]
            b = a + dt
            while g(b) < 0.0:
                a, b = b, b + dt
                if a > two_pi:
                    return None
            t[i] = brentq(g, a, b, xtol=1e-15, rtol=8.9e-16, maxiter=200)
            if t[i] >= two_pi:
                return None
        return t

    def defect(c):
        t = walk(c)
        if t is None:
            return -c
        return float(np.hypot(*(trig_point(trig, two_pi) - trig_point(trig, t[-1])))) - c

    hi = length / n
    while defect(hi) > 0.0:          # the polyline length is slightly below the curve length
        hi *= 1.0 + 1.0 / 1024
    c = brentq(defect, 0.5 * length / n, hi, xtol=1e-17, rtol=8.9e-16, maxiter=200)
    return walk(c), c


def equal_chord_nodes(trig, n: int) -> np.ndarray:
    """Nodes (n, 2) of the equal-chord mesh (equal_chord_params)."""
    t, _ = equal_chord_params(trig, n)
    return trig_point(trig, t)
