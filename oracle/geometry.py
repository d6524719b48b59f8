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
