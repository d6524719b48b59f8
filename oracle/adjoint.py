"""Far-field objective of the inverse-problem use case and its gradient (oracle;
test infrastructure, never called by the library).

The paper's introduction names inverse problems among the settings that need many
solves with one operator; it defines no objective. The reading adopted here:

Forward model: the unfiltered Galerkin TE-EFIE of the paper's Notation and
Background, N j = -f (the constant (ik)^-1 moved into f as in the normalised
formulation), for plane waves u_inc = A exp(i k d.x); on the sound-hard boundary
the total field is u = -j (sign convention of the paper's TE-MFIE).

Far field (convention u_s ~ u_inf(theta) exp(ikr)/sqrt(r)): with du/dn = 0 on
the boundary, Green's representation gives the scattered field as the double
layer of the total field, u_s(x) = int_Gamma d/dn_y g(|x - y|) u(y) ds_y; the
large-|x| form of g then gives
    u_inf(theta) = e^{i pi/4} / sqrt(8 pi k) int_Gamma (-i k th.n_y) e^{-i k th.y} u(y) ds_y,
th = (cos theta, sin theta), evaluated with the same 8-point Gauss rule per panel
as the right-hand sides, u = -sum_i j_i phi_i. As a matrix: (F j)_l.

Objective: J = sum_r sum_l |(F j_r)_l - T_{l,r}|^2.

Gradient by the adjoint method. With e_r = F j_r - T_r and N^H lambda_r = F^H e_r,
    dJ = sum_r 2 Re[e_r^H (dF) j_r] - 2 Re[lambda_r^H (df_r + (dN) j_r)].
The oracle takes dN, df, dF with respect to each node coordinate by central
differences of its own assembly, Richardson-extrapolated to fourth order,
D = (4 D(d) - D(2d))/3 with D(d) the central difference of step d = 1e-3 of the
mean panel length: the assembled entries are analytic in the node coordinates on
the scale of the panel length, so the error is ~(d/h)^4 ~ 1e-12 of the entry
scale, where a plain central difference would need a step near 1e-6 h and lose
~1e-10 to rounding (slow, plainly correct, independent of the HIP derivative
kernels). The amplitude gradient is closed-form: J is quadratic in
A_r with F j_r = A_r a_r, so dJ/dRe A_r + i dJ/dIm A_r = 2 sum_l e_rl conj(a_rl).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import assembly
from .geometry import Mesh, mesh


def farfield_matrix(m: Mesh, k: float, thetas, nq: int = 8) -> np.ndarray:
    """F (nang x N): (F j)_l = u_inf(theta_l) for the current j (u = -j)."""
    thetas = np.atleast_1d(np.asarray(thetas, dtype=np.float64))
    xi, w, psi, wpsi = assembly._rule(nq)
    pts = m.points(xi)                                          # (N, nq, 2)
    th = np.stack([np.cos(thetas), np.sin(thetas)], axis=1)     # (L, 2)
    c_inf = np.exp(0.25j * np.pi) / np.sqrt(8.0 * np.pi * k)
    phase = np.einsum("pad,ld->lpa", pts, th)                   # (L, N, nq)
    tn = th @ m.nrm.T                                           # (L, N)
    ker = c_inf * (-1j * k) * tn[:, :, None] * np.exp(-1j * k * phase)
    # u(x) = -(j_p psi_0 + j_{p+1} psi_1) on panel p
    loc = -m.h[None, :, None] * np.einsum("ia,lpa->lpi", wpsi, ker)      # (L, N, 2)
    return loc[:, :, 0] + np.roll(loc[:, :, 1], 1, axis=1)


def forward(nodes, k: float, angles, amps, thetas):
    """j (N x R) of N j = -f and the far fields F j (nang x R)."""
    m = mesh(nodes)
    _, Nm, _ = assembly.assemble(m, k)
    f, _ = assembly.rhs_planewave(m, k, angles, amps)
    j = sla.solve(Nm, -f.T)
    return j, farfield_matrix(m, k, thetas) @ j


def objective(nodes, k: float, angles, amps, thetas, T) -> float:
    _, FJ = forward(nodes, k, angles, amps, thetas)
    return float(np.sum(np.abs(FJ - T) ** 2))


def gradient(nodes, k: float, angles, amps, thetas, T, rel_step: float = 1e-3):
    """(J, dJ/d nodes (N x 2), dJ/dRe A + i dJ/dIm A (R,)) by the adjoint method."""
    nodes = np.asarray(nodes, dtype=np.float64)
    amps = np.atleast_1d(np.asarray(amps, dtype=np.complex128))
    m = mesh(nodes)
    _, Nm, _ = assembly.assemble(m, k)
    f, _ = assembly.rhs_planewave(m, k, angles, amps)
    F = farfield_matrix(m, k, thetas)
    lu = sla.lu_factor(Nm)
    j = sla.lu_solve(lu, -f.T)
    FJ = F @ j
    E = FJ - T
    J = float(np.sum(np.abs(E) ** 2))
    lam = sla.lu_solve(lu, (F.conj().T @ E), trans=2)           # N^H lambda = F^H e
    g_amp = 2.0 * np.sum(E * np.conj(FJ / amps[None, :]), axis=0)

    delta = rel_step * float(np.mean(m.h))
    grad = np.zeros_like(nodes)
    for i in range(nodes.shape[0]):
        for a in range(2):
            ops = []
            for s in (1.0, -1.0, 2.0, -2.0):
                x = nodes.copy()
                x[i, a] += s * delta
                mm = mesh(x)
                _, Nx, _ = assembly.assemble(mm, k)
                fx, _ = assembly.rhs_planewave(mm, k, angles, amps)
                ops.append((Nx, fx.T, farfield_matrix(mm, k, thetas)))
            # central differences of steps delta and 2 delta, then (4 D1 - D2) / 3
            d1 = [(ops[0][t] - ops[1][t]) / (2.0 * delta) for t in range(3)]
            d2 = [(ops[2][t] - ops[3][t]) / (4.0 * delta) for t in range(3)]
            dN, df, dF = [(4.0 * u - v) / 3.0 for u, v in zip(d1, d2)]
            grad[i, a] = (2.0 * np.sum(np.real(np.conj(E) * (dF @ j)))
                          - 2.0 * np.sum(np.real(np.conj(lam) * (df + dN @ j))))
    return J, grad, g_amp
