"""Galerkin matrices of the 2D TE problem (oracle; test infrastructure).

Paper, Notation and Background:
  [S]_ij = <phi_i, S phi_j>, [D]_ij = <phi_i, D phi_j>, [N]_ij = <phi_i, N phi_j>,
  [G]_ij = <phi_i, phi_j>, [e]_i = <phi_i, e_t^inc>, [h]_i = <phi_i, h_z^inc>,
with the bilinear pairing <a, b> = int a b ds (no conjugation), and (Laplacian
Filters, 2D case) [L]_ij = <grad phi_i, grad phi_j>.

The paper defines N only as the hypersingular operator -d/dn int d/dn' g. The
oracle evaluates it in Maue's integrated-by-parts form,
  <phi_i, N phi_j> = int int g(|x-y|) [phi_i'(x) phi_j'(y) - k^2 (n_x.n_y) phi_i(x) phi_j(y)],
(' = arc-length derivative), which leaves only the log-singular kernel g.

Entries are sums of 2x2 local blocks over the panel pairs (p, q) touching
nodes i and j: panel p carries psi_0 of node p and psi_1 of node p+1.
For a pair, with s_0 = -1, s_1 = +1:
  S_ab = int_p int_q psi_a psi_b g,   I0 = int_p int_q g = sum_ab S_ab,
  N_ab = s_a s_b I0 / (h_p h_q) - k^2 (n_p.n_q) S_ab,
  D_ab = int_p int_q psi_a psi_b (dg/dn_y).
Quadrature: see oracle.quadrature. The S and N bands |i - j| <= 2 (mod N),
which receive the singular-pair contributions, are symmetrised.
"""
from __future__ import annotations

import numpy as np

from . import quadrature as qd
from . import special as sf
from .geometry import Mesh

TWO_PI = 2.0 * np.pi
SIGNS = np.array([-1.0, 1.0])


# ----------------------------------------------------------------------------- sparse
def gram(m: Mesh):
    """P1 Gram matrix: G_ii = (h_{i-1} + h_i)/3, G_{i,i+1} = h_i/6 (periodic).

    Returns (diag, off) with off[i] = G[i, i+1 mod N]."""
    return (np.roll(m.h, 1) + m.h) / 3.0, m.h / 6.0


def laplacian(m: Mesh):
    """P1 stiffness matrix: L_ii = 1/h_{i-1} + 1/h_i, L_{i,i+1} = -1/h_i (periodic)."""
    inv = 1.0 / m.h
    return np.roll(inv, 1) + inv, -inv


def periodic_dense(diag: np.ndarray, off: np.ndarray) -> np.ndarray:
    n = diag.shape[0]
    A = np.diag(diag).astype(np.float64)
    i = np.arange(n)
    A[i, (i + 1) % n] += off
    A[(i + 1) % n, i] += off
    return A


# ----------------------------------------------------------------------------- local blocks
def _rule(nq: int):
    xi, w = qd.gauss_legendre_01(nq)
    psi = qd.shape_values(xi)                                # (2, nq)
    wpsi = w[None, :] * psi                                  # (2, nq)
    return xi, w, psi, wpsi


def regular_blocks(m: Mesh, k: float, P: np.ndarray, Q: np.ndarray, nq: int = 8):
    """Tensor Gauss rule for arrays of panel pairs (P[t], Q[t]).

    Returns S (T,2,2), I0 (T,), D (T,2,2) (complex)."""
    xi, w, psi, wpsi = _rule(nq)
    pts = m.points(xi)                                       # (N, nq, 2)
    xa = pts[P][:, :, None, :]
    yb = pts[Q][:, None, :, :]
    diff = xa - yb
    R = np.hypot(diff[..., 0], diff[..., 1])                 # (T, nq, nq)
    g = sf.green(k, R)
    dn = diff[..., 0] * m.nrm[Q][:, None, None, 0] + diff[..., 1] * m.nrm[Q][:, None, None, 1]
    dk = sf.dgreen_coef(k, R) * dn
    hh = (m.h[P] * m.h[Q])[:, None, None]
    S = hh * np.einsum("ia,jb,tab->tij", wpsi, wpsi, g)
    D = hh * np.einsum("ia,jb,tab->tij", wpsi, wpsi, dk)
    I0 = hh[:, 0, 0] * np.einsum("a,b,tab->t", w, w, g)
    return S, I0, D


def near_block(m: Mesh, k: float, p: int, q: int, nq: int = 8, nt: int = 32):
    """Local blocks for a self (p == q) or adjacent pair, singular parts exact."""
    n = m.n
    xi, w, psi, wpsi = _rule(nq)
    pts = m.points(xi)
    diff = pts[p][:, None, :] - pts[q][None, :, :]
    R = np.hypot(diff[..., 0], diff[..., 1])
    hp, hq = m.h[p], m.h[q]
    greg = sf.green_reg(k, R)
    Sreg = hp * hq * np.einsum("ia,jb,ab->ij", wpsi, wpsi, greg)
    if p == q:
        Lg = qd.self_log(hp)
        D = np.zeros((2, 2), dtype=np.complex128)
    else:
        if q == (p + 1) % n:      # shared node = end of p = start of q
            a, b, end_x, end_y = -m.tau[p], m.tau[q], True, False
        elif q == (p - 1) % n:    # shared node = start of p = end of q
            a, b, end_x, end_y = m.tau[p], -m.tau[q], False, True
        else:
            raise ValueError("not a near pair")
        Lg, Dl = qd.adjacent_singular(hp, hq, a, b, m.nrm[q], end_x, end_y, nt)
        dn = diff[..., 0] * m.nrm[q][0] + diff[..., 1] * m.nrm[q][1]
        rem = (sf.dgreen_coef(k, R) - sf.dgreen_laplace_coef(R)) * dn
        D = Dl + hp * hq * np.einsum("ia,jb,ab->ij", wpsi, wpsi, rem)
    S = Sreg - Lg / TWO_PI
    I0 = S.sum()
    return S, I0, D


def is_near(n: int, p, q):
    d = np.abs(np.asarray(p) - np.asarray(q)) % n
    return (d <= 1) | (d >= n - 1)


def pair_blocks(m: Mesh, k: float, P, Q, nq: int = 8):
    """S, N, D local blocks for arbitrary panel pairs (near pairs handled)."""
    P = np.atleast_1d(np.asarray(P, dtype=np.int64))
    Q = np.atleast_1d(np.asarray(Q, dtype=np.int64))
    S = np.empty((P.size, 2, 2), dtype=np.complex128)
    D = np.empty_like(S)
    I0 = np.empty(P.size, dtype=np.complex128)
    near = is_near(m.n, P, Q)
    far = ~near
    if far.any():
        S[far], I0[far], D[far] = regular_blocks(m, k, P[far], Q[far], nq)
    for t in np.nonzero(near)[0]:
        S[t], I0[t], D[t] = near_block(m, k, int(P[t]), int(Q[t]), nq)
    hh = m.h[P] * m.h[Q]
    npq = np.sum(m.nrm[P] * m.nrm[Q], axis=1)
    Nb = (SIGNS[None, :, None] * SIGNS[None, None, :] * (I0 / hh)[:, None, None]
          - (k * k) * npq[:, None, None] * S)
    return S, Nb, D


# ----------------------------------------------------------------------------- full assembly
def assemble(m: Mesh, k: float, nq: int = 8, row_chunk: int | None = None):
    """Dense S, N, D (N x N complex128)."""
    n = m.n
    S = np.zeros((n, n), dtype=np.complex128)
    Nm = np.zeros_like(S)
    D = np.zeros_like(S)
    if row_chunk is None:
        row_chunk = max(1, 2 ** 21 // (n * nq * nq))
    qs = np.arange(n)
    for p0 in range(0, n, row_chunk):
        ps = np.arange(p0, min(n, p0 + row_chunk))
        P = np.repeat(ps, n)
        Q = np.tile(qs, ps.size)
        Sb, Nb, Db = pair_blocks(m, k, P, Q, nq)
        for M, B in ((S, Sb), (Nm, Nb), (D, Db)):
            B = B.reshape(ps.size, n, 2, 2)
            for al in range(2):
                rows = (ps + al) % n
                # entry (p+al, q+be) += block[p, q, al, be]
                M[rows, :] += B[:, :, al, 0] + np.roll(B[:, :, al, 1], 1, axis=1)
    _symmetrise_band(S)
    _symmetrise_band(Nm)
    return S, Nm, D


# ----------------------------------------------------------------------------- Yukawa single layer
def yukawa_pair_blocks(m: Mesh, kappa: float, P, Q, nq: int = 8, nt: int = 32):
    """2 x 2 blocks of the single layer with the Yukawa kernel (1/2 pi) K0(kappa R)
    (the Calderon preconditioner of the Yukawa-Calderon TE-CFIE, paper, Filters
    Based Fast Direct Solver, 2D case) for panel pairs (P[t], Q[t]): far pairs by
    the tensor Gauss rule, self and adjacent pairs with the same exact logarithmic
    parts as S (the kernel has the Laplace singularity -(1/2 pi) log R)."""
    P = np.atleast_1d(np.asarray(P, dtype=np.int64))
    Q = np.atleast_1d(np.asarray(Q, dtype=np.int64))
    n = m.n
    xi, w, psi, wpsi = _rule(nq)
    pts = m.points(xi)
    out = np.empty((P.size, 2, 2), dtype=np.float64)
    near = is_near(n, P, Q)
    far = ~near
    if far.any():
        Pf, Qf = P[far], Q[far]
        diff = pts[Pf][:, :, None, :] - pts[Qf][:, None, :, :]
        g = sf.yukawa(kappa, np.hypot(diff[..., 0], diff[..., 1]))
        hh = (m.h[Pf] * m.h[Qf])[:, None, None]
        out[far] = hh * np.einsum("ia,jb,tab->tij", wpsi, wpsi, g)
    for t in np.nonzero(near)[0]:
        p, q = int(P[t]), int(Q[t])
        diff = pts[p][:, None, :] - pts[q][None, :, :]
        greg = sf.yukawa_reg(kappa, np.hypot(diff[..., 0], diff[..., 1]))
        Sreg = m.h[p] * m.h[q] * np.einsum("ia,jb,ab->ij", wpsi, wpsi, greg)
        if p == q:
            Lg = qd.self_log(m.h[p])
        else:
            if q == (p + 1) % n:
                a, b, end_x, end_y = -m.tau[p], m.tau[q], True, False
            else:
                a, b, end_x, end_y = m.tau[p], -m.tau[q], False, True
            Lg, _ = qd.adjacent_singular(m.h[p], m.h[q], a, b, m.nrm[q], end_x, end_y, nt)
        out[t] = Sreg - Lg / TWO_PI
    return out


def assemble_yukawa(m: Mesh, kappa: float, nq: int = 8, row_chunk: int | None = None):
    """Dense Yukawa single layer S_y (N x N real), symmetrised on |i - j| <= 2 like S."""
    n = m.n
    Sy = np.zeros((n, n), dtype=np.float64)
    if row_chunk is None:
        row_chunk = max(1, 2 ** 21 // (n * nq * nq))
    qs = np.arange(n)
    for p0 in range(0, n, row_chunk):
        ps = np.arange(p0, min(n, p0 + row_chunk))
        B = yukawa_pair_blocks(m, kappa, np.repeat(ps, n), np.tile(qs, ps.size), nq).reshape(ps.size, n, 2, 2)
        for al in range(2):
            rows = (ps + al) % n
            Sy[rows, :] += B[:, :, al, 0] + np.roll(B[:, :, al, 1], 1, axis=1)
    _symmetrise_band(Sy)
    return Sy


def entries_yukawa(m: Mesh, kappa: float, I, J, nq: int = 8):
    """Sampled entries of S_y one by one, the same rule as assemble_yukawa()."""
    I = np.asarray(I, dtype=np.int64)
    J = np.asarray(J, dtype=np.int64)
    n = m.n

    def raw(I, J):
        v = np.zeros(I.size, dtype=np.float64)
        for al in range(2):
            for be in range(2):
                v += yukawa_pair_blocks(m, kappa, (I - al) % n, (J - be) % n, nq)[:, al, be]
        return v

    v = raw(I, J)
    band = band_mask(n, I, J)
    if band.any():
        v[band] = 0.5 * (v[band] + raw(J[band], I[band]))
    return v


def band_mask(n: int, i, j, width: int = 2):
    d = np.abs(np.asarray(i) - np.asarray(j)) % n
    return (d <= width) | (d >= n - width)


def _symmetrise_band(M: np.ndarray):
    n = M.shape[0]
    for off in range(0, 3):
        i = np.arange(n)
        j = (i + off) % n
        avg = 0.5 * (M[i, j] + M[j, i])
        M[i, j] = avg
        M[j, i] = avg


def entries(m: Mesh, k: float, I, J, nq: int = 8):
    """Sampled entries (S_ij, N_ij, D_ij) computed one by one, same rule as
    assemble() (including the band symmetrisation of S and N)."""
    I = np.asarray(I, dtype=np.int64)
    J = np.asarray(J, dtype=np.int64)
    n = m.n

    def raw(I, J):
        out = [np.zeros(I.size, dtype=np.complex128) for _ in range(3)]
        for al in range(2):
            for be in range(2):
                P = (I - al) % n
                Q = (J - be) % n
                Sb, Nb, Db = pair_blocks(m, k, P, Q, nq)
                out[0] += Sb[:, al, be]
                out[1] += Nb[:, al, be]
                out[2] += Db[:, al, be]
        return out

    s, nn, d = raw(I, J)
    band = band_mask(n, I, J)
    if band.any():
        sT, nT, _ = raw(J[band], I[band])
        s[band] = 0.5 * (s[band] + sT)
        nn[band] = 0.5 * (nn[band] + nT)
    return s, nn, d


# ----------------------------------------------------------------------------- RHS
def rhs_planewave(m: Mesh, k: float, angles, amps, nq: int = 8):
    """Incident plane waves u = A exp(i k d.x), d = (cos phi, sin phi).

    Returns f[r, i] = <phi_i, du/dn> and h[r, i] = <phi_i, u> (nrhs x N), by an
    nq-point Gauss rule per panel. du/dn = i k (n.d) u."""
    angles = np.atleast_1d(np.asarray(angles, dtype=np.float64))
    amps = np.atleast_1d(np.asarray(amps, dtype=np.complex128))
    xi, w, psi, wpsi = _rule(nq)
    pts = m.points(xi)                                          # (N, nq, 2)
    d = np.stack([np.cos(angles), np.sin(angles)], axis=1)       # (R, 2)
    phase = np.einsum("pad,rd->rpa", pts, d)
    u = amps[:, None, None] * np.exp(1j * k * phase)              # (R, N, nq)
    nd = m.nrm @ d.T                                              # (N, R)
    dudn = 1j * k * nd.T[:, :, None] * u
    n = m.n
    out = []
    for fld in (dudn, u):
        loc = m.h[None, :, None] * np.einsum("ia,rpa->rpi", wpsi, fld)   # (R, N, 2)
        out.append(loc[:, :, 0] + np.roll(loc[:, :, 1], 1, axis=1))
    return out[0], out[1]
