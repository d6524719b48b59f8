"""Pins of the CPU oracle against facts fixed outside it (closed forms,
brute-force integrals, identities). No GPU involved."""
import math
import os

import mpmath as mp
import numpy as np
import pytest
from scipy import special as sp

from oracle import assembly, geometry, quadrature, rng, special
from paper_2210_08580_amd import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def circle_eigs(m, k, a=1.0):
    """Fourier-mode eigenvalues on the circle of radius a (Graf's addition theorem):
    lam_S = (i pi a/2) J_m H_m, lam_N = -(i pi a k^2/2) J_m' H_m',
    lam_D = (i pi x/4)(J_m H_m' + J_m' H_m), x = k a."""
    x = k * a
    J, H = sp.jv(m, x), sp.hankel1(m, x)
    Jp, Hp = sp.jvp(m, x), sp.h1vp(m, x)
    return (0.5j * np.pi * a * J * H, -0.5j * np.pi * a * k * k * Jp * Hp,
            0.25j * np.pi * x * (J * Hp + Jp * H))


def circulant_eigs(A, G, ms):
    n = A.shape[0]
    th = 2 * np.pi * np.arange(n) / n
    E = np.exp(1j * np.outer(th, ms))
    return (A[0] @ E) / (G[0] @ E)


# ----------------------------------------------------------------------------- special functions
def test_gauss_legendre_exactness():
    x, w = quadrature.gauss_legendre_01(8)
    for d in range(16):
        assert abs(w @ x ** d - 1.0 / (d + 1)) < 1e-15
    assert abs(w @ x ** 16 - 1.0 / 17) > 1e-12   # degree 2n is not integrated exactly


def test_hankel_against_mpmath():
    mp.mp.dps = 30
    xs = np.concatenate([np.geomspace(1e-8, 100.0, 240), np.linspace(0.5, 40.0, 160)])
    h0, h1 = special.hankel1_01(xs)
    for x, a, b in zip(xs, h0, h1):
        ref0 = complex(mp.besselj(0, x) + 1j * mp.bessely(0, x))
        ref1 = complex(mp.besselj(1, x) + 1j * mp.bessely(1, x))
        assert abs(a.real - ref0.real) <= 1e-14 * max(1.0, abs(ref0.real))
        assert abs(a.imag - ref0.imag) <= 1e-14 * max(1.0, abs(ref0.imag))
        assert abs(b.real - ref1.real) <= 1e-14 * max(1.0, abs(ref1.real))
        assert abs(b.imag - ref1.imag) <= 1e-14 * max(1.0, abs(ref1.imag))


def test_wronskian():
    xs = np.linspace(0.01, 100.0, 5000)
    h0, h1 = special.hankel1_01(xs)
    w = h1.real * h0.imag - h0.real * h1.imag           # J1 Y0 - J0 Y1 = 2/(pi x)
    assert np.max(np.abs(w * xs * np.pi / 2 - 1.0)) < 1e-13


def test_green_regular_part_limit():
    k = 3.7
    g0 = special.green_reg_at_zero(k)
    for R in (1e-6, 1e-8):
        assert abs(special.green_reg(k, np.array([R]))[0] - g0) < 1e-10
    mp.mp.dps = 30
    ref = complex(mp.mpf(1) / 4 * 1j - (mp.log(mp.mpf(k) / 2) + mp.euler) / (2 * mp.pi))
    assert abs(g0 - ref) < 1e-15


def test_dgreen_laplace_limit():
    k = 2.0
    R = np.array([1e-7])
    c = special.dgreen_coef(k, R)
    assert abs(c[0] / special.dgreen_laplace_coef(R)[0] - 1.0) < 1e-9


# ----------------------------------------------------------------------------- singular integrals
def _read_gold(name):
    vals = {}
    with open(os.path.join(GOLD, name)) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            a, b = line.split()
            vals[a] = b
    return vals


def test_self_panel_constants():
    gold = _read_gold("self_panel_log.txt")
    J = quadrature.SELF_LOG_J
    assert J[0, 0] == float(gold["J00"]) and J[1, 1] == float(gold["J11"])
    assert J[0, 1] == float(gold["J01"]) and J[1, 0] == float(gold["J01"])
    mp.mp.dps = 25

    def lg(x, y):
        d = abs(x - y)
        return mp.log(d) if d != 0 else mp.mpf(0)
    psi = [lambda s: 1 - s, lambda s: s]
    for a in range(2):
        for b in range(2):
            v = mp.quad(lambda x: mp.quad(lambda y: psi[a](x) * psi[b](y) * lg(x, y),
                                          [0, x, 1]), [0, 1])
            assert abs(float(v) - J[a, b]) < 1e-15
    h = 0.37
    ref = h * h * (0.25 * math.log(h) + J)
    assert np.allclose(quadrature.self_log(h), ref, rtol=0, atol=1e-16)


@pytest.mark.parametrize("angle", [math.pi * 0.97, math.pi * 0.7, math.pi * 0.4])
@pytest.mark.parametrize("case", [(True, False), (False, True)])
def test_adjacent_singular_vs_mpmath(angle, case):
    """Brute-force 2D tanh-sinh quadrature of the corner-singular integrals."""
    end_x, end_y = case
    hp, hq = 0.3, 0.45
    a = np.array([1.0, 0.0])
    b = np.array([math.cos(angle), math.sin(angle)])
    nq = np.array([b[1], -b[0]])
    Lg, Dl = quadrature.adjacent_singular(hp, hq, a, b, nq, end_x, end_y)
    mp.mp.dps = 20
    ab, anq = float(a @ b), float(a @ nq)

    def psi(al, s, end):
        xi = 1 - s if end else s
        return (1 - xi) if al == 0 else xi

    for al in range(2):
        for be in range(2):
            def R2(s1, s2):
                return hp * hp * s1 * s1 + hq * hq * s2 * s2 - 2 * hp * hq * s1 * s2 * ab

            def fl(s1, s2):
                r2 = R2(s1, s2)
                return psi(al, s1, end_x) * psi(be, s2, end_y) * (mp.log(r2) / 2 if r2 > 0 else 0)

            def fd(s1, s2):
                r2 = R2(s1, s2)
                return (psi(al, s1, end_x) * psi(be, s2, end_y) * hp * s1 * anq / r2
                        if r2 > 0 else 0)
            vl = hp * hq * mp.quad(fl, [0, 1], [0, 1])
            vd = hp * hq * mp.quad(fd, [0, 1], [0, 1]) / (2 * mp.pi)
            assert abs(Lg[al, be] - float(vl)) < 1e-13
            assert abs(Dl[al, be] - float(vd)) < 1e-13


# ----------------------------------------------------------------------------- sparse matrices
def test_gram_laplacian_closed_forms():
    nodes = wl.star(200)
    m = geometry.mesh(nodes)
    Gd, Go = assembly.gram(m)
    Ld, Lo = assembly.laplacian(m)
    G = assembly.periodic_dense(Gd, Go)
    L = assembly.periodic_dense(Ld, Lo)
    one = np.ones(m.n)
    assert np.abs(L @ one).max() < 1e-10 * np.abs(L).max()
    assert abs(one @ G @ one - m.h.sum()) < 1e-13 * m.h.sum()
    # uniform circle: g_m = h (2 + cos th)/3, l_m = (2/h)(1 - cos th)
    n = 64
    mc = geometry.mesh(wl.circle(n))
    h = mc.h[0]
    th = 2 * np.pi * np.arange(n) / n
    Gc = assembly.periodic_dense(*assembly.gram(mc))
    Lc = assembly.periodic_dense(*assembly.laplacian(mc))
    E = np.exp(1j * np.outer(np.arange(n), th))
    assert np.allclose((Gc[0] @ E).real, h * (2 + np.cos(th)) / 3, atol=1e-15)
    assert np.allclose((Lc[0] @ E).real, (2 / h) * (1 - np.cos(th)), rtol=1e-12, atol=1e-12)


# ----------------------------------------------------------------------------- Galerkin matrices
def test_closed_form_maue_identity():
    """lam_N(m) = (m/a)^2 lam_S(m) - (k^2/2)(lam_S(m-1) + lam_S(m+1)) on the circle."""
    for k, a in ((1.0, 1.0), (4.0, 0.7)):
        ms = np.arange(-6, 7)
        lS, lN, _ = circle_eigs(ms, k, a)
        lSm, _, _ = circle_eigs(ms - 1, k, a)
        lSp, _, _ = circle_eigs(ms + 1, k, a)
        rhs = (ms / a) ** 2 * lS - 0.5 * k * k * (lSm + lSp)
        assert np.max(np.abs(lN - rhs)) < 1e-12 * np.max(np.abs(lN))


@pytest.mark.parametrize("k", [1.0, 5.0])
def test_circle_eigenvalues_second_order(k):
    ms = np.arange(0, 6)
    errs = []
    for n in (64, 128, 256):
        m = geometry.mesh(wl.circle(n))
        S, Nm, D = assembly.assemble(m, k)
        G = assembly.periodic_dense(*assembly.gram(m))
        lS, lN, lD = circle_eigs(ms, k)
        errs.append([np.max(np.abs(circulant_eigs(A, G, ms) - lam) / np.abs(lam))
                     for A, lam in ((S, lS), (Nm, lN), (D, lD))])
    errs = np.array(errs)
    order = np.log2(errs[:-1] / errs[1:])
    assert np.all(order > 1.8), (errs, order)
    assert np.all(errs[-1] < 2e-3)


def test_gauss_lemma_and_constant_in_N():
    """k -> 0: sum_j D_ij = -1/2 sum_j G_ij (solid angle of a closed curve) and
    N 1 = 0 (Maue form; the tangential derivative of a constant vanishes)."""
    m = geometry.mesh(wl.star(128))
    S, Nm, D = assembly.assemble(m, 1e-7)
    G = assembly.periodic_dense(*assembly.gram(m))
    assert np.abs(D.sum(1) + 0.5 * G.sum(1)).max() < 1e-12
    assert np.abs(Nm.sum(1)).max() < 1e-12 * np.abs(Nm).max()


def test_symmetry_and_sampled_entries():
    m = geometry.mesh(wl.ellipse(96))
    k = 3.0
    S, Nm, D = assembly.assemble(m, k)
    for A in (S, Nm):
        assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    rs = np.random.default_rng(5)
    I = np.concatenate([rs.integers(0, 96, 40), np.arange(96), [0, 95, 1]])
    J = np.concatenate([rs.integers(0, 96, 40), (np.arange(96) + 1) % 96, [95, 0, 94]])
    s, nn, d = assembly.entries(m, k, I, J)
    assert np.abs(s - S[I, J]).max() < 1e-15 * np.abs(S).max() * 10
    assert np.abs(nn - Nm[I, J]).max() < 1e-15 * np.abs(Nm).max() * 10
    assert np.abs(d - D[I, J]).max() < 1e-15 * np.abs(D).max() * 10


def test_rhs_planewave_moments():
    """<phi_i, u> against a dense 40-point panel rule; f is the moment of du/dn."""
    m = geometry.mesh(wl.star(64))
    k = 2.5
    f, h = assembly.rhs_planewave(m, k, [0.4], [1.0 + 0.5j], nq=8)
    f40, h40 = assembly.rhs_planewave(m, k, [0.4], [1.0 + 0.5j], nq=40)
    assert np.abs(h - h40).max() < 1e-13 and np.abs(f - f40).max() < 1e-12
    # sum_i h_i = int u ds on the polygon; a constant field integrates to the perimeter
    f0, h0 = assembly.rhs_planewave(m, 0.0, [0.0], [1.0])
    assert abs(h0.sum() - m.h.sum()) < 1e-13 and np.abs(f0).max() == 0.0


# ----------------------------------------------------------------------------- RNG
def test_splitmix64_published_outputs():
    with open(os.path.join(GOLD, "splitmix64_state0.txt")) as fh:
        rows = [l.split() for l in fh if l.strip() and not l.startswith("#")]
    for s_in, s_out in rows:
        assert int(rng.splitmix64(np.uint64(int(s_in, 16)))) == int(s_out, 16)


def test_sketch_matches_integer_reference():
    """Pure-Python big-int re-derivation of the counter rule (independent code)."""
    mask = (1 << 64) - 1

    def mix(z):
        z = (z + 0x9E3779B97F4A7C15) & mask
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        return z ^ (z >> 31)
    seed, n, ell = 0xDEADBEEF12345, 7, 5
    Om = rng.sketch(seed, n, ell)
    for i in range(n):
        for j in range(ell):
            z = mix(seed ^ (i * ell + j))
            ref = complex(1 - 2 * (z & 1), 1 - 2 * ((z >> 1) & 1)) / math.sqrt(2)
            assert Om[i, j] == ref
    big = rng.sketch(3, 300, 40)
    assert abs(big.real.mean()) < 0.05 and abs(big.imag.mean()) < 0.05
