"""Planted mistakes: each test breaks the oracle on purpose (on the CPU, via
monkeypatch) and checks that one of the pins would have caught it."""
import numpy as np
from scipy import special as sp

from oracle import assembly, filters, geometry, quadrature, special, woodbury
from paper_2210_08580_amd import workloads as wl


def _circle_error(k=1.0, n=64):
    ms = np.arange(0, 6)
    m = geometry.mesh(wl.circle(n))
    S, Nm, D = assembly.assemble(m, k)
    G = assembly.periodic_dense(*assembly.gram(m))
    th = 2 * np.pi * np.arange(n) / n
    E = np.exp(1j * np.outer(th, ms))
    g = G[0] @ E
    x = k
    lS = 0.5j * np.pi * sp.jv(ms, x) * sp.hankel1(ms, x)
    lN = -0.5j * np.pi * k * k * sp.jvp(ms, x) * sp.h1vp(ms, x)
    lD = 0.25j * np.pi * x * (sp.jv(ms, x) * sp.h1vp(ms, x) + sp.jvp(ms, x) * sp.hankel1(ms, x))
    return [np.max(np.abs((A[0] @ E) / g - lam)) / np.max(np.abs(lam)) for A, lam in
            ((S, lS), (Nm, lN), (D, lD))]


def test_pin_baseline_is_small():
    assert max(_circle_error()) < 2e-3


def test_dropped_k2_term_in_maue_form_is_caught(monkeypatch):
    orig = assembly.pair_blocks

    def broken(m, k, P, Q, nq=8):
        S, Nb, D = orig(m, k, P, Q, nq)
        hh = m.h[np.atleast_1d(P)] * m.h[np.atleast_1d(Q)]
        npq = np.sum(m.nrm[np.atleast_1d(P)] * m.nrm[np.atleast_1d(Q)], axis=1)
        return S, Nb + (k * k) * npq[:, None, None] * S, D    # drop -k^2 (n.n) S
    monkeypatch.setattr(assembly, "pair_blocks", broken)
    assert _circle_error()[1] > 0.1


def test_wrong_double_layer_sign_is_caught(monkeypatch):
    monkeypatch.setattr(special, "dgreen_coef",
                        lambda k, R: -0.25j * k * (sp.j1(k * R) + 1j * sp.y1(k * R)) / R)
    m = geometry.mesh(wl.star(64))
    S, Nm, D = assembly.assemble(m, 1e-7)
    G = assembly.periodic_dense(*assembly.gram(m))
    assert np.abs(D.sum(1) + 0.5 * G.sum(1)).max() > 1e-2


def test_transposed_self_constants_are_caught(monkeypatch):
    """Swapped same-node / cross-node constants leave the smooth circle modes
    almost unchanged; the brute-force mpmath pin of the self-panel integral catches it."""
    import mpmath as mp
    monkeypatch.setattr(quadrature, "SELF_LOG_J", quadrature.SELF_LOG_J[::-1].copy())
    mp.mp.dps = 20
    h = 0.37

    def lg(x, y):
        d = abs(x - y)
        return mp.log(h * d) if d != 0 else mp.mpf(0)
    ref = h * h * mp.quad(lambda x: mp.quad(lambda y: (1 - x) * (1 - y) * lg(x, y), [0, x, 1]),
                          [0, 1])
    assert abs(quadrature.self_log(h)[0, 0] - float(ref)) > 1e-3 * h * h


def test_dropped_green_regular_part_is_caught(monkeypatch):
    monkeypatch.setattr(special, "green_reg_at_zero", lambda k: 0.0)
    assert _circle_error()[0] > 2e-3


def test_woodbury_sign_slip_is_caught(monkeypatch):
    rs = np.random.default_rng(1)
    n, r, beta = 40, 5, 0.3
    U = rs.standard_normal((n, r)) + 0j
    W = rs.standard_normal((r, n)) * 0.1 + 0j
    v = rs.standard_normal((n, 1)) + 0j
    orig = woodbury.solve
    monkeypatch.setattr(woodbury, "solve",
                        lambda U, W, b, lu, v: 2 * v / b - orig(U, W, b, lu, v))
    lu = woodbury.factor(U, W, beta)
    y = woodbury.solve(U, W, beta, lu, v)
    ref = np.linalg.solve(beta * np.eye(n) + U @ W, v)
    assert np.abs(y - ref).max() > 1e-3


def test_unorthonormalised_laplacian_is_caught(monkeypatch):
    """Filtering with plain L instead of G^-1/2 L G^-1/2 breaks P G^1/2 1 = G^1/2 1."""
    m = geometry.mesh(wl.ellipse(100))
    from oracle import formulation
    Gh, Gmh, _ = formulation.gram_powers(*assembly.gram(m))
    monkeypatch.setattr(filters, "orthonormal_laplacian",
                        lambda m, Gmh=None: assembly.periodic_dense(*assembly.laplacian(m)))
    Vn, _, _ = filters.laplacian_filter(m, 21, Gmh=Gmh)
    null = Gh @ np.ones(m.n)
    assert np.abs(Vn @ (Vn.T @ null) - null).max() > 1e-6 * np.abs(null).max()
