"""Pins of the oracle's far field, objective and adjoint gradient (CPU only)."""
import numpy as np
import scipy.special as sp

from oracle import adjoint, assembly, geometry
from paper_2210_08580_amd import workloads as wl


def _farfield_circle_exact(k, a, thetas, phi, mmax=60):
    """Sound-hard circle: u_inf = -sqrt(2/(pi k)) e^{-i pi/4} sum_m J'_m(ka)/H'_m(ka) e^{im(theta-phi)}."""
    x = k * a
    m = np.arange(-mmax, mmax + 1)
    ratio = sp.jvp(m, x) / sp.h1vp(m, x)
    return -np.sqrt(2.0 / (np.pi * k)) * np.exp(-0.25j * np.pi) * np.array(
        [np.sum(ratio * np.exp(1j * m * (t - phi))) for t in thetas])


def test_farfield_circle_closed_form():
    k, a, phi = 3.0, 1.0, 0.4
    thetas = np.linspace(0.0, 2 * np.pi, 13, endpoint=False)
    ref = _farfield_circle_exact(k, a, thetas, phi)
    errs = []
    for n in (128, 256):
        _, FJ = adjoint.forward(wl.circle(n), k, [phi], [1.0], thetas)
        errs.append(np.abs(FJ[:, 0] - ref).max() / np.abs(ref).max())
    assert errs[1] < 2e-4
    assert errs[0] / errs[1] > 3.0          # second-order convergence in h


def test_farfield_reciprocity():
    """u_inf(theta; d) = u_inf(-d; -theta): exact for the Galerkin model (N symmetric)."""
    k = 4.0
    nodes = wl.curve_nodes("random", 96)
    t1, t2 = 0.7, 2.9
    _, A = adjoint.forward(nodes, k, [t1], [1.0], [t2])
    _, B = adjoint.forward(nodes, k, [t2 + np.pi], [1.0], [t1 + np.pi])
    assert abs(A[0, 0] - B[0, 0]) <= 1e-12 * abs(A[0, 0])


def _problem(n=48, nrhs=3, nang=20, seed=5):
    rs = np.random.default_rng(seed)
    nodes = wl.curve_nodes("random", n)
    angles = rs.uniform(0, 2 * np.pi, nrhs)
    amps = (rs.standard_normal(nrhs) + 1j * rs.standard_normal(nrhs)) / np.sqrt(2)
    thetas = 2 * np.pi * np.arange(nang) / nang
    T = 0.1 * (rs.standard_normal((nang, nrhs)) + 1j * rs.standard_normal((nang, nrhs)))
    return nodes, 3.0, angles, amps, thetas, T


def test_adjoint_gradient_vs_objective_fd():
    nodes, k, angles, amps, thetas, T = _problem()
    J, g, ga = adjoint.gradient(nodes, k, angles, amps, thetas, T)
    assert abs(J - adjoint.objective(nodes, k, angles, amps, thetas, T)) <= 1e-12 * J
    rs = np.random.default_rng(9)
    h = 1e-6 * np.mean(geometry.mesh(nodes).h)
    for _ in range(3):
        dirn = rs.standard_normal(nodes.shape)
        fd = (adjoint.objective(nodes + h * dirn, k, angles, amps, thetas, T)
              - adjoint.objective(nodes - h * dirn, k, angles, amps, thetas, T)) / (2 * h)
        assert abs(fd - np.sum(g * dirn)) <= 2e-6 * np.abs(g).sum()


def _objective_derivative(nodes, k, angles, amps, thetas, T, dirn, h):
    """d/dt J(nodes + t dirn) at t = 0 by Richardson extrapolation of central
    differences of the objective itself (dense LU solves; no adjoint, no dN)."""
    def J(t):
        return adjoint.objective(nodes + t * dirn, k, angles, amps, thetas, T)
    d1 = (J(h) - J(-h)) / (2 * h)
    d2 = (J(2 * h) - J(-2 * h)) / (4 * h)
    return (4 * d1 - d2) / 3


def test_adjoint_gradient_to_1e10():
    """The adjoint gradient with differentiated operators against the derivative
    of the objective along smooth and random directions, both to fourth order:
    agreement to 1e-10 of the directional derivative's scale."""
    nodes, k, angles, amps, thetas, T = _problem(n=40)
    _, g, _ = adjoint.gradient(nodes, k, angles, amps, thetas, T)
    n = nodes.shape[0]
    t = 2 * np.pi * np.arange(n) / n
    rs = np.random.default_rng(13)
    h = 1e-3 * np.mean(geometry.mesh(nodes).h)
    dirs = [np.stack([np.cos(t), np.sin(t)], 1) * np.cos(3 * t)[:, None], rs.standard_normal(nodes.shape)]
    for dirn in dirs:
        fd = _objective_derivative(nodes, k, angles, amps, thetas, T, dirn, h)
        an = float(np.sum(g * dirn))
        scale = float(np.sum(np.abs(g * dirn)))
        assert abs(fd - an) <= 1e-10 * scale, (fd, an, scale)


def test_amplitude_gradient_closed_form_vs_fd():
    nodes, k, angles, amps, thetas, T = _problem(n=40)
    _, _, ga = adjoint.gradient(nodes, k, angles, amps, thetas, T, rel_step=1e-3)
    h = 1e-6
    for r in range(len(amps)):
        for unit, part in ((1.0, np.real), (1j, np.imag)):
            ap, am = amps.copy(), amps.copy()
            ap[r] += h * unit
            am[r] -= h * unit
            fd = (adjoint.objective(nodes, k, angles, ap, thetas, T)
                  - adjoint.objective(nodes, k, angles, am, thetas, T)) / (2 * h)
            assert abs(fd - part(ga[r])) <= 1e-6 * np.abs(ga).max()
