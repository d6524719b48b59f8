"""Seeded synthetic inputs shared by the tests, the bench and the oracle checks.

This module holds only input generation: closed curves sampled at nodes, wave
numbers, plane-wave directions and amplitudes. It contains none of the solver's
arithmetic (no panels, quadrature, kernels or linear algebra), so both the HIP
path and the CPU oracle can take their inputs from it without sharing code.

Curves are shaped like the paper's scatterers (Numerical Results: an ellipse
and a perturbed circle r = 2 + 0.2 sin 8t) and like the star / random smooth
curves of the benchmark configurations. Nodes sit at t_i = 2*pi*i/N on each
parametrised curve, counter-clockwise, so the mesh is non-uniform in arc length
whenever the curve is not a circle (the paper's Laplacian-filter section
assumes non-homogeneous meshes).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Workload", "curve_nodes", "circle", "star", "ellipse", "perturbed_circle",
    "random_polar", "random_coeffs", "random_curve", "curve_trig", "planewaves", "workload",
]


def _polar(r: np.ndarray, t: np.ndarray) -> np.ndarray:
    return np.stack([r * np.cos(t), r * np.sin(t)], axis=1)


def _params(n: int) -> np.ndarray:
    return 2.0 * math.pi * np.arange(n, dtype=np.float64) / n


def circle(n: int, radius: float = 1.0) -> np.ndarray:
    t = _params(n)
    return _polar(np.full(n, radius), t)


def star(n: int, amp: float = 0.3, lobes: int = 5) -> np.ndarray:
    """r(t) = 1 + amp cos(lobes t)."""
    t = _params(n)
    return _polar(1.0 + amp * np.cos(lobes * t), t)


def ellipse(n: int, a: float = 2.0, b: float = 0.5) -> np.ndarray:
    t = _params(n)
    return np.stack([a * np.cos(t), b * np.sin(t)], axis=1)


def perturbed_circle(n: int) -> np.ndarray:
    """The paper's Table I scatterer, r(t) = 2 + 0.2 sin 8t."""
    t = _params(n)
    return _polar(2.0 + 0.2 * np.sin(8.0 * t), t)


def random_polar(n: int, coeffs: np.ndarray, base: float = 1.0,
                 star_amp: float = 0.0) -> np.ndarray:
    """r(t) = base + star_amp cos 5t + sum_m a_m cos(m t) + b_m sin(m t).

    ``coeffs`` has shape (M, 2): row m-1 holds (a_m, b_m)."""
    t = _params(n)
    r = np.full(n, base) + star_amp * np.cos(5.0 * t)
    for m in range(1, coeffs.shape[0] + 1):
        r = r + coeffs[m - 1, 0] * np.cos(m * t) + coeffs[m - 1, 1] * np.sin(m * t)
    return _polar(r, t)


def random_coeffs(seed: int, modes: int = 16, scale: float = 0.1,
                  min_radius: float = 0.3, base: float = 1.0) -> np.ndarray:
    """a_m, b_m ~ N(0, (scale/m)^2); redrawn until min r >= min_radius."""
    rng = np.random.default_rng(seed)
    m = np.arange(1, modes + 1, dtype=np.float64)
    t = _params(4096)
    while True:
        c = rng.standard_normal((modes, 2)) * (scale / m)[:, None]
        r = base + sum(c[i, 0] * np.cos((i + 1) * t) + c[i, 1] * np.sin((i + 1) * t)
                       for i in range(modes))
        if r.min() >= min_radius:
            return c


def random_curve(n: int, seed: int = 1000) -> np.ndarray:
    """A smooth random curve: random_polar with random_coeffs(seed)."""
    return random_polar(n, random_coeffs(seed))


def curve_nodes(kind: str, n: int, **kw) -> np.ndarray:
    fn = {"circle": circle, "star": star, "ellipse": ellipse,
          "perturbed_circle": perturbed_circle, "random": random_curve}[kind]
    return np.ascontiguousarray(fn(n, **kw), dtype=np.float64)


def curve_trig(kind: str, degree: int = 24, **kw):
    """The same curve as curve_nodes(kind) as a trigonometric polynomial in
    Cartesian form, x(t) = sum_m ax[m] cos(m t) + bx[m] sin(m t) (y likewise),
    m = 0 .. degree: every curve here is one (degree 1 for the circle and the
    ellipse, 6 for the star, 9 for the perturbed circle, 17 for the random curves).
    Coefficients from the DFT of 4 (degree + 1) samples, entries below 1e-14 of the
    largest set to zero. Returns (ax, bx, ay, by)."""
    K = 4 * (degree + 1)
    pts = curve_nodes(kind, K, **kw)
    out = []
    for col in (0, 1):
        X = np.fft.rfft(pts[:, col]) / K
        a = 2.0 * X.real[:degree + 1]
        b = -2.0 * X.imag[:degree + 1]
        a[0] *= 0.5
        b[0] = 0.0
        out += [a, b]
    big = max(np.abs(v).max() for v in out)
    return tuple(np.where(np.abs(v) < 1e-14 * big, 0.0, v) for v in out)


def planewaves(seed: int, nrhs: int):
    """Seeded plane-wave directions phi ~ U[0, 2pi) and unit amplitudes."""
    rng = np.random.default_rng(seed)
    angles = rng.uniform(0.0, 2.0 * math.pi, size=nrhs)
    amps = np.ones(nrhs, dtype=np.complex128)
    return angles.astype(np.float64), amps


def random_amplitudes(seed: int, nrhs: int) -> np.ndarray:
    """Complex amplitudes ~ CN(0, 1)."""
    rng = np.random.default_rng(seed)
    return ((rng.standard_normal(nrhs) + 1j * rng.standard_normal(nrhs))
            / math.sqrt(2.0)).astype(np.complex128)


@dataclasses.dataclass
class Workload:
    """One solver configuration: geometry, wave number, formulation and sizes."""
    name: str
    nodes: np.ndarray
    k: float
    form: str = "efie"          # efie | mfie | cfie
    alpha: float = 1.0          # CFIE combination weight
    n_modes: int = 21           # filtering point n (number of kept Laplacian modes)
    rank_cap: int = 32
    oversample: int = 0
    power_iters: int = 0
    tol: float = 0.0
    seed: int = 0               # sketch seed
    angles: np.ndarray = None
    amps: np.ndarray = None
    # equal-chord workloads: nodes is None; the caller meshes the curve `trig`
    # (curve_trig coefficients) with n_nodes equal chords
    trig: tuple = None
    n_nodes: int = 0

    @property
    def n(self) -> int:
        return int(self.nodes.shape[0]) if self.nodes is not None else int(self.n_nodes)

    @property
    def nrhs(self) -> int:
        return int(self.angles.shape[0])


def workload(name: str, n: int | None = None, nrhs: int | None = None,
             form: str | None = None) -> Workload:
    """Named configurations.

    circle256   unit circle, k=1, EFIE, n=21 kept modes (M=10), rank cap 32, 8 RHS
    star4096    star r=1+0.3cos5t, k=10, n=255 (M=127), r=256, p=10, q=2, 256 RHS
    star8192    the same star at N=8192 (the throughput workload)
    star8192ec  the same star and parameters on an equal-chord (homogeneous) mesh of
                N=8192 nodes: nodes is None, the caller meshes w.trig
    ellipse16384  ellipse 2 x 0.5, k=5, n=511, r=128 (lossy), p=10, q=2, 1024 RHS
    """
    if name == "circle256":
        N = n or 256
        ang, amp = planewaves(0, nrhs or 8)
        return Workload(name, circle(N), 1.0, form or "efie", 1.0, 21, 32, 0, 0,
                        0.0, 0, ang, amp)
    if name in ("star4096", "star8192"):
        N = n or (4096 if name == "star4096" else 8192)
        ang, amp = planewaves(1 if name == "star4096" else 2, nrhs or 256)
        return Workload(name, star(N), 10.0, form or "efie", 1.0, 255, 256, 10, 2,
                        0.0, 7, ang, amp)
    if name == "star8192ec":
        N = n or 8192
        ang, amp = planewaves(2, nrhs or 256)
        return Workload(name, None, 10.0, form or "efie", 1.0, 255, 256, 10, 2,
                        0.0, 7, ang, amp, curve_trig("star"), N)
    if name == "ellipse16384":
        N = n or 16384
        ang, amp = planewaves(3, nrhs or 1024)
        return Workload(name, ellipse(N), 5.0, form or "efie", 1.0, 511, 128, 10, 2,
                        1e-8, 11, ang, amp)
    raise KeyError(name)
