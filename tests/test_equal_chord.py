"""Equal-chord (homogeneous) meshes and the Laplacian filter on them (CPU).

Paper, Laplacian Filters, Two-Dimensional Case: on a homogeneously discretised
curve the filter is diagonalised by the DFT, so it needs no eigensolver. The
oracle mesher is pinned by the circle (equal chords <=> equal angles) and by the
chord lengths themselves; the oracle filter and Gram powers on such meshes are
pinned by the DFT closed forms; the library's host mesher (C ABI, no GPU) is
checked against the oracle mesher."""
import numpy as np
import pytest

from oracle import assembly, filters, formulation, geometry
from paper_2210_08580_amd import binding as B
from paper_2210_08580_amd import workloads as wl


def _chords(nodes):
    return np.hypot(*(np.roll(nodes, -1, axis=0) - nodes).T)


def test_trig_curves_match_sampled_curves():
    for kind in ("circle", "star", "ellipse", "perturbed_circle", "random"):
        tr = wl.curve_trig(kind)
        t = 2 * np.pi * np.arange(29) / 29
        assert np.abs(geometry.trig_point(tr, t) - wl.curve_nodes(kind, 29)).max() < 1e-14


def test_oracle_mesher_circle_closed_form():
    # on a circle equal chords are equal central angles: t_i = 2 pi i / n
    for n in (5, 16, 77):
        t, c = geometry.equal_chord_params(wl.curve_trig("circle"), n)
        assert np.abs(t - 2 * np.pi * np.arange(n) / n).max() < 1e-13
        assert abs(c - 2 * np.sin(np.pi / n)) < 1e-14


@pytest.mark.parametrize("kind,n", [("star", 64), ("ellipse", 101), ("random", 80), ("perturbed_circle", 120)])
def test_oracle_mesher_equal_chords(kind, n):
    tr = wl.curve_trig(kind)
    t, c = geometry.equal_chord_params(tr, n)
    assert t[0] == 0.0 and np.all(np.diff(t) > 0) and t[-1] < 2 * np.pi
    h = _chords(geometry.trig_point(tr, t))
    assert np.abs(h - c).max() <= 2e-13 * c
    assert geometry.signed_area(geometry.trig_point(tr, t)) > 0


@pytest.mark.parametrize("kind,n", [("star", 64), ("ellipse", 101), ("random", 80), ("circle", 33)])
def test_native_mesher_matches_oracle(kind, n):
    tr = wl.curve_trig(kind)
    nodes, c = B.fds_equal_chord_nodes(tr, n)
    ref = geometry.equal_chord_nodes(tr, n)
    assert np.abs(nodes - ref).max() <= 1e-12
    h = _chords(nodes)
    assert np.abs(h - c).max() <= 1e-13 * c


def test_native_mesher_errors():
    tr = wl.curve_trig("star")
    with pytest.raises(B.FdsError):
        B.fds_equal_chord_nodes(tr, 3)
    z = tuple(np.zeros(3) for _ in range(4))
    with pytest.raises(B.FdsError):
        B.fds_equal_chord_nodes(z, 16)


def _dft_mu(n, h):
    m = np.arange(n)
    return 12 * np.sin(np.pi * m / n) ** 2 / (h * h * (2 + np.cos(2 * np.pi * m / n)))


@pytest.mark.parametrize("kind,n", [("star", 160), ("ellipse", 121)])
def test_oracle_filter_is_dft_on_equal_chords(kind, n):
    """The oracle's dense eigensolver reproduces the DFT closed form: eigenvalues
    12 sin^2(pi m/n) / (h^2 (2 + cos(2 pi m/n))) and the subspace of the lowest
    frequencies."""
    nodes = geometry.equal_chord_nodes(wl.curve_trig(kind), n)
    m = geometry.mesh(nodes)
    h = m.h.mean()
    assert np.ptp(m.h) <= 1e-12 * h
    nm = 41
    V, lam, ne = filters.laplacian_filter(m, nm, True, 1e-6)
    assert ne == nm                          # 0 and 20 (cos, sin) pairs: no split pair
    mu = np.sort(_dft_mu(n, h))
    Lt = filters.orthonormal_laplacian(m)
    assert np.abs(lam[:ne] - mu[:ne]).max() <= 1e-10 * mu[ne - 1]
    lam_all = np.linalg.eigvalsh(Lt)
    assert np.abs(lam_all - mu).max() <= 1e-9 * mu.max()
    # DFT basis of the kept frequencies (|m| <= 20), orthonormal in the plain inner product
    j = np.arange(n)
    cols = [np.ones(n)]
    for k in range(1, 21):
        cols += [np.cos(2 * np.pi * k * j / n), np.sin(2 * np.pi * k * j / n)]
    F = np.stack(cols, axis=1)
    F /= np.linalg.norm(F, axis=0)
    assert np.abs(V @ V.T - F @ F.T).max() <= 1e-10


def test_oracle_gram_powers_are_dft_circulants():
    """G^{+-1/2} of an equal-chord mesh are the circulants with first rows
    ifft(lambda^{+-1/2}), lambda_m = (h/3)(2 + cos(2 pi m/n))."""
    n = 150
    m = geometry.mesh(geometry.equal_chord_nodes(wl.curve_trig("random"), n))
    Gh, Gmh, Gi = formulation.gram_powers(*assembly.gram(m))
    lam = (m.h.mean() / 3) * (2 + np.cos(2 * np.pi * np.arange(n) / n))
    for p, R in ((1, Gh), (-1, Gmh), (-2, Gi)):
        row = np.fft.ifft(lam ** (p / 2)).real
        C = np.stack([np.roll(row, i) for i in range(n)])
        assert np.abs(R - C).max() <= 1e-12 * np.abs(R).max(), p
