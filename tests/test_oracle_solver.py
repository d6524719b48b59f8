"""Pins of the oracle's formulation, filter, compression and Woodbury stages."""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy import special as sp

from oracle import (assembly, compress, filters, formulation, geometry, rng, solver,
                    woodbury)
from paper_2210_08580_amd import workloads as wl


def exact_circle_u(k, a, theta, phi, M=60):
    """Total field of a plane wave on a sound-hard circle, from the Wronskian
    J_m H_m' - J_m' H_m = 2i/(pi x): u = sum_m i^m (2i/(pi k a)) / H_m'(ka) e^{im(theta-phi)}."""
    u = 0
    for m in range(-M, M + 1):
        u = u + (1j ** m) * (2j / (np.pi * k * a)) / sp.h1vp(m, k * a) * np.exp(1j * m * (theta - phi))
    return u


def _circle_ops(n, k, form="efie", n_modes=None):
    pb = solver.Problem(wl.circle(n), k, form=form, n_modes=n_modes or n, rank_cap=n)
    return pb, solver.build_operators(pb)


def test_calderon_circle_modes():
    """Discrete Z_e eigenvalues -> lam_S lam_N (Calderon SN = I/4 + compact)."""
    k = 1.0
    ms = np.arange(0, 9)
    x = k
    lS = 0.5j * np.pi * sp.jv(ms, x) * sp.hankel1(ms, x)
    lN = -0.5j * np.pi * k * k * sp.jvp(ms, x) * sp.h1vp(ms, x)
    errs = []
    for n in (64, 128):
        _, ops = _circle_ops(n, k)
        Z = ops.C + 0.25 * np.eye(n)
        th = 2 * np.pi * np.arange(n) / n
        E = np.exp(1j * np.outer(th, ms)) / np.sqrt(n)
        z = np.einsum("im,ij,jm->m", E.conj(), Z, E)
        errs.append(np.abs(z - lS * lN).max())
    assert errs[1] < 2e-3 and errs[0] / errs[1] > 3.3
    # the continuous symbols tend to 1/4 (compact perturbation)
    assert abs(lS[8] * lN[8] - 0.25) < 1e-6


@pytest.mark.parametrize("form", ["efie", "mfie", "cfie"])
def test_exact_circle_solution(form):
    k = 1.0
    ang = np.array([0.3, 2.0])
    amp = np.array([1.0, 0.5 - 0.2j])
    errs = []
    for n in (64, 128):
        _, ops = _circle_ops(n, k, form)
        f, h = assembly.rhs_planewave(ops.mesh, k, ang, amp)
        v = formulation.rhs_vector(form, ops.S, ops.Gmh, ops.Gi, f.T, h.T)
        j = ops.Gmh @ solver.y_unfiltered(ops, v)
        th = 2 * np.pi * np.arange(n) / n
        ue = np.stack([a * exact_circle_u(k, 1.0, th, p) for p, a in zip(ang, amp)], 1)
        errs.append(np.abs(j + ue).max() / np.abs(ue).max())
    assert errs[1] < 3e-4 and errs[0] / errs[1] > 3.5, errs


def test_efie_mfie_agree_on_star():
    k = 3.0
    n = 128
    js = []
    for form in ("efie", "mfie"):
        pb = solver.Problem(wl.star(n), k, form=form, n_modes=n, rank_cap=n)
        ops = solver.build_operators(pb)
        f, h = assembly.rhs_planewave(ops.mesh, k, [1.1], [1.0])
        v = formulation.rhs_vector(form, ops.S, ops.Gmh, ops.Gi, f.T, h.T)
        js.append(ops.Gmh @ solver.y_unfiltered(ops, v))
    assert np.abs(js[0] - js[1]).max() / np.abs(js[0]).max() < 5e-3


def test_gram_powers():
    m = geometry.mesh(wl.ellipse(80))
    G = assembly.periodic_dense(*assembly.gram(m))
    Gh, Gmh, Gi = formulation.gram_powers(*assembly.gram(m))
    I = np.eye(80)
    assert np.abs(Gh @ Gh - G).max() < 1e-15 * 10
    assert np.abs(Gmh @ Gh - I).max() < 1e-13
    assert np.abs(Gi @ G - I).max() < 1e-12


def test_filter_on_circle_is_fourier_projector():
    n, M = 96, 10
    m = geometry.mesh(wl.circle(n))
    Vn, lam, neff = filters.laplacian_filter(m, 2 * M + 1)
    assert neff == 2 * M + 1
    th = 2 * np.pi * np.arange(n) / n
    cols = [np.ones(n)] + [f(mm * th) for mm in range(1, M + 1) for f in (np.cos, np.sin)]
    F = np.stack(cols, 1)
    F /= np.linalg.norm(F, axis=0)
    assert np.abs(Vn @ Vn.T - F @ F.T).max() < 1e-12


def test_filter_projector_properties_and_cluster_guard():
    m = geometry.mesh(wl.star(120))
    Gh, Gmh, _ = formulation.gram_powers(*assembly.gram(m))
    Vn, lam, neff = filters.laplacian_filter(m, 21, Gmh=Gmh)
    P = Vn @ Vn.T
    assert np.abs(P @ P - P).max() < 1e-13 and np.abs(P - P.T).max() < 1e-15
    null = Gh @ np.ones(m.n)                    # null vector of G^-1/2 L G^-1/2
    assert np.abs(P @ null - null).max() < 1e-12 * np.abs(null).max()
    assert abs(np.trace(P) - neff) < 1e-11
    Lt = filters.orthonormal_laplacian(m, Gmh)
    assert np.abs(Lt @ Vn - Vn * lam).max() < 1e-9 * np.abs(lam).max()
    # literal reading drops the null mode
    V0, _, n0 = filters.laplacian_filter(m, 21, keep_nullspace=False, Gmh=Gmh)
    assert n0 == 20 and np.abs(V0.T @ null).max() < 1e-10 * np.linalg.norm(null)
    # an even cut splits a +-m pair on the circle: the guard closes the cluster
    mc = geometry.mesh(wl.circle(64))
    _, _, ne = filters.laplacian_filter(mc, 20)
    assert ne == 21


def test_full_filter_reduces_to_unfiltered():
    """n = N gives P = I, so (beta I + P C) is the unfiltered system Z."""
    pb, ops = _circle_ops(48, 1.5)
    assert np.abs(ops.Vn @ ops.Vn.T - np.eye(48)).max() < 1e-12
    v = np.random.default_rng(0).standard_normal((48, 2)) + 0j
    assert solver.relerr(solver.y_filtered(ops, v), solver.y_unfiltered(ops, v)) < 1e-12


def test_woodbury_matches_dense_lu():
    rs = np.random.default_rng(1)
    n, r, beta = 60, 9, 0.37
    U = rs.standard_normal((n, r)) + 1j * rs.standard_normal((n, r))
    W = (rs.standard_normal((r, n)) + 1j * rs.standard_normal((r, n))) * 0.1
    v = rs.standard_normal((n, 3)) + 1j * rs.standard_normal((n, 3))
    lu = woodbury.factor(U, W, beta)
    y = woodbury.solve(U, W, beta, lu, v)
    ref = sla.solve(beta * np.eye(n) + U @ W, v)
    assert solver.relerr(y, ref) < 1e-12


def test_woodbury_singular_core_detected():
    n = 20
    U = np.zeros((n, 2), complex)
    U[0, 0] = 1.0
    U[1, 1] = 1.0
    W = np.zeros((2, n), complex)
    W[0, 0] = -0.5          # beta + u w = 0 on the first direction
    W[1, 1] = 2.0
    with pytest.raises(woodbury.SingularCore):
        woodbury.factor(U, W, 0.5)


def _decaying(n, s, seed=0):
    rs = np.random.default_rng(seed)
    X = np.linalg.qr(rs.standard_normal((n, n)) + 1j * rs.standard_normal((n, n)))[0]
    Y = np.linalg.qr(rs.standard_normal((n, n)) + 1j * rs.standard_normal((n, n)))[0]
    return (X[:, :s.size] * s) @ Y[:, :s.size].conj().T


def test_compression_lossless_and_hmt_bound():
    n = 120
    s = 0.5 ** np.arange(40)
    A = _decaying(n, s)
    Om = rng.sketch(9, n, 50)
    U, W, sig = compress.compress(A, Om, power_iters=2, rank_cap=50, tol=0.0)
    assert np.abs(U @ W - A).max() < 1e-13          # rank 40 < l: lossless
    # lossy: spectral error within a modest factor of sigma_{r+1}
    Om = rng.sketch(9, n, 30)
    U, W, sig = compress.compress(A, Om, power_iters=2, rank_cap=20, tol=0.0)
    err = np.linalg.norm(U @ W - A, 2)
    assert U.shape[1] == 20 and err < 5.0 * s[20]
    # tolerance truncation: sigma_i > eps sigma_1
    U, W, sig = compress.compress(A, Om, power_iters=2, rank_cap=30, tol=1e-3)
    assert U.shape[1] == int(np.count_nonzero(s > 1e-3))


def test_truncation_never_splits_a_pair():
    s = np.array([1.0, 0.5, 0.5 * (1 + 1e-9), 0.1])
    s = np.sort(s)[::-1]
    assert compress.truncation_rank(s, 2, 0.0) == 1
    assert compress.truncation_rank(s, 3, 0.0) == 3


def test_pipeline_lossless_equals_filtered_solution():
    """Headline-style parameters at small N: r >= n makes the compression exact,
    so the Woodbury solve equals y_fil without refinement."""
    n = 160
    pb = solver.Problem(wl.star(n), 10.0, form="efie", n_modes=31, rank_cap=32,
                        oversample=4, power_iters=2, seed=7)
    ops = solver.build_operators(pb)
    ang, amp = wl.planewaves(1, 4)
    sol = solver.solve(pb, ops, ang, amp)
    yf = solver.y_filtered(ops, sol.v)
    assert sol.rank == ops.n_eff
    assert solver.relerr(sol.y_fast, yf) < 1e-11
    assert solver.relerr(sol.y, yf) < 1e-12


def test_pipeline_lossy_refinement_converges():
    n = 200
    pb = solver.Problem(wl.ellipse(n), 5.0, form="efie", n_modes=41, rank_cap=20,
                        oversample=6, power_iters=2, tol=0.0, seed=11,
                        refine_tol=1e-12, max_refine=30)
    ops = solver.build_operators(pb)
    ang, amp = wl.planewaves(3, 3)
    sol = solver.solve(pb, ops, ang, amp)
    yf = solver.y_filtered(ops, sol.v)
    assert sol.rank == 20
    assert solver.relerr(sol.y_fast, yf) > 1e-6         # compression is lossy
    assert solver.relerr(sol.y, yf) < 1e-11             # refinement recovers y_fil
    assert sol.history[-1] <= 1e-12
