"""GPU parity of the Laplacian filter on equal-chord (homogeneous) meshes,
where the library builds the filter from the DFT in closed form and applies
G^{+-1/2} as circulant bands (paper, Laplacian Filters, Two-Dimensional Case),
against the CPU oracle's dense eigensolver and dense Gram powers on the same
meshes (made by the oracle mesher)."""
import numpy as np
import pytest
import torch

from oracle import assembly, filters, formulation, geometry, solver
from paper_2210_08580_amd import binding as B
from paper_2210_08580_amd import workloads as wl

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = B.fds_ctx_create(0)
    yield c
    c.close()


def _ec(kind, n):
    nodes = geometry.equal_chord_nodes(wl.curve_trig(kind), n)
    return np.ascontiguousarray(nodes), geometry.mesh(nodes)


# n even and odd (an even n has the single mode m = n/2); n_modes even (the cut
# guard takes the partner of the split pair); the null mode dropped; almost all modes
FILTER_CASES = [("star", 300, 10.0, 41, True), ("ellipse", 301, 5.0, 40, True),
                ("random", 258, 2.0, 31, False), ("star", 130, 3.0, 129, True), ("star", 64, 3.0, 64, True)]


@pytest.mark.parametrize("kind,n,k,nm,keep", FILTER_CASES)
def test_dft_filter_parity(ctx, kind, n, k, nm, keep):
    _say(f"case: dft filter {kind} n={n} n_modes={nm} keep={keep}")
    nodes, m = _ec(kind, n)
    op = B.fds_assemble(ctx, torch.from_numpy(nodes).cuda(), k)
    B.fds_profile_enable(ctx, True)
    B.fds_profile_read(ctx)
    ne = B.fds_filter(op, "efie", 1.0, nm, keep_nullspace=keep)
    prof = B.fds_profile_read(ctx)
    B.fds_profile_enable(ctx, False)
    assert "filter_dft" in prof and "filter_bisect" not in prof, sorted(prof)
    Vn = B.fds_op_filter_basis(op).cpu().numpy().T
    Gh, Gmh, _ = formulation.gram_powers(*assembly.gram(m))
    Vo, lam, neo = filters.laplacian_filter(m, nm, keep, 1e-6, Gmh)
    assert ne == neo
    lam_all = np.linalg.eigvalsh(filters.orthonormal_laplacian(m, Gmh))
    s0 = 0 if keep else 1
    if s0 + ne < n:
        gap = lam_all[s0 + ne] - lam_all[s0 + ne - 1]
        tol = max(1e-12, 64 * EPS * lam_all[-1] / gap)
    else:
        tol = 1e-12
    assert np.abs(Vn @ Vn.T - Vo @ Vo.T).max() <= tol
    assert np.abs(Vn.T @ Vn - np.eye(ne)).max() < 1e-12
    lam_gpu = np.array(B.fds_op_filter_eigenvalues(op)[:ne])
    assert np.abs(lam_gpu - lam[:ne]).max() <= 64 * EPS * lam_all[-1] + 1e-12 * np.abs(lam[:ne]).max()
    op.close()


# n > 256: circulant bands; n <= 256: the Chebyshev series (the band would wrap)
GRAM_CASES = [("star", 300), ("ellipse", 513), ("random", 200)]


@pytest.mark.parametrize("kind,n", GRAM_CASES)
def test_dft_gram_powers_parity(ctx, kind, n):
    _say(f"case: dft gram powers {kind} n={n}")
    nodes, m = _ec(kind, n)
    op = B.fds_assemble(ctx, torch.from_numpy(nodes).cuda(), 4.0)
    Gh, Gmh, Gi = formulation.gram_powers(*assembly.gram(m))
    rs = np.random.default_rng(3)
    X = rs.standard_normal((4, n)) + 1j * rs.standard_normal((4, n))
    for p, R in ((-2, Gi), (-1, Gmh), (1, Gh)):
        t = torch.from_numpy(X.copy()).cuda()
        B.fds_apply_gram(op, p, t)
        ref = (R @ X.T).T
        err = np.abs(t.cpu().numpy() - ref).max() / np.abs(ref).max()
        assert err < 1e-13, (p, err)
    op.close()


SOLVE_CASES = [("star", 400, 10.0, "efie", 41, "fp64"), ("ellipse", 301, 5.0, "cfie", 31, "fp64"),
               ("random", 300, 3.0, "ycfie", 31, "fp64"), ("star", 400, 10.0, "cfie", 41, "fp32")]


@pytest.mark.parametrize("kind,n,k,form,nm,prec", SOLVE_CASES)
def test_dft_filter_solve_parity(ctx, kind, n, k, form, nm, prec):
    _say(f"case: dft solve {kind} n={n} k={k} {form} n_modes={nm} {prec}")
    nodes, m = _ec(kind, n)
    ang, _ = wl.planewaves(11, 5)
    amps = wl.random_amplitudes(12, 5)
    op = B.fds_assemble(ctx, torch.from_numpy(nodes).cuda(), k, precision=prec)
    f, h = B.fds_rhs_planewave(op, torch.from_numpy(ang), torch.from_numpy(amps))
    ne = B.fds_filter(op, form, 1.0, nm)
    B.fds_compress(op, rank_cap=ne + 1, oversample=10, power_iters=2, seed=7)
    B.fds_factor(op)
    j, y, st = B.fds_solve(op, f, h, max_iters=8, tol=1e-12, want_y=True)
    assert st["converged"], st
    pb = solver.Problem(nodes, k, form=form, n_modes=nm, rank_cap=ne + 1, oversample=10, power_iters=2, seed=7)
    ops = solver.build_operators(pb)
    assert ops.n_eff == ne
    fo, ho = assembly.rhs_planewave(m, k, ang, amps)
    v = formulation.rhs_vector(form, ops.S, ops.Gmh, ops.Gi, fo.T, ho.T, 1.0, ops.Sy)
    yf = solver.y_filtered(ops, v)
    tol = 1e-10 if prec == "fp64" else 1e-6
    ey, ej = solver.relerr(y.cpu().numpy().T, yf), solver.relerr(j.cpu().numpy().T, ops.Gmh @ yf)
    _say(f"  y vs y_fil {ey:.2e}, j vs j_fil {ej:.2e} (bound {tol:g})")
    assert ey <= tol and ej <= tol
    op.close()


def test_native_mesher_feeds_the_pipeline(ctx):
    """Nodes from the library's host mesher are recognised as homogeneous."""
    _say("case: native mesher -> dft filter")
    nodes, _ = B.fds_equal_chord_nodes(wl.curve_trig("star"), 2048)
    op = B.fds_assemble(ctx, torch.from_numpy(nodes).cuda(), 10.0)
    B.fds_profile_enable(ctx, True)
    B.fds_profile_read(ctx)
    ne = B.fds_filter(op, "efie", 1.0, 101)
    prof = B.fds_profile_read(ctx)
    B.fds_profile_enable(ctx, False)
    assert ne == 101 and "filter_dft" in prof
    Vn = B.fds_op_filter_basis(op)
    assert (Vn @ Vn.T - torch.eye(ne, dtype=Vn.dtype, device=Vn.device)).abs().max().item() < 1e-12
    op.close()
