"""GPU parity of the mixed-precision path: the FP32 Bessel evaluator, complex64
GEMM on the FP32 matrix cores, FP32 far-field assembly (complex64 operators)
and the whole solve, whose FP64 refinement must land within 1e-6 of the FP64
oracle's filtered solution."""
import numpy as np
import pytest
import scipy.special as sp
import torch

from oracle import assembly, formulation, geometry, solver
from paper_2210_08580_amd import binding as B
from paper_2210_08580_amd import workloads as wl

pytestmark = pytest.mark.gpu
EPS32 = float(np.finfo(np.float32).eps)


@pytest.fixture(scope="module")
def ctx():
    c = B.fds_ctx_create(0)
    yield c
    c.close()


def test_hankel_f32_accuracy(ctx):
    print("case: hankel fp32", flush=True)
    x = np.concatenate([np.geomspace(1e-4, 2.0, 2000, endpoint=False), np.linspace(2.0, 25.0, 20000,
                        endpoint=False), np.linspace(25.0, 400.0, 5000)])
    got = B.fds_hankel_eval_f32(ctx, torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    ref = np.stack([sp.j0(x), sp.y0(x), sp.j1(x), sp.y1(x)], axis=1)
    err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
    assert err.max() <= 4e-7, err.max()


@pytest.mark.parametrize("opa,opb", [(0, 0), (1, 0), (2, 0), (0, 1), (0, 2), (2, 2)])
@pytest.mark.parametrize("m,n,k", [(70, 33, 129), (40, 40, 3000), (128, 64, 64), (1, 65, 17)])
def test_cgemm_parity(ctx, opa, opb, m, n, k):
    print(f"case: cgemm op=({opa},{opb}) m={m} n={n} k={k}", flush=True)
    rs = np.random.default_rng(m + 3 * n + 7 * k + 11 * opa + opb)

    def cr(shape):
        return (rs.standard_normal(shape) + 1j * rs.standard_normal(shape)).astype(np.complex64)
    A = cr((m, k) if opa == 0 else (k, m))
    Bm = cr((k, n) if opb == 0 else (n, k))
    C0 = cr((m, n))
    alpha, beta = 0.7 - 0.2j, -0.3 + 0.5j

    def op(X, o):
        X = X.astype(np.complex128)
        return X if o == 0 else (X.T if o == 1 else X.conj().T)
    ref = alpha * op(A, opa) @ op(Bm, opb) + beta * C0.astype(np.complex128)
    tA = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
    tB = torch.from_numpy(np.ascontiguousarray(Bm.T)).cuda()
    tC = torch.from_numpy(np.ascontiguousarray(C0.T)).cuda()
    B.fds_cgemm(ctx, opa, opb, tA, tB, tC, alpha, beta)
    got = tC.cpu().numpy().T.astype(np.complex128)
    scale = np.abs(A).max() * np.abs(Bm).max() * k
    assert np.abs(got - ref).max() <= 8 * EPS32 * scale


ASM_CASES = [("star", 300, 10.0, 0), ("ellipse", 257, 5.0, 0), ("circle", 64, 1.0, 0), ("random", 400, 20.0, 0),
             ("star", 190, 10.0, 0), ("star", 40, 3.0, 0),
             # band widths around the runs of 8 offsets and the row blocks of 63 panels
             ("ellipse", 127, 4.0, 0), ("random", 130, 6.0, 0), ("star", 64, 2.0, 0),
             ("star", 600, 10.0, 127), ("ellipse", 301, 5.0, 100), ("random", 200, 3.0, 5), ("circle", 9, 1.0, 0)]


@pytest.mark.parametrize("kind,n,k,bw", ASM_CASES)
def test_fp32_assembly_parity(ctx, kind, n, k, bw):
    print(f"case: fp32 assembly {kind} n={n} k={k} band_width={bw}", flush=True)
    nodes = wl.curve_nodes(kind, n)
    op = B.fds_assemble(ctx, torch.from_numpy(nodes).cuda(), k, precision="fp32", band_width=bw)
    assert B.fds_op_precision(op) == B.FDS_FP32
    got = [t.cpu().numpy().astype(np.complex128) for t in B.fds_op_matrices(op)]
    # N near the diagonal is kept in complex128 beside zeros in the complex64 matrix
    band, w = B.fds_op_nband(op)
    band = band.cpu().numpy()
    assert w == min(bw if bw > 0 else 63, (n - 1) // 2)
    i = np.arange(n)
    ref = assembly.assemble(geometry.mesh(nodes), k)
    smax = np.abs(ref[0]).max()
    for d in range(-w, w + 1):
        j = (i + d) % n
        assert np.all(got[1][i, j] == 0)
        got[1][i, j] = band[:, d + w]
        # the band is FP64: same tolerance as the FP64 assembly parity
        assert np.abs(band[:, d + w] - ref[1][i, j]).max() <= 1e-12 * np.abs(ref[1]).max()
        # S there: FP64 values rounded to complex64 (twice on |d| <= 2, where the
        # near-pair blocks are added to the stored far part)
        assert np.all(np.abs(got[0][i, j] - ref[0][i, j]) <= 2.5e-7 * np.abs(ref[0][i, j]) + 1e-13 * smax)
    for name, g, r in zip("SND", got, ref):
        err = np.abs(g - r).max() / np.abs(r).max()
        assert err <= 2e-6, (name, err)
    op.close()


MIXED_CASES = [("star", 600, 10.0, "efie", 63), ("ellipse", 350, 5.0, "cfie", 51),
               ("circle", 256, 1.0, "mfie", 21), ("random", 500, 8.0, "efie", 41),
               ("star", 2048, 10.0, "efie", 127)]


@pytest.mark.parametrize("kind,n,k,form,nm", MIXED_CASES)
def test_mixed_solve_parity(ctx, kind, n, k, form, nm):
    print(f"case: mixed solve {kind} n={n} k={k} {form} n_modes={nm}", flush=True)
    nodes = wl.curve_nodes(kind, n)
    ang, _ = wl.planewaves(5, 8)
    amps = wl.random_amplitudes(6, 8)
    op = B.fds_assemble(ctx, torch.from_numpy(nodes).cuda(), k, precision="fp32")
    ne = B.fds_filter(op, form, 1.0, nm)
    B.fds_compress(op, rank_cap=ne + 1, oversample=10, power_iters=2, seed=7)
    B.fds_factor(op)
    f, h = B.fds_rhs_planewave(op, torch.from_numpy(ang), torch.from_numpy(amps))
    j, y, st = B.fds_solve(op, f, h, max_iters=4, tol=1e-12, want_y=True)
    assert st["converged"], st
    pb = solver.Problem(nodes, k, form=form, n_modes=nm, rank_cap=ne + 1)
    ops = solver.build_operators(pb)
    assert ops.n_eff == ne
    fo, ho = assembly.rhs_planewave(geometry.mesh(nodes), k, ang, amps)
    v = formulation.rhs_vector(form, ops.S, ops.Gmh, ops.Gi, fo.T, ho.T)
    err = solver.relerr(y.cpu().numpy().T, solver.y_filtered(ops, v))
    assert err <= 1e-6, err
    op.close()
