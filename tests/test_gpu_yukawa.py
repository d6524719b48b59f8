"""GPU parity of the Yukawa-Calderon TE-CFIE (the CFIE with the Calderon single
layer at the imaginary wavenumber i k, kernel (1/2 pi) K0(k R)) against the CPU
oracle, through the C ABI: the K0 kernel values, the assembled Yukawa single
layer, and the filtered fast direct solve."""
import numpy as np
import pytest
import torch

from oracle import assembly, formulation, geometry, solver, special
from paper_2210_08580_amd import binding as B
from paper_2210_08580_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = B.fds_ctx_create(0)
    yield c
    c.close()


@pytest.mark.parametrize("kappa", [0.5, 5.0, 20.0])
def test_yukawa_eval_parity(ctx, kappa):
    _say(f"case: yukawa_eval kappa={kappa}")
    R = np.concatenate([[0.0], np.geomspace(1e-7, 60.0 / kappa, 4000)])
    out = B.fds_yukawa_eval(ctx, kappa, torch.from_numpy(R)).cpu().numpy()
    ref = special.yukawa(kappa, R[1:])
    assert out[0, 0] == 0.0
    # scipy's K0 (the oracle's) is itself good to about 1.2e-15 relative; the
    # device tables to 6e-16 (checked against mpmath when they are generated)
    assert np.all(np.abs(out[1:, 0] - ref) <= 4e-15 * np.abs(ref) + 1e-300), \
        np.max(np.abs(out[1:, 0] - ref) / np.abs(ref))
    reg = special.yukawa_reg(kappa, R)
    # the oracle forms K0/2pi + log(R)/2pi directly: its rounding is that of the
    # larger of the two terms, which cancel as R -> 0
    terms = np.maximum(np.abs(np.log(np.where(R > 0, R, 1.0))) / (2 * np.pi),
                       np.abs(np.concatenate([[0.0], ref])))
    assert np.all(np.abs(out[:, 1] - reg) <= 4e-15 * np.maximum(terms, 1.0))


# n = 16, 46, 151 leave one entry in the last 15-wide tile (the tile classes of
# the assembly meet at the wrap-around); k = 60 on the star takes most
# arguments k R past the table into the asymptotic range; k = 1 on the unit
# circle keeps every argument in the series range.
YUK_CASES = [("circle", 64, 1.0), ("star", 200, 10.0), ("ellipse", 257, 5.0), ("random", 131, 2.0),
             ("ellipse", 16, 2.0), ("circle", 46, 3.0), ("random", 151, 7.0), ("star", 300, 60.0)]


@pytest.mark.parametrize("kind,n,k", YUK_CASES)
def test_yukawa_operator_parity(ctx, kind, n, k):
    _say(f"case: yukawa operator {kind} n={n} k={k}")
    nodes = wl.curve_nodes(kind, n)
    m = geometry.mesh(nodes)
    Sy_o = assembly.assemble_yukawa(m, k)
    op = B.fds_assemble(ctx, torch.from_numpy(nodes).cuda(), k)
    assert B.fds_op_yukawa(op) is None
    f, h = B.fds_rhs_planewave(op, torch.zeros(1, dtype=torch.float64), torch.ones(1, dtype=torch.complex128))
    B.fds_rhs_system(op, "ycfie", 1.0, f, h)
    Sy = B.fds_op_yukawa(op).cpu().numpy()
    assert np.abs(Sy.imag).max() == 0.0
    err = np.abs(Sy.real - Sy_o).max() / np.abs(Sy_o).max()
    assert err <= 1e-13, err
    op.close()


def test_yukawa_operator_sampled_entries_large(ctx):
    """N = 4096 (several row and column tiles, a ragged last tile): entries
    sampled on and off the band against the oracle one by one."""
    n, k = 4096, 10.0
    _say(f"case: yukawa operator sampled n={n}")
    nodes = wl.curve_nodes("star", n)
    m = geometry.mesh(nodes)
    op = B.fds_assemble(ctx, torch.from_numpy(nodes).cuda(), k)
    f, h = B.fds_rhs_planewave(op, torch.zeros(1, dtype=torch.float64), torch.ones(1, dtype=torch.complex128))
    B.fds_rhs_system(op, "ycfie", 1.0, f, h)
    Sy = B.fds_op_yukawa(op)
    rs = np.random.default_rng(11)
    I = np.concatenate([rs.integers(0, n, 200), np.arange(0, n, 97), [n - 1, n - 1, 0]])
    J = np.concatenate([rs.integers(0, n, 200), (np.arange(0, n, 97) + rs.integers(-2, 3, 43)) % n, [0, n - 2, n - 1]])
    got = Sy[torch.from_numpy(I).cuda(), torch.from_numpy(J).cuda()].cpu().numpy()
    ref = assembly.entries_yukawa(m, k, I, J)
    scale = np.abs(np.diag(Sy.real.cpu().numpy())).max()
    assert np.abs(got.real - ref).max() <= 1e-13 * scale
    op.close()


SOLVE_CASES = [("star", 300, 10.0, 41, 1.0), ("ellipse", 257, 5.0, 31, 0.5), ("circle", 128, 1.0, 21, 1.0)]


@pytest.mark.parametrize("kind,n,k,nm,alpha", SOLVE_CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_yukawa_cfie_solve_parity(ctx, kind, n, k, nm, alpha, prec):
    _say(f"case: ycfie solve {kind} n={n} k={k} n_modes={nm} alpha={alpha} {prec}")
    nodes = wl.curve_nodes(kind, n)
    m = geometry.mesh(nodes)
    ang, _ = wl.planewaves(11, 5)
    amps = wl.random_amplitudes(12, 5)
    op = B.fds_assemble(ctx, torch.from_numpy(nodes).cuda(), k, precision=prec)
    f, h = B.fds_rhs_planewave(op, torch.from_numpy(ang), torch.from_numpy(amps))
    ne = B.fds_filter(op, "ycfie", alpha, nm)
    B.fds_compress(op, rank_cap=ne + 1, oversample=10, power_iters=2, seed=7)
    B.fds_factor(op)
    j, y, st = B.fds_solve(op, f, h, max_iters=8, tol=1e-12, want_y=True)
    assert st["converged"], st
    pb = solver.Problem(nodes, k, form="ycfie", alpha=alpha, n_modes=nm, rank_cap=ne + 1, oversample=10,
                        power_iters=2, seed=7)
    ops = solver.build_operators(pb)
    assert ops.n_eff == ne
    fo, ho = assembly.rhs_planewave(m, k, ang, amps)
    v = formulation.rhs_vector("ycfie", ops.S, ops.Gmh, ops.Gi, fo.T, ho.T, alpha, ops.Sy)
    yf = solver.y_filtered(ops, v)
    tol = 1e-10 if prec == "fp64" else 1e-6
    err = solver.relerr(y.cpu().numpy().T, yf)
    _say(f"  y vs y_fil {err:.2e} (bound {tol:g})")
    assert err <= tol
    # the split path gives the same solution
    w = B.fds_rhs_system(op, "ycfie", alpha, f, h)
    j2, _, st2 = B.fds_solve_system(op, w, max_iters=8, tol=1e-12)
    assert (torch.linalg.vector_norm(j2 - j) / torch.linalg.vector_norm(j)).item() <= 1e-14
    op.close()


def test_yukawa_batch_rejected(ctx):
    _say("case: ycfie batch rejected")
    nodes = wl.curve_nodes("circle", 64)
    ops = B.fds_assemble_batch(ctx, [torch.from_numpy(nodes).cuda()], [1.0])
    with pytest.raises(B.FdsError) as e:
        B.fds_filter_batch(ops, "ycfie", 1.0, 21)
    assert e.value.name == "FDS_ERR_ARG"
    for o in ops:
        o.close()
