"""GPU parity of the adjoint solve (fds_solve_adjoint) against the oracle, through
the C ABI: (beta I + P C)^H y = v for the filtered operator (lossless and
truncating skeletons, plain FP64 and mixed precision) and (beta I + C)^H y = v for
the unfiltered one, with v in the paper's normalised coordinates. The oracle side
solves the conjugate-transposed dense systems by LU (paper, Inversion of the
structured matrices: the Woodbury identity holds for beta I + W^H U^H as well)."""
import numpy as np
import pytest
import scipy.linalg as sla
import torch

from oracle import solver
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


def _v(n, nrhs, seed):
    rs = np.random.default_rng(seed)
    return (rs.standard_normal((n, nrhs)) + 1j * rs.standard_normal((n, nrhs))) / np.sqrt(2.0)


# kind, n, k, form, n_modes, rank_cap, oversample, power_iters, tol, precision
CASES = [("star", 400, 10.0, "efie", 41, 42, 10, 2, 0.0, "fp64"),       # exact skeleton
         ("ellipse", 350, 5.0, "cfie", 51, 20, 6, 2, 0.0, "fp64"),      # truncating (sketched)
         ("circle", 256, 1.0, "mfie", 21, 22, 10, 2, 0.0, "fp64"),
         ("random", 300, 8.0, "ycfie", 31, 32, 10, 2, 0.0, "fp64"),
         ("star", 600, 10.0, "efie", 63, 64, 10, 2, 0.0, "fp32"),       # mixed precision
         ("ellipse", 350, 5.0, "cfie", 51, 20, 6, 2, 0.0, "fp32")]


@pytest.mark.parametrize("kind,n,k,form,nm,cap,p,q,tol,prec", CASES)
def test_adjoint_solve_filtered(ctx, kind, n, k, form, nm, cap, p, q, tol, prec):
    _say(f"case: adjoint filtered {kind} n={n} k={k} {form} n_modes={nm} r={cap} {prec}")
    nodes = wl.curve_nodes(kind, n)
    op = B.fds_assemble(ctx, torch.from_numpy(nodes).cuda(), k, precision=prec)
    ne = B.fds_filter(op, form, 1.0, nm)
    r = B.fds_compress(op, cap, p, q, tol, seed=5)
    B.fds_factor(op)
    pb = solver.Problem(nodes, k, form=form, n_modes=nm)
    ops = solver.build_operators(pb)
    assert ops.n_eff == ne
    v = _v(n, 5, n + 3)
    A = ops.beta * np.eye(n) + ops.Ac
    yo = sla.solve(A.conj().T, v)
    y, u, st = B.fds_solve_adjoint(op, torch.from_numpy(np.ascontiguousarray(v.T)).cuda(), max_iters=60,
                                   tol=1e-12 if prec == "fp64" else 1e-9, want_u=True)
    assert st["converged"], st
    bound = 1e-10 if prec == "fp64" else 1e-6
    e = solver.relerr(y.cpu().numpy().T, yo)
    eu = solver.relerr(u.cpu().numpy().T, ops.Gmh @ yo)
    _say(f"  rank {r} of {ne}, {st['iters']} sweeps: y vs oracle {e:.2e}, u vs oracle {eu:.2e} (bound {bound:g})")
    assert e <= bound and eu <= bound
    if r == ne and prec == "fp64":
        # exact skeleton: the adjoint Woodbury solve alone is already the solution
        y0, _, _ = B.fds_solve_adjoint(op, torch.from_numpy(np.ascontiguousarray(v.T)).cuda(), max_iters=0,
                                       tol=1e300)
        assert solver.relerr(y0.cpu().numpy().T, yo) <= 1e-10
    op.close()


@pytest.mark.parametrize("kind,n,k,form,nm,prec", [("star", 300, 10.0, "efie", 41, "fp64"),
                                                   ("ellipse", 256, 5.0, "cfie", 41, "fp64"),
                                                   ("circle", 200, 1.0, "mfie", 21, "fp64"),
                                                   ("random", 240, 6.0, "ycfie", 31, "fp64"),
                                                   ("star", 300, 10.0, "efie", 41, "fp32")])
def test_adjoint_solve_unfiltered(ctx, kind, n, k, form, nm, prec):
    _say(f"case: adjoint unfiltered {kind} n={n} k={k} {form} n_modes={nm} {prec}")
    nodes = wl.curve_nodes(kind, n)
    op = B.fds_assemble(ctx, torch.from_numpy(nodes).cuda(), k, precision=prec)
    ne = B.fds_filter(op, form, 1.0, nm)
    B.fds_compress(op, ne, 10, 2, 0.0, seed=5)
    B.fds_factor(op)
    ops = solver.build_operators(solver.Problem(nodes, k, form=form, n_modes=nm))
    v = _v(n, 4, n + 7)
    A = ops.beta * np.eye(n) + ops.C
    yo = sla.solve(A.conj().T, v)
    y, _, st = B.fds_solve_adjoint(op, torch.from_numpy(np.ascontiguousarray(v.T)).cuda(), max_iters=200,
                                   tol=1e-12 if prec == "fp64" else 1e-9, unfiltered=True)
    assert st["converged"], st
    e = solver.relerr(y.cpu().numpy().T, yo)
    bound = 1e-10 if prec == "fp64" else 1e-6
    _say(f"  {st['iters']} sweeps: y vs oracle {e:.2e} (bound {bound:g})")
    assert e <= bound
    op.close()


def test_adjoint_solve_errors(ctx):
    _say("case: adjoint solve argument and state errors")
    nodes = wl.circle(64)
    op = B.fds_assemble(ctx, torch.from_numpy(nodes).cuda(), 1.0)
    v = torch.zeros((2, 64), dtype=torch.complex128, device="cuda")
    with pytest.raises(B.FdsError) as e:
        B.fds_solve_adjoint(op, v)
    assert e.value.name == "FDS_ERR_STATE"
    B.fds_filter(op, "efie", 1.0, 9)
    B.fds_compress(op, 9)
    B.fds_factor(op)
    with pytest.raises(B.FdsError) as e:
        B.fds_solve_adjoint(op, v, max_iters=-1)
    assert e.value.name == "FDS_ERR_ARG"
    # a residual target that one sweep cannot reach is reported
    rs = np.random.default_rng(1)
    vr = torch.from_numpy(rs.standard_normal((2, 64)) + 0j).cuda()
    with pytest.raises(B.FdsError) as e:
        B.fds_solve_adjoint(op, vr, max_iters=0, tol=1e-30, unfiltered=True)
    assert e.value.name == "FDS_ERR_NOCONV"
    op.close()
