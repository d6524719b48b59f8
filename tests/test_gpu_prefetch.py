"""The filter's eigensolver started by fds_assemble (fds_asm_opts.filter_modes):
the same eigenvalues, basis and filtered solution as without the hint, the hint
discarded by a filter call with another filtering point or without the null mode,
and an operator destroyed while its eigensolver may still run. The basis is also
checked against the oracle's filter (paper, Laplacian Filters, Two-Dimensional
Case, eq. (LapFilter))."""
import numpy as np
import pytest
import torch

from oracle import assembly, filters, formulation, geometry
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


def _filtered(ctx, nodes, k, nm, prec, hint, keep=True, nm_filter=None):
    op = B.fds_assemble(ctx, nodes, k, precision=prec, filter_modes=hint)
    ne = B.fds_filter(op, "efie", 1.0, nm if nm_filter is None else nm_filter, keep_nullspace=keep)
    lam = B.fds_op_filter_eigenvalues(op)
    Vn = B.fds_op_filter_basis(op).clone()
    return op, ne, lam, Vn


@pytest.mark.parametrize("kind,n,k,nm,prec", [("star", 1200, 10.0, 63, "fp32"), ("ellipse", 777, 5.0, 41, "fp64"),
                                              ("random", 300, 3.0, 255, "fp64")])
def test_prefetched_eigensolver_matches(ctx, kind, n, k, nm, prec):
    _say(f"case: prefetched eigensolver {kind} n={n} n_modes={nm} {prec}")
    nodes = torch.from_numpy(wl.curve_nodes(kind, n)).cuda()
    op0, ne0, lam0, V0 = _filtered(ctx, nodes, k, nm, prec, 0)
    op1, ne1, lam1, V1 = _filtered(ctx, nodes, k, nm, prec, nm)
    assert ne0 == ne1
    assert np.array_equal(np.asarray(lam0), np.asarray(lam1))
    assert torch.equal(V0, V1)
    # and the projector against the oracle's
    m = geometry.mesh(nodes.cpu().numpy())
    _, Gmh, _ = formulation.gram_powers(*assembly.gram(m))
    Vo, _, neo = filters.laplacian_filter(m, nm, True, 1e-6, Gmh)
    assert neo == ne1
    Vn = V1.cpu().numpy().T
    err = np.abs(Vn @ Vn.T - Vo @ Vo.T).max()
    # subspace conditioning: eps ||L~|| / (gap at the cut)
    lam_all = np.linalg.eigvalsh(filters.orthonormal_laplacian(m, Gmh))
    tol = max(1e-12, 64 * 2.2e-16 * lam_all[-1] / (lam_all[ne1] - lam_all[ne1 - 1]))
    _say(f"  n_eff {ne1}, projector vs oracle {err:.2e} (bound {tol:.1e})")
    assert err <= tol
    # a full solve from the prefetched operator equals the plain one
    rs = np.random.default_rng(3)
    ang = torch.from_numpy(rs.uniform(0, 2 * np.pi, 3))
    amp = torch.from_numpy(wl.random_amplitudes(4, 3))
    js = []
    for op in (op0, op1):
        B.fds_compress(op, ne1, 10, 2, 0.0, seed=1)
        B.fds_factor(op)
        f, h = B.fds_rhs_planewave(op, ang, amp)
        j, _, _ = B.fds_solve(op, f, h, max_iters=2, tol=1e-12)
        js.append(j)
    assert torch.equal(js[0], js[1])
    op0.close()
    op1.close()


def test_prefetch_discarded_and_destroyed(ctx):
    _say("case: prefetch discarded by another filtering point / no null mode; destroy before filter")
    nodes = torch.from_numpy(wl.curve_nodes("star", 900)).cuda()
    ref_a = _filtered(ctx, nodes, 8.0, 41, "fp64", 0)
    got_a = _filtered(ctx, nodes, 8.0, 63, "fp64", 63, nm_filter=41)      # hint for 63, filter at 41
    assert ref_a[1] == got_a[1] and torch.equal(ref_a[3], got_a[3])
    ref_b = _filtered(ctx, nodes, 8.0, 41, "fp64", 0, keep=False)
    got_b = _filtered(ctx, nodes, 8.0, 41, "fp64", 41, keep=False)        # hint keeps the null mode
    assert ref_b[1] == got_b[1] and torch.equal(ref_b[3], got_b[3])
    for t in (ref_a, got_a, ref_b, got_b):
        t[0].close()
    # destroyed while the started eigensolver may still be running
    op = B.fds_assemble(ctx, nodes, 8.0, filter_modes=63)
    op.close()
    torch.cuda.synchronize()
    # the context is still usable
    op = B.fds_assemble(ctx, nodes, 8.0, filter_modes=41)
    assert B.fds_filter(op, "efie", 1.0, 41) == ref_a[1]
    op.close()
    with pytest.raises(B.FdsError) as e:
        B.fds_assemble(ctx, nodes, 8.0, filter_modes=901)
    assert e.value.name == "FDS_ERR_ARG"
