"""GPU parity of the linear-algebra stages and of the whole filtered fast
direct solve against the CPU oracle, through the C ABI."""
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


def _crand(rs, shape):
    return rs.standard_normal(shape) + 1j * rs.standard_normal(shape)


@pytest.mark.parametrize("opa,opb", [(a, b) for a in range(3) for b in range(3)])
@pytest.mark.parametrize("m,n,k", [(70, 33, 129), (40, 40, 5000), (1, 65, 17), (128, 64, 64), (300, 200, 700),
                                   (257, 130, 3000),
                                   # outputs of at most 32 columns (the 128 x 32 tile), ragged rows
                                   (300, 32, 700), (129, 1, 513), (257, 17, 3000)])
def test_zgemm_parity(ctx, opa, opb, m, n, k):
    _say(f"case: zgemm op=({opa},{opb}) m={m} n={n} k={k}")
    rs = np.random.default_rng(m * 7 + n * 3 + k + opa * 11 + opb)
    A = _crand(rs, (m, k) if opa == 0 else (k, m))
    Bm = _crand(rs, (k, n) if opb == 0 else (n, k))
    C0 = _crand(rs, (m, n))
    alpha, beta = 0.7 - 0.2j, -0.3 + 0.5j

    def op(X, o):
        return X if o == 0 else (X.T if o == 1 else X.conj().T)
    ref = alpha * op(A, opa) @ op(Bm, opb) + beta * C0
    # column-major device storage: a tensor of shape (cols, rows) holding M.T
    tA = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
    tB = torch.from_numpy(np.ascontiguousarray(Bm.T)).cuda()
    tC = torch.from_numpy(np.ascontiguousarray(C0.T)).cuda()
    B.fds_zgemm(ctx, opa, opb, tA, tB, tC, alpha, beta)
    got = tC.cpu().numpy().T
    scale = np.abs(A).max() * np.abs(Bm).max() * k
    assert np.abs(got - ref).max() <= 8 * EPS * scale


def _op_and_oracle(kind, n, k):
    nodes = wl.curve_nodes(kind, n)
    m = geometry.mesh(nodes)
    return nodes, m


def _graded_circle(n, a):
    """Unit circle with nodes at t = s + a sin s, s uniform: panel ratio (1 + a)/(1 - a)."""
    s = 2.0 * np.pi * np.arange(n) / n
    t = s + a * np.sin(s)
    return np.stack([np.cos(t), np.sin(t)], axis=1)


# (curve, n, grading): grading a > 0 replaces the curve by a graded circle whose
# Gram spectrum is wide (panel ratio 3 and 99), so the Chebyshev degree is high.
GRAM_CASES = [("star", 400, 0.0), ("ellipse", 512, 0.0), ("graded", 300, 0.5), ("graded", 256, 0.98)]


@pytest.mark.parametrize("kind,n,a", GRAM_CASES)
def test_gram_powers_parity(ctx, kind, n, a):
    _say(f"case: apply_gram {kind} n={n} a={a}")
    if kind == "graded":
        nodes = _graded_circle(n, a)
        m = geometry.mesh(nodes)
    else:
        nodes, m = _op_and_oracle(kind, n, 4.0)
    op = B.fds_assemble(ctx, torch.from_numpy(nodes).cuda(), 4.0)
    Gh, Gmh, Gi = formulation.gram_powers(*assembly.gram(m))
    rs = np.random.default_rng(2)
    X = _crand(rs, (5, n))
    for p, R in ((-2, Gi), (-1, Gmh), (1, Gh)):
        t = torch.from_numpy(X.copy()).cuda()
        B.fds_apply_gram(op, p, t)
        ref = (R @ X.T).T
        err = np.abs(t.cpu().numpy() - ref).max() / np.abs(ref).max()
        assert err < 1e-13, (p, err)
    op.close()


FILTER_CASES = [("circle", 256, 1.0, 21, True), ("star", 512, 10.0, 63, True),
                ("ellipse", 301, 5.0, 41, True), ("perturbed_circle", 200, 0.4, 21, False),
                ("circle", 64, 1.0, 20, True),
                # smallest sizes of the two-ended elimination (top/bottom halves of 2..5 steps), odd n
                ("star", 8, 1.0, 5, True), ("ellipse", 9, 1.0, 9, True), ("random", 13, 2.0, 7, False),
                ("star", 131, 3.0, 131, True)]


@pytest.mark.parametrize("kind,n,k,nm,keep", FILTER_CASES)
def test_filter_projector_parity(ctx, kind, n, k, nm, keep):
    _say(f"case: filter {kind} n={n} n_modes={nm} keep={keep}")
    nodes, m = _op_and_oracle(kind, n, k)
    op = B.fds_assemble(ctx, torch.from_numpy(nodes).cuda(), k)
    ne = B.fds_filter(op, "efie", 1.0, nm, keep_nullspace=keep)
    Vn = B.fds_op_filter_basis(op).cpu().numpy().T           # n x ne
    Gh, Gmh, _ = formulation.gram_powers(*assembly.gram(m))
    Vo, lam, neo = filters.laplacian_filter(m, nm, keep, 1e-6, Gmh)
    assert ne == neo
    P = Vn @ Vn.T
    Po = Vo @ Vo.T
    # subspace conditioning: eps * ||L~|| / gap at the cut
    Lt = filters.orthonormal_laplacian(m, Gmh)
    lam_all = np.linalg.eigvalsh(Lt)
    s0 = 0 if keep else 1
    if s0 + ne < len(lam_all):
        gap = lam_all[s0 + ne] - lam_all[s0 + ne - 1]
        tol = max(1e-12, 64 * EPS * lam_all[-1] / gap)
    else:                       # every mode kept: P = I, no cut to condition it
        tol = 1e-12
    assert np.abs(P - Po).max() <= tol, (np.abs(P - Po).max(), tol)
    assert np.abs(Vn.T @ Vn - np.eye(ne)).max() < 1e-12
    # reported eigenvalues (Rayleigh quotients of the final vectors) vs the oracle's,
    # within the backward-error scale of a symmetric eigensolver (eps ||L~||)
    lam_gpu = np.array(B.fds_op_filter_eigenvalues(op)[:ne])
    assert np.abs(lam_gpu - lam[:ne]).max() <= 64 * EPS * lam_all[-1] + 1e-13 * np.abs(lam[:ne]).max()
    op.close()


SOLVE_CASES = [("circle", 256, 1.0, "efie", 21), ("star", 600, 10.0, "efie", 63),
               ("star", 400, 10.0, "mfie", 41), ("ellipse", 350, 5.0, "cfie", 51),
               ("perturbed_circle", 333, 0.4, "efie", 31)]


@pytest.mark.parametrize("kind,n,k,form,nm", SOLVE_CASES)
def test_lossless_solve_parity(ctx, kind, n, k, form, nm):
    _say(f"case: solve {kind} n={n} k={k} {form} n_modes={nm}")
    nodes, m = _op_and_oracle(kind, n, k)
    ang, _ = wl.planewaves(11, 6)
    amps = wl.random_amplitudes(12, 6)
    op = B.fds_assemble(ctx, torch.from_numpy(nodes).cuda(), k)
    ne = B.fds_filter(op, form, 1.0, nm)
    r = B.fds_compress(op, rank_cap=ne + 1, oversample=10, power_iters=2, seed=7)
    assert r == ne
    B.fds_factor(op)
    f, h = B.fds_rhs_planewave(op, torch.from_numpy(ang), torch.from_numpy(amps))
    j, y, st = B.fds_solve(op, f, h, max_iters=3, tol=1e-12, want_y=True)
    assert st["converged"], st
    pb = solver.Problem(nodes, k, form=form, n_modes=nm, rank_cap=ne + 1, oversample=10,
                        power_iters=2, seed=7)
    ops = solver.build_operators(pb)
    fo, ho = assembly.rhs_planewave(m, k, ang, amps)
    v = formulation.rhs_vector(form, ops.S, ops.Gmh, ops.Gi, fo.T, ho.T)
    yf = solver.y_filtered(ops, v)
    assert solver.relerr(y.cpu().numpy().T, yf) <= 1e-10
    assert solver.relerr(j.cpu().numpy().T, ops.Gmh @ yf) <= 1e-10
    # skeleton in y coordinates equals the filtered compact part
    Ut, Wt = B.fds_op_factors(op)
    UWy = ops.Gh @ (Ut.cpu().numpy().T @ Wt.cpu().numpy()) @ ops.Gmh
    assert np.abs(UWy - ops.Ac).max() <= 1e-11 * np.abs(ops.Ac).max()
    op.close()


def test_state_machine_errors(ctx):
    _say("case: state machine")
    nodes = wl.circle(32)
    op = B.fds_assemble(ctx, torch.from_numpy(nodes).cuda(), 1.0)
    with pytest.raises(B.FdsError) as e:
        B.fds_factor(op)
    assert e.value.name == "FDS_ERR_STATE"
    with pytest.raises(B.FdsError) as e:
        B.fds_compress(op, 8)
    assert e.value.name == "FDS_ERR_STATE"
    with pytest.raises(B.FdsError) as e:
        B.fds_filter(op, "efie", 1.0, 0)
    assert e.value.name == "FDS_ERR_ARG"
    B.fds_filter(op, "efie", 1.0, 9)
    with pytest.raises(B.FdsError) as e:
        f = torch.zeros((1, 32), dtype=torch.complex128, device="cuda")
        B.fds_solve(op, f, None)
    assert e.value.name == "FDS_ERR_STATE"
    op.close()


@pytest.mark.parametrize("r,kind", [(1, "random"), (7, "zero_lead"), (255, "second_kind"), (300, "zero_lead"),
                                    (64, "permuted"), (33, "random")])
def test_dense_inverse(ctx, r, kind):
    """The Woodbury-core inverse: the unpivoted fast path (second-kind matrices) and the
    partial-pivoting fallback (a zero leading pivot, a permuted identity-like matrix)."""
    _say(f"case: dense inverse r={r} {kind}")
    rs = np.random.default_rng(r + len(kind))
    R = rs.standard_normal((r, r)) + 1j * rs.standard_normal((r, r))
    if kind == "second_kind":
        A = np.eye(r) + 0.3 * R / np.sqrt(r)
    elif kind == "zero_lead":
        A = R.copy()
        A[0, 0] = 0.0
    elif kind == "permuted":
        A = (np.eye(r) + 0.05 * R / np.sqrt(r))[rs.permutation(r)]
    else:
        A = R
    At = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
    X, (pmin, amax) = B.fds_zinv(ctx, At)
    Xn = X.cpu().numpy().T
    ref = np.linalg.inv(A)
    cond = np.linalg.cond(A)
    assert np.abs(A @ Xn - np.eye(r)).max() <= 1e-13 * cond * max(1, r / 16)
    assert np.abs(Xn - ref).max() <= 1e-14 * cond * r * np.abs(ref).max()
    assert pmin >= 64 * EPS * amax
    assert torch.equal(At, torch.from_numpy(np.ascontiguousarray(A.T)).cuda())   # input untouched


def test_dense_inverse_singular(ctx):
    _say("case: dense inverse singular")
    rs = np.random.default_rng(5)
    A = rs.standard_normal((20, 20)) + 1j * rs.standard_normal((20, 20))
    A[:, 7] = A[:, 3]
    _, (pmin, amax) = B.fds_zinv(ctx, torch.from_numpy(np.ascontiguousarray(A.T)).cuda())
    assert pmin < 64 * EPS * amax


SPLIT_CASES = [("star", 600, 10.0, "efie", 63, "fp64"), ("ellipse", 301, 5.0, "cfie", 41, "fp64"),
               ("circle", 256, 1.0, "mfie", 21, "fp64"), ("star", 600, 10.0, "efie", 63, "fp32")]


@pytest.mark.parametrize("kind,n,k,form,nm,prec", SPLIT_CASES)
def test_split_solve_matches_solve(ctx, kind, n, k, form, nm, prec):
    """fds_rhs_system enqueued right after the assembly (before the filter) and
    fds_solve_system give fds_solve's solution; the oracle pins it as well."""
    _say(f"case: split solve {kind} n={n} k={k} {form} {prec}")
    nodes, m = _op_and_oracle(kind, n, k)
    ang, _ = wl.planewaves(11, 6)
    amps = wl.random_amplitudes(12, 6)
    op = B.fds_assemble(ctx, torch.from_numpy(nodes).cuda(), k, precision=prec)
    f, h = B.fds_rhs_planewave(op, torch.from_numpy(ang), torch.from_numpy(amps))
    w = B.fds_rhs_system(op, form, 1.0, f, h)
    with pytest.raises(B.FdsError) as e:
        B.fds_solve_system(op, w)
    assert e.value.name == "FDS_ERR_STATE"
    ne = B.fds_filter(op, form, 1.0, nm)
    B.fds_compress(op, rank_cap=ne + 1, oversample=10, power_iters=2, seed=7)
    B.fds_factor(op)
    j1, y1, st1 = B.fds_solve_system(op, w, max_iters=3, tol=1e-12, want_y=True)
    j2, y2, st2 = B.fds_solve(op, f, h, max_iters=3, tol=1e-12, want_y=True)
    assert st1["converged"] and st2["converged"], (st1, st2)
    assert st1["iters"] == st2["iters"]
    d = (torch.linalg.vector_norm(j1 - j2) / torch.linalg.vector_norm(j2)).item()
    assert d <= 1e-14, d
    if prec == "fp64":
        pb = solver.Problem(nodes, k, form=form, n_modes=nm, rank_cap=ne + 1, oversample=10,
                            power_iters=2, seed=7)
        ops = solver.build_operators(pb)
        fo, ho = assembly.rhs_planewave(m, k, ang, amps)
        v = formulation.rhs_vector(form, ops.S, ops.Gmh, ops.Gi, fo.T, ho.T)
        # w = G^{-1/2} v
        assert solver.relerr(w.cpu().numpy().T, ops.Gmh @ v) <= 1e-12
        assert solver.relerr(y1.cpu().numpy().T, solver.y_filtered(ops, v)) <= 1e-10
    with pytest.raises(B.FdsError) as e:
        B.fds_rhs_system(op, "efie", 1.0, None, h)
    assert e.value.name == "FDS_ERR_ARG"
    op.close()
