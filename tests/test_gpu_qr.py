"""GPU checks of the QR that orthonormalises the sketch and projected blocks of
the truncating compression (fds_zqr): orthonormal Q, A = Q R with R upper
triangular, |R| equal to LAPACK's (R is unique up to unit row phases), and the
choice between CholeskyQR2 and Householder: CholeskyQR2 on well-conditioned
blocks of at most 140 columns, Householder on wider blocks, on blocks whose
condition number defeats CholeskyQR2 and on rank-deficient ones."""
import numpy as np
import pytest
import torch

from paper_2210_08580_amd import binding as B

pytestmark = pytest.mark.gpu
EPS = float(np.finfo(np.float64).eps)


@pytest.fixture(scope="module")
def ctx():
    c = B.fds_ctx_create(0)
    yield c
    c.close()


def _rand(rs, M, m):
    return rs.standard_normal((M, m)) + 1j * rs.standard_normal((M, m))


def _with_singular_values(rs, M, m, s):
    U, _ = np.linalg.qr(_rand(rs, M, m))
    V, _ = np.linalg.qr(_rand(rs, m, m))
    return (U * s) @ V.conj().T


def _run(ctx, A, method):
    M, m = A.shape
    t = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
    Q, hh = B.fds_zqr(ctx, t, method)
    Qn = Q.cpu().numpy().T
    R = np.triu(t.cpu().numpy().T[:m, :])
    return Qn, R, hh


def _check(A, Q, R, orth_tol, res_tol):
    m = A.shape[1]
    assert np.abs(Q.conj().T @ Q - np.eye(m)).max() <= orth_tol
    assert np.abs(Q @ R - A).max() <= res_tol * np.abs(A).max()


@pytest.mark.parametrize("M,m", [(3000, 100), (16384, 138), (511, 138), (64, 64), (7, 1), (600, 140), (600, 141),
                                 (2000, 17), (40037, 138)])   # 40037 rows: more 64-row chunks than workgroups
@pytest.mark.parametrize("method", [B.FDS_QR_AUTO, B.FDS_QR_HOUSEHOLDER])
def test_qr_well_conditioned(ctx, M, m, method):
    print(f"case: zqr M={M} m={m} method={method}", flush=True)
    rs = np.random.default_rng(M + 7 * m + method)
    A = _rand(rs, M, m)
    Q, R, hh = _run(ctx, A, method)
    assert hh == (method == B.FDS_QR_HOUSEHOLDER or m > 140)
    _check(A, Q, R, 64 * EPS * np.sqrt(m), 64 * EPS * np.sqrt(m))
    Rn = np.linalg.qr(A, mode="r")
    assert np.abs(np.abs(R) - np.abs(Rn)).max() <= 1e-12 * np.abs(Rn).max()


@pytest.mark.parametrize("cond", [1e5, 1e7])
def test_qr_moderately_ill_conditioned_stays_on_cholesky(ctx, cond):
    # kappa^2 u well below one: the first pass leaves Q1 close to orthonormal
    print(f"case: zqr cond={cond}", flush=True)
    rs = np.random.default_rng(3)
    A = _with_singular_values(rs, 4000, 120, np.geomspace(1.0, 1.0 / cond, 120))
    Q, R, hh = _run(ctx, A, B.FDS_QR_AUTO)
    assert not hh
    _check(A, Q, R, 1e-13, 1e-13)


@pytest.mark.parametrize("cond", [1e10, 1e14])
def test_qr_ill_conditioned_falls_back(ctx, cond):
    print(f"case: zqr fallback cond={cond}", flush=True)
    rs = np.random.default_rng(4)
    A = _with_singular_values(rs, 3000, 80, np.geomspace(1.0, 1.0 / cond, 80))
    Q, R, hh = _run(ctx, A, B.FDS_QR_AUTO)
    assert hh
    _check(A, Q, R, 1e-13, 1e-13)


def test_qr_rank_deficient_falls_back(ctx):
    print("case: zqr rank deficient", flush=True)
    rs = np.random.default_rng(5)
    A = _rand(rs, 500, 40)
    A[:, 7] = 0.0
    A[:, 30] = A[:, 3]
    Q, R, hh = _run(ctx, A, B.FDS_QR_AUTO)
    assert hh
    _check(A, Q, R, 1e-13, 1e-13)


def test_qr_bad_arguments(ctx):
    print("case: zqr bad arguments", flush=True)
    t = torch.zeros((4, 3), dtype=torch.complex128, device="cuda")   # 3 x 4: fewer rows than columns
    with pytest.raises(B.FdsError) as e:
        B.fds_zqr(ctx, t)
    assert e.value.name == "FDS_ERR_ARG"
    t = torch.zeros((3, 8), dtype=torch.complex128, device="cuda")
    with pytest.raises(B.FdsError) as e:
        B.fds_zqr(ctx, t, method=7)
    assert e.value.name == "FDS_ERR_ARG"
