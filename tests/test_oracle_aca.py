"""Pins of the oracle's adaptive cross approximation (Bebendorf's ACA with
partial pivoting, the second skeleton-detecting algorithm the paper cites in
Inversion of the structured matrices): exact recovery of low-rank matrices, the
interpolation property on the pivot rows and columns, a hand-worked 2 x 2 case,
the stopping rule, and the skeleton of a filtered compact part."""
import numpy as np
import pytest

from oracle import compress, solver
from paper_2210_08580_amd import workloads as wl


def _lowrank(rs, m, n, r):
    return ((rs.standard_normal((m, r)) + 1j * rs.standard_normal((m, r)))
            @ (rs.standard_normal((r, n)) + 1j * rs.standard_normal((r, n))))


@pytest.mark.parametrize("r", [1, 3, 7])
def test_aca_recovers_low_rank_exactly(r):
    rs = np.random.default_rng(r)
    M = _lowrank(rs, 50, 70, r)
    U, V, rows, cols, nrm = compress.aca(M, 30, 1e-14)
    # after r crosses the residual is rounding; a further cross, if any, is tiny
    assert U.shape[1] in (r, r + 1)
    assert np.abs(M - U[:, :r] @ V[:, :r].T).max() <= 1e-12 * np.abs(M).max()
    if U.shape[1] == r + 1:
        assert nrm[r] <= 1e-13 * nrm[0]
    assert len(set(rows)) == len(rows) and len(set(cols)) == len(cols)


def test_aca_interpolates_pivot_rows_and_columns():
    rs = np.random.default_rng(5)
    x = np.linspace(0, 1, 60)
    M = 1.0 / (1.0 + np.abs(x[:, None] - x[None, :] - 2.5)) + 0j   # smooth, numerically low rank
    U, V, rows, cols, _ = compress.aca(M, 6, 0.0)
    S = U @ V.T
    assert np.abs(S[rows, :] - M[rows, :]).max() <= 1e-13
    assert np.abs(S[:, cols] - M[:, cols]).max() <= 1e-13


def test_aca_two_by_two_by_hand():
    M = np.array([[1.0, 4.0], [2.0, 3.0]], dtype=complex)
    U, V, rows, cols, nrm = compress.aca(M, 1, 0.0)
    # row 0, pivot 4 at column 1: b = (1/4, 1), a = column 1 = (4, 3)
    assert rows == [0] and cols == [1]
    assert np.allclose(V[:, 0], [0.25, 1.0]) and np.allclose(U[:, 0], [4.0, 3.0])
    U, V, rows, cols, nrm = compress.aca(M, 2, 0.0)
    # second cross: residual row 1 = (2 - 0.75, 0), pivot at column 0; exact
    assert rows == [0, 1] and cols == [1, 0]
    assert np.abs(U @ V.T - M).max() <= 1e-15


def test_aca_stopping_rule():
    rs = np.random.default_rng(9)
    U0 = np.linalg.qr(rs.standard_normal((80, 20)))[0]
    V0 = np.linalg.qr(rs.standard_normal((90, 20)))[0]
    M = (U0 * (10.0 ** -np.arange(20))) @ V0.T + 0j
    for tol in (1e-3, 1e-6, 1e-9):
        U, V, rows, cols, nrm = compress.aca(M, 40, tol)
        S = U @ V.T
        k = U.shape[1]
        # the last cross met the rule, the earlier ones did not
        sk = [np.linalg.norm(U[:, :q + 1] @ V[:, :q + 1].T) for q in range(k)]
        assert nrm[-1] <= tol * sk[-1] * (1 + 1e-12)
        assert all(nrm[q] > tol * sk[q] for q in range(k - 1))
        # and the error is about the first neglected singular value
        assert np.linalg.norm(M - S, 2) <= 100 * 10.0 ** -(k)


def test_aca_skeleton_of_filtered_compact_part():
    nodes = wl.curve_nodes("random", 160)
    pb = solver.Problem(nodes, 3.0, form="efie", n_modes=41)
    ops = solver.build_operators(pb)
    U, V, rows, cols, nrm = compress.aca(ops.Ac, 60, 1e-10)
    # the filtered compact part has rank n_eff: ACA needs no more crosses than that
    assert U.shape[1] <= ops.n_eff + 1
    assert np.abs(ops.Ac - U @ V.T).max() <= 1e-8 * np.abs(ops.Ac).max()
