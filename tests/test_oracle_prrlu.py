"""Pins of the oracle's LDU with full pivoting (Alg. 2) against LAPACK's
complete-pivoting LU, exact-rank matrices, the dense residual and small
hand-checked tie cases."""

import numpy as np
import pytest
from scipy.linalg import lapack

from oracle import prrlu


def _getc2_order(ipiv, jpiv, n):
    rows = np.arange(n)
    cols = np.arange(n)
    for i in range(n):
        p = ipiv[i]          # the scipy wrapper returns 0-based interchanges
        q = jpiv[i]
        rows[[i, p]] = rows[[p, i]]
        cols[[i, q]] = cols[[q, i]]
    return rows, cols


@pytest.mark.parametrize("n,seed", [(5, 1), (17, 2), (40, 3)])
def test_pivots_match_lapack_getc2_real(n, seed):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n))
    lu, ipiv, jpiv, info = lapack.dgetc2(M.copy(order="F"))
    assert info == 0
    rows, cols = _getc2_order(ipiv, jpiv, n)
    res = prrlu(M, 0.0, n, log_gaps=True)
    assert min(res.gaps) > 1e-10          # tie-free, so the order is unique
    assert res.rank == n and res.eps == 0.0
    np.testing.assert_array_equal(res.rows, rows[:n])
    np.testing.assert_array_equal(res.cols, cols[:n])
    Ulap = np.triu(lu)
    Llap = np.tril(lu, -1) + np.eye(n)
    np.testing.assert_allclose(res.pivots, np.diag(Ulap), rtol=1e-12, atol=0)
    np.testing.assert_allclose(res.L[rows, :], Llap, rtol=0, atol=1e-12)
    np.testing.assert_allclose(res.U[:, cols], Ulap / np.diag(Ulap)[:, None], rtol=0, atol=1e-11)


@pytest.mark.parametrize("n,seed", [(6, 4), (23, 5)])
def test_pivots_match_lapack_getc2_complex(n, seed):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    lu, ipiv, jpiv, info = lapack.zgetc2(M.copy(order="F"))
    assert info == 0
    rows, cols = _getc2_order(ipiv, jpiv, n)
    res = prrlu(M, 0.0, n, log_gaps=True)
    assert min(res.gaps) > 1e-10
    np.testing.assert_array_equal(res.rows, rows[:n])
    np.testing.assert_array_equal(res.cols, cols[:n])
    np.testing.assert_allclose(res.pivots, np.diag(lu), rtol=1e-12)


@pytest.mark.parametrize("m,n,r", [(30, 20, 7), (64, 96, 33), (5, 5, 5)])
def test_exact_rank_gives_rank_pivots(m, n, r):
    rng = np.random.default_rng(m * n + r)
    M = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    res = prrlu(M, 1e-9 * np.abs(M).max(), 1000)
    assert res.rank == r
    assert res.eps <= 1e-12 * np.abs(M).max()
    np.testing.assert_allclose(res.L @ res.D @ res.U, M, atol=1e-12 * np.abs(M).max())


@pytest.mark.parametrize("cplx", [False, True])
def test_error_estimate_is_max_residual(cplx):
    rng = np.random.default_rng(11)
    M = rng.standard_normal((40, 50))
    if cplx:
        M = M + 1j * rng.standard_normal((40, 50))
    for k in (1, 5, 17, 39):
        res = prrlu(M, 0.0, k)
        assert res.rank == k
        dense = np.abs(M - res.L @ res.D @ res.U).max()
        assert abs(res.eps - dense) <= 1e-12 * np.abs(M).max()


def test_tolerance_stop_and_literal_rule():
    rng = np.random.default_rng(12)
    # singular values spread over many decades
    U, _ = np.linalg.qr(rng.standard_normal((30, 30)))
    V, _ = np.linalg.qr(rng.standard_normal((30, 30)))
    M = (U * (10.0 ** -np.arange(30) * 1.0)) @ V.T
    ex = prrlu(M, 1e-6, 100)
    li = prrlu(M, 1e-6, 100, rule="literal")
    assert ex.eps <= 1e-6
    # the exclusive rule never accepts a pivot of magnitude <= tol
    assert np.all(np.abs(ex.pivots[1:]) > 1e-6)
    # the literal rule accepts exactly one more: the first pivot <= tol
    assert li.rank == ex.rank + 1
    np.testing.assert_array_equal(li.rows[:ex.rank], ex.rows)
    assert abs(li.pivots[-1]) <= 1e-6 and li.eps == abs(li.pivots[-1])


def test_tie_break_smallest_row_then_column():
    M = np.array([[0.0, 2.0], [2.0, 0.0]])
    res = prrlu(M, 0.0, 2)
    assert list(res.rows) == [0, 1] and list(res.cols) == [1, 0]
    M = np.ones((3, 4))
    res = prrlu(M, 0.0, 3)
    assert res.rank == 1 and list(res.rows) == [0] and list(res.cols) == [0]
    assert res.eps == 0.0


def test_maxrank_cap_and_shapes():
    rng = np.random.default_rng(13)
    M = rng.standard_normal((12, 7))
    res = prrlu(M, 0.0, 3)
    assert res.rank == 3 and res.L.shape == (12, 3) and res.U.shape == (3, 7)
    res = prrlu(M, 0.0, 100)
    assert res.rank == 7 and res.eps == 0.0


def test_zero_matrix_path():
    for cplx in (False, True):
        M = np.zeros((4, 6), dtype=complex if cplx else float)
        res = prrlu(M, 1e-12, 5)
        assert res.zero_path and res.rank == 1 and res.eps == 0.0
        assert list(res.rows) == [0] and list(res.cols) == [0]
        np.testing.assert_array_equal(res.L @ res.D @ res.U, M)


def test_first_pivot_always_accepted():
    M = np.full((3, 3), 1e-20)
    M[1, 2] = 2e-20
    res = prrlu(M, 1e-8, 3)
    assert res.rank == 1 and list(res.rows) == [1] and list(res.cols) == [2]
