"""Pins of the learned-proposal oracle (features, network, rook search)."""

import numpy as np
import pytest

from oracle import proposal as P
from oracle import prrlu


def test_rook_pivots_dominate_their_row_and_column():
    """With unlimited scans every accepted pivot is the largest residual of
    its row and of its column (checked against the dense residual)."""
    rng = np.random.default_rng(3)
    for trial in range(6):
        m, n = rng.integers(4, 14, 2)
        M = rng.standard_normal((m, n))
        rk = P.rook_lu(M, 0.0, min(m, n), max_iter=1000)
        assert rk.rank == min(m, n)
        for k in range(rk.rank):
            R = M - rk.L[:, :k] @ rk.Up[:k, :]
            R[rk.rows[:k], :] = 0.0
            R[:, rk.cols[:k]] = 0.0
            i, j = rk.rows[k], rk.cols[k]
            assert abs(R[i, j]) >= np.abs(R[i, :]).max() * (1 - 1e-12)
            assert abs(R[i, j]) >= np.abs(R[:, j]).max() * (1 - 1e-12)
            np.testing.assert_allclose(rk.Up[k], R[i], rtol=0, atol=1e-12 * np.abs(M).max())


def test_rook_recovers_exact_rank_and_is_accepted():
    rng = np.random.default_rng(5)
    M = rng.standard_normal((12, 4)) @ rng.standard_normal((4, 9))
    rk = P.rook_lu(M, 1e-10, 9)
    assert rk.rank == 4
    ok, eps = P.rook_accept(M, rk, 1e-10)
    assert ok and eps < 1e-12
    np.testing.assert_allclose(rk.L @ rk.Up, M, atol=1e-12)


def test_rook_right_factor_is_identity_on_pivot_columns():
    rng = np.random.default_rng(7)
    M = rng.standard_normal((9, 11))
    rk = P.rook_lu(M, 0.0, 6)
    Y = P.rook_right_factor(rk)
    assert np.array_equal(Y[:, rk.cols], np.eye(rk.rank))
    # the cross interpolation A B with A = M[:, J] reproduces the pivot rows
    A = M[:, rk.cols]
    np.testing.assert_allclose((A @ Y)[rk.rows], M[rk.rows], atol=1e-11)


def test_rook_capped_rank_error_is_checked_densely():
    rng = np.random.default_rng(9)
    M = rng.standard_normal((10, 10))
    rk = P.rook_lu(M, 1e-12, 3)
    ok, eps = P.rook_accept(M, rk, 1e-12)
    assert rk.rank == 3 and not ok
    full = prrlu(M, 1e-12, 3)
    # the full search's estimate is the same kind of quantity (max residual)
    assert eps >= full.eps * 0.5


def test_features_by_hand():
    M = np.array([[1.0, -4.0, 0.0, 2.0], [0.0, 1.0, -2.0, 0.0], [3.0, 0.0, 0.0, 1.0]])
    A = [np.array([[3.0, 4.0], [0.0, 0.0], [0.0, 10.0]])]
    F = P.row_features(M, A, prev_rows=[2])
    assert P.sample_columns(4) == [0, 1, 2, 3]
    np.testing.assert_allclose(F[:, 0], [0.5, 0.0, 1.0])
    assert np.all(F[:, 1] == 0)
    np.testing.assert_array_equal(F[:, 2], [0, 0, 1])
    np.testing.assert_allclose(F[0, 3:], [0.25, 1.0, 0.0, 0.5])
    np.testing.assert_allclose(F[2, 3:], [0.75, 0.0, 0.0, 0.25])


def test_network_gradients_match_central_differences():
    """float64 copy (roundings off): analytic gradients of the mean BCE loss
    against central differences."""
    net = P.mlp_init(11)
    net64 = P.MLP(*[p.astype(np.float64) for p in net.params()])
    rng = np.random.default_rng(13)
    X = rng.uniform(0, 1, (16, P.NFEAT))
    y = (rng.uniform(0, 1, 16) < 0.3).astype(np.float64)
    grads, _ = P.mlp_grads(net64, X, y, rounding=False)

    def loss():
        z, _ = P.mlp_forward(net64, X, rounding=False)
        return P.bce_loss(z, y)

    for pi, (p, g) in enumerate(zip(net64.params(), grads)):
        flat = p.reshape(-1)
        gflat = np.asarray(g).reshape(-1)
        for idx in rng.choice(flat.size, min(5, flat.size), replace=False):
            old = flat[idx]
            h = 1e-6
            flat[idx] = old + h
            lp = loss()
            flat[idx] = old - h
            lm = loss()
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gflat[idx]) <= 1e-6 + 1e-4 * abs(fd), (pi, idx, fd, gflat[idx])


def test_rounded_forward_is_close_to_exact():
    net = P.mlp_init(17)
    X = np.random.default_rng(1).uniform(0, 1, (32, P.NFEAT)).astype(np.float32)
    z16, _ = P.mlp_forward(net, X)
    z64, _ = P.mlp_forward(P.MLP(*[p.astype(np.float64) for p in net.params()]), X, rounding=False)
    assert z16.dtype == np.float32
    assert np.abs(z16 - z64).max() <= 2e-2 * (1 + np.abs(z64).max())


def test_adam_learns_a_separable_rule():
    rng = np.random.default_rng(19)
    X = rng.uniform(0, 1, (128, P.NFEAT)).astype(np.float32)
    y = (X[:, 0] + X[:, 3] > 1.0).astype(np.float32)
    net = P.mlp_init(23)
    st = {}
    _, l0 = P.mlp_grads(net, X, y)
    for _ in range(60):
        g, _ = P.mlp_grads(net, X, y)
        P.adam_step(net, g, st, lr=1e-2)
    _, l1 = P.mlp_grads(net, X, y)
    assert l1 < 0.5 * l0


class _Toy:
    """Two scalar parameters, the shape adam_step expects of a network."""

    def __init__(self, a, b):
        self.p = [np.array([a], np.float32), np.array([b], np.float32)]

    def params(self):
        return self.p


def test_adam_two_steps_by_hand():
    """Adam (Kingma and Ba, Algorithm 1) on two scalars, lr 0.1, b1 0.9,
    b2 0.999 and a large eps = 0.1 so that its place (added to sqrt(v_hat),
    not inside the root) shows.  Step 1: the bias corrections make
    m_hat = g and v_hat = g^2, so theta_1 = theta_0 - lr g / (|g| + eps):
    1 - 0.1 * 0.5 / 0.6 = 11/12 and -2 + 0.1 * 0.25 / 0.35 = -27/14.
    Step 2, by hand: m = (0.9 * 0.1 g1 + 0.1 g2), v = (0.999 * 0.001 g1^2 +
    0.001 g2^2), m_hat = m / 0.19, v_hat = v / 0.001999:
      a: m_hat = -0.055 / 0.19 = -0.2894737, sqrt(v_hat) = 0.7906881,
         theta_2 = 11/12 + 0.1 * 0.2894737 / 0.8906881 = 0.9491667;
      b: m_hat = -0.01 / 0.19 = -0.0526316, sqrt(v_hat) = 0.1976127,
         theta_2 = -27/14 + 0.1 * 0.0526316 / 0.2976127 = -1.9108868."""
    net = _Toy(1.0, -2.0)
    st = {}
    P.adam_step(net, [np.array([0.5], np.float32), np.array([-0.25], np.float32)], st, lr=0.1, eps=0.1)
    np.testing.assert_allclose([net.p[0][0], net.p[1][0]], [11 / 12, -27 / 14], rtol=2e-7)
    P.adam_step(net, [np.array([-1.0], np.float32), np.array([0.125], np.float32)], st, lr=0.1, eps=0.1)
    np.testing.assert_allclose([net.p[0][0], net.p[1][0]], [0.9491667, -1.9108868], rtol=3e-7)
    assert st["t"] == 2
