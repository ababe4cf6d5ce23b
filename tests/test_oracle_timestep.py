"""Pins of the oracle's TT operators and explicit step (oracle/timestep.py)
against what the mathematics fixes: the dense matrix of each stencil MPO
against a periodic stencil built on the grid itself, plane waves as
eigenvectors of the second difference with the closed-form eigenvalue, the
MPO-TT contraction against dense operator times dense vector (and the dense
matrix of an MPO against products of its core slices, entry by entry), and
the whole step against the dense Euler step on small grids."""

import itertools

import numpy as np
import pytest

import oracle
from oracle import timestep as T
import workloads as W


def quantics_to_coords(q, R, ndim):
    """Grid coordinates of quantics index q: site ndim*b + a (first site the
    most significant bit of q) holds bit R-1-b of axis a."""
    L = R * ndim
    x = [0] * ndim
    for s in range(L):
        bit = (q >> (L - 1 - s)) & 1
        b, a = divmod(s, ndim)
        x[a] |= bit << (R - 1 - b)
    return x


def coords_to_quantics(x, R, ndim):
    L = R * ndim
    q = 0
    for s in range(L):
        b, a = divmod(s, ndim)
        q |= ((x[a] >> (R - 1 - b)) & 1) << (L - 1 - s)
    return q


def dense_stencil(R, ndim, axis, weights):
    """(sum_delta w_delta S^delta psi)(x) = sum_delta w_delta psi(x + delta e_axis)."""
    n = 2 ** (R * ndim)
    M = np.zeros((n, n))
    for q in range(n):
        x = quantics_to_coords(q, R, ndim)
        for delta, w in zip((-1, 0, 1), weights):
            y = list(x)
            y[axis] = (y[axis] + delta) % (2 ** R)
            M[q, coords_to_quantics(y, R, ndim)] += w
    return M


@pytest.mark.parametrize("R,ndim", [(4, 1), (3, 2), (2, 3), (3, 3)])
def test_stencil_mpo_matches_grid_stencil(R, ndim):
    rng = np.random.default_rng(R * 10 + ndim)
    for axis in range(ndim):
        w = rng.standard_normal(3)
        got = T.mpo_dense(T.stencil_mpo(R, ndim, axis, w))
        assert np.abs(got - dense_stencil(R, ndim, axis, w)).max() <= 1e-15
        ranks = [T.stencil_mpo(R, ndim, axis, w)[l].shape[3] for l in range(R * ndim - 1)]
        assert max(ranks) <= 3


def test_pure_shifts_are_permutations():
    # w = (0, 0, 1): psi(x + h); every row holds one 1, columns a permutation
    for R, ndim, axis in [(5, 1, 0), (3, 2, 1)]:
        M = T.mpo_dense(T.stencil_mpo(R, ndim, axis, (0.0, 0.0, 1.0)))
        assert set(np.unique(M)) == {0.0, 1.0}
        assert (M.sum(axis=0) == 1).all() and (M.sum(axis=1) == 1).all()
        # applying it 2^R times gives the identity (periodicity)
        P = np.linalg.matrix_power(M, 2 ** R)
        assert np.array_equal(P, np.eye(M.shape[0]))


def plane_wave_tt(R, k):
    """Rank-1 TT of exp(2 pi i k . x) on the interleaved grid: the factor of
    the site holding bit R-1-b of axis a is exp(2 pi i k_a bit 2^(R-1-b) / 2^R)."""
    ndim = len(k)
    cores = []
    for s in range(R * ndim):
        b, a = divmod(s, ndim)
        ph = 2j * np.pi * k[a] * 2.0 ** (R - 1 - b) / 2.0 ** R
        cores.append(np.array([1.0, np.exp(ph)], dtype=complex).reshape(1, 2, 1))
    return cores


@pytest.mark.parametrize("R,k", [(6, (3,)), (4, (1, 5)), (3, (2, 7, 1))])
def test_laplacian_eigenvalue_of_plane_waves(R, k):
    ndim = len(k)
    psi = plane_wave_tt(R, k)
    v = W.tt_full(psi).reshape(-1)
    lam = sum((2.0 * np.cos(2 * np.pi * ka / 2 ** R) - 2.0) * 4.0 ** R for ka in k)
    got = sum(W.tt_full(T.mpo_apply(T.laplacian_mpo(R, ndim, a), psi)).reshape(-1) for a in range(ndim))
    assert np.abs(got - lam * v).max() <= 1e-11 * abs(lam)


def random_mpo(L, d, w, seed):
    rng = np.random.default_rng(seed)
    ranks = [1] + [w] * (L - 1) + [1]
    return [rng.standard_normal((ranks[l], d, d, ranks[l + 1])) for l in range(L)]


def test_mpo_dense_against_core_products():
    L, d = 4, 2
    Wm = random_mpo(L, d, 3, 11)
    M = T.mpo_dense(Wm)
    for s in itertools.product(range(d), repeat=L):
        for t in itertools.product(range(d), repeat=L):
            v = np.ones((1, 1))
            for l in range(L):
                v = v @ Wm[l][:, s[l], t[l], :]
            row = int("".join(map(str, s)), d)
            col = int("".join(map(str, t)), d)
            assert abs(M[row, col] - v[0, 0]) <= 1e-13 * max(1.0, abs(v[0, 0]))


@pytest.mark.parametrize("dtype", [np.float64, np.complex128])
def test_mpo_apply_is_dense_operator_times_vector(dtype):
    L = 7
    Wm = random_mpo(L, 2, 3, 12)
    X = W.random_tt(L, 2, 4, 13, dtype=dtype)
    Z = T.mpo_apply(Wm, X)
    assert [z.shape[2] for z in Z[:-1]] == [3 * 4] * (L - 1)
    ref = T.mpo_dense(Wm) @ W.tt_full(X).reshape(-1)
    got = W.tt_full(Z).reshape(-1)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_linear_cubic_reduces_to_abs2_mul():
    z = np.random.default_rng(4).standard_normal((5, 6)) + 1j
    f = T.linear_cubic([0.0], 1.0)
    assert np.array_equal(f(z), oracle.apply_op("abs2_mul", [z]))


def dense_step(psi_dense, R, ndim, c0, c_lap, c3):
    """Euler step on the grid: roll-based second differences."""
    g = np.empty((2 ** R,) * ndim, dtype=psi_dense.dtype)
    n = psi_dense.size
    for q in range(n):
        g[tuple(quantics_to_coords(q, R, ndim))] = psi_dense[q]
    lap = sum((np.roll(g, -1, a) - 2 * g + np.roll(g, 1, a)) * 4.0 ** R for a in range(ndim))
    y = c0 * g + c_lap * lap + c3 * np.abs(g) ** 2 * g
    out = np.empty_like(psi_dense)
    for q in range(n):
        out[q] = y[tuple(quantics_to_coords(q, R, ndim))]
    return out


@pytest.mark.parametrize("cplx", [False, True])
def test_cubic_step_against_dense_euler_step(cplx):
    R, ndim = 3, 2
    L = R * ndim
    dtype = np.complex128 if cplx else np.float64
    psi = W.random_tt(L, 2, 3, 21, dtype=dtype)
    dt = 1e-3
    if cplx:      # Gross-Pitaevskii: i psi_t = -1/2 Lap psi + |psi|^2 psi
        c0, c_lap, c3 = 1.0, 0.5j * dt, -1j * dt
    else:         # Allen-Cahn: psi_t = eps^2 Lap psi + psi - psi^3
        c0, c_lap, c3 = 1.0 + dt, 1e-2 * dt, -dt
    res, lap = T.cubic_step(psi, R, ndim, c0, c_lap, c3, 1e-13, 64)
    assert res.converged
    ref = dense_step(W.tt_full(psi).reshape(-1), R, ndim, c0, c_lap, c3)
    got = W.tt_full(res.cores).reshape(-1)
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()
    # the step's inputs: ranks of D_a psi are three times those of psi
    assert all(z.shape[2] == 3 * x.shape[2] for a in range(ndim) for z, x in zip(lap[a][:-1], psi[:-1]))
