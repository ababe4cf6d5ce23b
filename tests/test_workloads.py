"""Input generators: the torch (device) path of the quantics reordering
agrees with the numpy definition (a transpose of the bit axes), and the
central-difference derivative of a Fourier field is the grid stencil."""

import numpy as np
import pytest

import workloads as W
from workloads.fields import grid_to_quantics, quantics_to_grid

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("R,ndim", [(3, 3), (4, 2), (2, 3), (5, 1)])
def test_torch_quantics_order_matches_numpy(R, ndim):
    F = np.random.default_rng(R * 10 + ndim).standard_normal((2 ** R,) * ndim)
    ref = np.ascontiguousarray(grid_to_quantics(F, R, ndim)).reshape(-1)
    got = grid_to_quantics(torch.from_numpy(F), R, ndim).numpy()
    assert np.array_equal(ref, got)
    assert np.array_equal(quantics_to_grid(got, R, ndim), F)


def test_interleaved_site_holds_axis_bit():
    # site ndim*b + a holds bit b (most significant first) of axis a
    R, ndim = 3, 2
    n = 2 ** R
    x = np.arange(n)
    F = x[:, None] * 1000 + x[None, :]          # encodes (i0, i1)
    Q = grid_to_quantics(F, R, ndim)
    for idx in np.ndindex(*Q.shape):
        i0 = sum(idx[ndim * b + 0] << (R - 1 - b) for b in range(R))
        i1 = sum(idx[ndim * b + 1] << (R - 1 - b) for b in range(R))
        assert Q[idx] == i0 * 1000 + i1


def test_central_difference_derivative_is_the_grid_stencil():
    """deriv="central" equals (u(x+h e_j) - u(x-h e_j)) / 2h of the sampled
    field on the periodic grid, for every axis."""
    R = 4
    u = W.fourier3d_full(R, 3, 3001)
    for j in range(3):
        du = W.fourier3d_full(R, 3, 3001, deriv_axis=j, deriv="central")
        fd = (np.roll(u, -1, j) - np.roll(u, 1, j)) * 2 ** R / 2
        assert np.abs(du - fd).max() <= 1e-13 * np.abs(fd).max()


def test_tt_round_keeps_the_tensor_and_caps_ranks():
    """Rounding a TT with redundant ranks (a sum of two copies of a random TT,
    rank 2r) gives the same tensor at rank r, and a cap below the exact rank
    gives the best-approximation error the dropped singular values predict."""
    x = W.random_tt(8, 2, 5, 77)
    def block_diag(c):
        z = np.zeros_like(c)
        return np.concatenate([np.concatenate([c, z], axis=2), np.concatenate([z, c], axis=2)], axis=0)
    dbl = [np.concatenate([x[0], x[0]], axis=2)] + [block_diag(c) for c in x[1:-1]] + \
          [np.concatenate([x[-1], x[-1]], axis=0)]
    full = W.tt_full(dbl)
    assert np.abs(full - 2 * W.tt_full(x)).max() <= 1e-13 * np.abs(full).max()
    r = W.tt_round(dbl, 64, rtol=1e-12)
    assert max(W.tt_ranks(r)) <= 5
    assert np.abs(W.tt_full(r) - full).max() <= 1e-12 * np.abs(full).max()
    # capped: the error is bounded by the root of the sum of the squared dropped values over the bonds
    y = W.random_tt(8, 2, 6, 78)
    f = W.tt_full(y)
    r3 = W.tt_round(y, 3)
    assert max(W.tt_ranks(r3)) <= 3
    err = np.linalg.norm(W.tt_full(r3) - f)
    bound = 0.0
    for b in range(1, 8):
        sv = np.linalg.svd(f.reshape(2 ** b, -1), compute_uv=False)
        bound += (sv[3:] ** 2).sum()
    assert err <= np.sqrt(bound) * (1 + 1e-10)
