"""Pins of the oracle's 2-site TCI (oracle/tci.py) against what the
mathematics fixes: exact recovery of tensors of low TT rank (brute force
over all entries), rank one for product functions, the interpolation
property at the bond-1 crosses, nested right index sets, and a quantics
Gaussian against its closed form."""

import numpy as np
import pytest

import oracle
import workloads as W


def full_of(f, dims):
    grids = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    pts = np.stack([g.reshape(-1) for g in grids], axis=1)
    return f(pts).reshape(dims)


@pytest.mark.parametrize("L,chi", [(8, 3), (10, 5)])
def test_recovers_low_rank_tensors_exactly(L, chi):
    x, _ = W.random_pair(L=L, chi=chi, seeds=(4101 + L, 4201 + L))
    f = lambda pts: W.tt_eval(x, pts)
    res = oracle.tci(f, [2] * L, 1e-12, 64)
    assert res.converged
    ref = W.tt_full(x)
    got = W.tt_full(res.cores)
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()
    # no bond needs more than the input's rank
    assert all(r <= x[l].shape[2] for l, r in enumerate(res.ranks))


def test_product_function_has_rank_one():
    rng = np.random.default_rng(3)
    L, d = 9, 3
    g = rng.uniform(0.5, 2.0, (L, d))
    f = lambda pts: np.prod(g[np.arange(L)[None, :], pts], axis=1)
    res = oracle.tci(f, [d] * L, 1e-13, 8)
    assert res.ranks == [1] * (L - 1)
    ref = full_of(f, [d] * L)
    assert np.abs(W.tt_full(res.cores) - ref).max() <= 1e-13 * np.abs(ref).max()


def test_interpolation_at_bond1_crosses_and_nested_right_sets():
    x, _ = W.random_pair(L=10, chi=6, seeds=(4301, 4302))
    f = lambda pts: W.tt_eval(x, pts)
    res = oracle.tci(f, [2] * 10, 1e-6, 12, maxiter=6)
    # the output reproduces f exactly on I_1 x J_2 (the bond-1 factorisation)
    pts = np.array([i + j for i in res.I[1] for j in res.J[2]])
    assert np.abs(W.tt_eval(res.cores, pts) - f(pts)).max() <= 1e-11 * np.abs(f(pts)).max()
    # right index sets are nested: every J_{l+1} entry continues with a J_{l+2} entry
    for l in range(1, 9):
        nxt = set(res.J[l + 2])
        assert all(j[1:] in nxt for j in res.J[l + 1])


def test_quantics_gaussian_against_closed_form():
    R = 12
    w = np.array([2.0 ** -(l + 1) for l in range(R)])
    f = lambda pts: np.exp(-((pts @ w) - 0.5) ** 2 / (2 * 0.05 ** 2))
    res = oracle.tci(f, [2] * R, 1e-10, 64)
    assert res.converged
    ref = full_of(f, [2] * R).reshape(-1)
    got = W.tt_full(res.cores).reshape(-1)
    assert np.abs(got - ref).max() <= 1e-8
    assert max(res.ranks) <= 16


def test_pivots_seed_the_index_sets():
    L = 6
    f = lambda pts: 1.0 + pts.sum(axis=1).astype(float)
    piv = [(1, 0, 1, 0, 1, 0), (0, 1, 1, 0, 0, 1)]
    res = oracle.tci(f, [2] * L, 1e-14, 16, maxiter=1, pivots=piv)
    # f is a sum of one-site terms: TT rank 2
    assert max(res.ranks) <= 2
    ref = full_of(f, [2] * L)
    assert np.abs(W.tt_full(res.cores) - ref).max() <= 1e-12 * np.abs(ref).max()
