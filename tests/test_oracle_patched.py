"""Pins of the oracle's patched ACI (oracle/patched.py): the restriction of
an input TT against slicing the dense tensor, max_depth 0 against the
unpatched ACI, the kept prefixes partitioning the index space, and the
assembled patches against the exact product (brute force over all
entries) when one TT at the rank cap cannot reach the tolerance."""

import itertools

import numpy as np
import pytest

import oracle
from oracle import patched as P
import workloads as W


@pytest.mark.parametrize("prefix", [(), (1,), (0, 1, 1), (2, 0)])
def test_restriction_is_the_slice(prefix):
    X = W.random_tt(6, 3, 4, 71, dtype=np.complex128)
    got = W.tt_full(P.restrict(X, prefix))
    assert np.abs(got - W.tt_full(X)[prefix]).max() <= 1e-13


def test_depth_zero_is_the_unpatched_aci():
    x1, x2 = W.random_pair(L=10, chi=5, seeds=(3101, 3102))
    pts = P.patched_aci([x1, x2], "product", 1e-12, 40, 0, seed=3)
    ref = oracle.aci([x1, x2], "product", 1e-12, 40, seed=3)
    assert len(pts) == 1 and pts[0].prefix == ()
    assert pts[0].result.ranks == ref.ranks
    for a, b in zip(pts[0].result.cores, ref.cores):
        assert np.array_equal(a, b)


def is_partition(prefixes, dims):
    covered = 0
    for p in prefixes:
        covered += int(np.prod(dims[len(p):]))
        for q in prefixes:
            if q != p and len(q) < len(p) and p[:len(q)] == q:
                return False
    return covered == int(np.prod(dims))


@pytest.mark.parametrize("cplx", [False, True])
def test_patches_reach_the_tolerance_the_cap_denies(cplx):
    dtype = np.complex128 if cplx else np.float64
    L = 10
    x1 = W.random_tt(L, 2, 6, 3111, dtype=dtype)
    x2 = W.random_tt(L, 2, 6, 3112, dtype=dtype)
    exact = W.tt_full(x1) * W.tt_full(x2)
    cap = 8
    whole = oracle.aci([x1, x2], "product", 1e-10, cap, seed=4)
    assert not whole.converged                      # rank 36 products need more than 8
    pts = P.patched_aci([x1, x2], "product", 1e-10, cap, 4, seed=4)
    prefixes = [p.prefix for p in pts]
    assert is_partition(prefixes, [2] * L)
    assert all(p.result.converged for p in pts)
    assert max(len(p) for p in prefixes) <= 4 and len(pts) > 1
    assert all(max(p.result.ranks) <= cap for p in pts)
    got = P.assemble(pts, [2] * L)
    assert np.abs(got - exact).max() <= 1e-9 * np.abs(exact).max()


def test_low_rank_products_need_no_patches():
    x1, x2 = W.random_pair(L=9, chi=3, seeds=(3121, 3122))
    pts = P.patched_aci([x1, x2], "product", 1e-12, 16, 3, seed=2)
    assert [p.prefix for p in pts] == [()]


def test_max_depth_keeps_unconverged_patches():
    x1 = W.random_tt(8, 2, 6, 3131)
    x2 = W.random_tt(8, 2, 6, 3132)
    pts = P.patched_aci([x1, x2], "product", 1e-12, 2, 1, seed=5)
    assert [p.prefix for p in pts] == [(0,), (1,)]
    assert not all(p.result.converged for p in pts)
    with pytest.raises(ValueError):
        P.patched_aci([x1, x2], "product", 1e-12, 2, 7)
