"""Pins of the random index sketch used as ACI's initial guess (oracle/sketch.py)."""

import numpy as np
import pytest

import oracle
import workloads as W
from oracle.sketch import sketch_init, sketch_ranks


def test_sketch_ranks_follow_caps():
    # k, maxrank and the number of index points on either side all cap the ranks
    assert sketch_ranks([2] * 6, 5, 64) == [1, 2, 4, 5, 4, 2, 1]
    assert sketch_ranks([2] * 6, 8, 3) == [1, 2, 3, 3, 3, 2, 1]
    assert sketch_ranks([3, 2, 4], 100, 100) == [1, 3, 4, 1]


def _init_records(res, L):
    return [t for t in res.trace if t["dir"] == "init"]   # sites L .. 2


@pytest.mark.parametrize("k", [3, 12, 40])
def test_initialisation_selects_the_drawn_points_in_row_order(k):
    """Every initialisation LDU takes its pivots at rows 0, 1, 2, ... in
    order, at distinct columns, and the resulting right index sets have the
    sketch's ranks, are nested and distinct."""
    x1, x2 = W.random_pair(L=10, chi=5, seeds=(1001, 1002))
    res = oracle.aci([x1, x2], "product", 1e-12, 25, maxiter=1, seed=77, sketch_rank=k)
    dims = [c.shape[1] for c in x1]
    rho = sketch_ranks(dims, k, 25)
    assert res.init_ranks == rho[1:-1]
    recs = _init_records(res, 10)
    assert len(recs) == 9
    J = {11: [()]}
    for t in recs:
        l = t["bond"]
        m, n = t["shape"]
        assert m == rho[l - 1] and n == dims[l - 1] * rho[l]
        assert list(t["rows"]) == list(range(m))
        assert len(set(int(q) for q in t["cols"])) == m
        c = len(J[l + 1])
        J[l] = [(int(q) // c,) + J[l + 1][int(q) % c] for q in t["cols"]]
        assert len(set(J[l])) == len(J[l])
        assert all(j[1:] in J[l + 1] for j in J[l])


def test_draws_are_uniform_without_replacement():
    """Over 3000 seeds every column of a site is drawn with frequency
    rho_{l-1} / (d rho_l), within five binomial standard deviations."""
    dims, k, trials = [2] * 6, 5, 3000
    rho = sketch_ranks(dims, k, 64)
    l = 4                                    # site 4 of 6: 4 rows out of 2 * 4 = 8 columns
    n, draws = dims[l - 1] * rho[l], rho[l - 1]
    counts = np.zeros(n)
    for seed in range(trials):
        core = sketch_init(dims, k, 64, seed)[l - 1]
        nz = np.argwhere(core != 0)
        assert len(nz) == draws and len({(s, b) for _, s, b in nz}) == draws
        for _, s, b in nz:
            counts[s * rho[l] + b] += 1
    p = draws / n
    sd = np.sqrt(trials * p * (1 - p))
    assert np.all(np.abs(counts - trials * p) <= 5 * sd), counts


def test_aci_from_the_sketch_reaches_the_exact_product():
    """The 12-site random product (exact rank 64 at the middle) started from
    a sketch of size 64: every one of the 4096 entries within 1e-12."""
    x1, x2 = W.random_pair(L=12, chi=8, seeds=(1001, 1002))
    res = oracle.aci([x1, x2], "product", 1e-12, 64, maxiter=20, seed=1003, sketch_rank=64)
    f = W.tt_full(x1) * W.tt_full(x2)
    y = W.tt_full(res.cores)
    assert res.converged
    assert np.abs(y - f).max() <= 1e-12 * np.abs(f).max()
