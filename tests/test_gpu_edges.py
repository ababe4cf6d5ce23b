"""Edge cases of the whole sweep against the oracle: the shortest chain
(L = 2, also with d = 4), the longest (L = ACI_MAX_SITES = 128, checked at
sampled points) and one site more (rejected), rank-1 inputs (rank-1
output), a result that is exactly zero (the zero path of the LDU), the rank
cap 1, and the largest and one more than the largest number of inputs."""

import numpy as np
import pytest

import oracle
import workloads as W
from helpers import compare_records, rel_max_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
aci = pytest.importorskip("paper_2604_00037_amd")


def both(inputs, op, tol, maxrank, seed=3, maxiter=20):
    ref = oracle.aci(inputs, op, tol, maxrank, maxiter=maxiter, seed=seed, log_gaps=True)
    cores, info = aci.elementwise([to_dev(x) for x in inputs], op, tol, maxrank, maxiter=maxiter, seed=seed,
                                  trace=True)
    n = compare_records(info.records, ref.trace)
    assert n == len(ref.trace)
    assert info.ranks[1:-1] == ref.ranks and info.converged == ref.converged
    return ref, [c.cpu().numpy() for c in cores], info


@pytest.mark.parametrize("d", [2, 4])
def test_two_sites(d):
    x1 = W.random_tt(2, d, 3, 4001)
    x2 = W.random_tt(2, d, 2, 4002)
    ref, cores, info = both([x1, x2], "product", 1e-13, 16)
    y = W.tt_full(cores)
    assert rel_max_err(y, W.tt_full(x1) * W.tt_full(x2)) <= 1e-12


def unit_phase_tt(L, seed, terms=2):
    """Sum of `terms` rank-1 TTs whose factors are unit-modulus phases: every
    entry has modulus <= terms at any length (random real cores would span
    many orders of magnitude over 2^128 entries)."""
    rng = np.random.default_rng(seed)
    cores = []
    for l in range(L):
        ph = np.exp(2j * np.pi * rng.uniform(0, 1, (terms, 2)))
        if l == 0:
            c = ph.T[None, :, :]
        elif l == L - 1:
            c = ph[:, :, None]
        else:
            c = np.zeros((terms, 2, terms), complex)
            for t in range(terms):
                c[t, :, t] = ph[t]
        cores.append(np.ascontiguousarray(c))
    return cores


def test_longest_chain_and_one_site_more():
    L = 128
    x1, x2 = unit_phase_tt(L, 4011), unit_phase_tt(L, 4012)
    ref, cores, info = both([x1, x2], "product", 1e-10, 8, maxiter=6)
    assert info.converged and max(info.ranks) == 4
    pts = np.random.default_rng(4).integers(0, 2, (512, L))
    f = W.tt_eval(x1, pts) * W.tt_eval(x2, pts)
    assert np.abs(W.tt_eval(cores, pts) - W.tt_eval(ref.cores, pts)).max() <= 1e-10 * np.abs(f).max()
    assert np.abs(W.tt_eval(cores, pts) - f).max() <= 1e-10 * np.abs(f).max()
    y1 = unit_phase_tt(L + 1, 4013)
    with pytest.raises(aci._lib.HipError, match="LIMIT"):
        aci.elementwise([to_dev(y1)], "sum", 1e-12, 4)


def test_rank_one_inputs_give_rank_one_output():
    x1 = W.random_tt(12, 3, 1, 4021, dtype=np.complex128)
    x2 = W.random_tt(12, 3, 1, 4022, dtype=np.complex128)
    ref, cores, info = both([x1, x2], "product", 1e-13, 16)
    assert info.ranks[1:-1] == [1] * 11
    assert rel_max_err(W.tt_full(cores), W.tt_full(x1) * W.tt_full(x2)) <= 1e-12


def test_exactly_zero_result():
    x = W.random_tt(8, 2, 3, 4031)
    neg = [c.copy() for c in x]
    neg[0] = -neg[0]
    ref, cores, info = both([x, neg], "sum", 1e-12, 16)
    assert info.ranks[1:-1] == [1] * 7
    assert all(e == 0.0 for e in info.eps)
    assert np.all(W.tt_full(cores) == 0.0)


def test_rank_cap_one():
    x1, x2 = W.random_pair(L=9, chi=4, seeds=(4041, 4042))
    ref, cores, info = both([x1, x2], "product", 1e-12, 1, maxiter=3)
    assert info.ranks[1:-1] == [1] * 8 and not info.converged
    assert rel_max_err(W.tt_full(cores), W.tt_full(ref.cores)) <= 1e-10


def test_most_inputs_and_one_more():
    xs = [W.left_orthogonalise(W.random_tt(8, 2, 2, 4051 + i)) for i in range(4)]
    ref, cores, info = both(xs, "product", 1e-12, 64)
    exact = np.prod([W.tt_full(x) for x in xs], axis=0)
    assert rel_max_err(W.tt_full(cores), exact) <= 1e-10
    with pytest.raises(aci._lib.HipError, match="LIMIT"):
        aci.elementwise([to_dev(x) for x in xs + xs[:1]], "sum", 1e-12, 8)
