"""A general elementwise f (ACI_OP_CUSTOM): the two-site tensors of every
input are contracted on the matrix cores, then the caller's f (here torch
operations on the library's stream) writes the matrix the LDU factorises.
Against the oracle running the same f on NumPy with the same operations in
the same order: identical pivots, ranks, error estimates and index sets."""

import numpy as np
import pytest

import oracle
import workloads as W
from helpers import compare_records, rel_max_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
aci = pytest.importorskip("paper_2604_00037_amd")


def f_np(u, v):
    return u * v + u          # (u*v) + u, rounded after each operation


def f_dev(u, v):
    return torch.add(torch.mul(u, v), u)


def test_custom_f_matches_oracle():
    x1, x2 = W.random_pair(L=10, chi=5, seeds=(2801, 2802))
    ref = oracle.aci([x1, x2], f_np, 1e-12, 40, seed=3, log_gaps=True)
    cores, info = aci.elementwise([to_dev(x1), to_dev(x2)], f_dev, 1e-12, 40, seed=3, trace=True)
    n = compare_records(info.records, ref.trace, "custom f")
    assert n == len(ref.trace)
    assert info.ranks[1:-1] == ref.ranks and info.converged == ref.converged
    for l in range(1, 10):
        assert info.I[l] == [tuple(int(v) for v in t) for t in ref.I[l]]
    y = W.tt_full([c.cpu().numpy() for c in cores])
    exact = f_np(W.tt_full(x1), W.tt_full(x2))
    assert rel_max_err(y, W.tt_full(ref.cores)) <= 1e-10
    assert rel_max_err(y, exact) <= 1e-10


def test_custom_f_complex_and_nonpolynomial():
    psi = W.gp_field(R=5, chi=32, seed=5001, width_scale=2.0)
    f = lambda z: torch.exp(1j * z.real) * z          # a phase rotation: not in the built-in ops
    cores, info = aci.elementwise([to_dev(psi)], f, 1e-9, 64, seed=6)
    assert info.converged
    z = W.tt_full(psi)
    exact = np.exp(1j * z.real) * z
    y = W.tt_full([c.cpu().numpy() for c in cores])
    assert np.abs(y - exact).max() <= 100 * 1e-9 * max(1.0, np.abs(exact).max())


def test_custom_f_in_a_joint_batch_and_with_graphs_requested():
    prods = []
    for b in range(3):
        x1, x2 = W.random_pair(L=10, chi=4 + b, seeds=(2811 + 2 * b, 2812 + 2 * b))
        prods.append([to_dev(x1), to_dev(x2)])
    res = aci.elementwise_batched(prods, f_dev, 1e-12, 40, seed=4, use_graph=True, mode="joint")
    for b, (cores, info) in enumerate(res):
        sc, si = aci.elementwise(prods[b], f_dev, 1e-12, 40, seed=4)
        assert info.ranks == si.ranks
        for p, q in zip(cores, sc):
            assert torch.equal(p, q)


def test_custom_f_failure_is_reported():
    x1, x2 = W.random_pair(L=8, chi=3, seeds=(2821, 2822))

    def bad(u, v):
        raise ValueError("f broke")
    with pytest.raises(ValueError, match="f broke"):
        aci.elementwise([to_dev(x1), to_dev(x2)], bad, 1e-12, 20, seed=1)
