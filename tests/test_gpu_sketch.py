"""The random index sketch as initial guess (options.sketch_rank, the
RSI-style start of Sec. 2.8) against the oracle: the same initialisation
pivots (rows in order at the drawn columns), the same pivots in every later
prrLU call up to the oracle's first near tie, the same ranks, error
estimates and outputs."""

import numpy as np
import pytest

import oracle
import workloads as W
from helpers import GAP_TIE, rel_max_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
aci = pytest.importorskip("paper_2604_00037_amd")


def _field(R, kmax, s, chi):
    g = W.fourier3d_full(R, kmax, s)
    q = np.ascontiguousarray(W.grid_to_quantics(g, R, 3)).reshape(-1)
    return W.tt_svd(q, 2, chi, rtol=1e-12)


def _compare(gpu, trace):
    assert len(gpu) == len(trace)
    for i, (g, o) in enumerate(zip(gpu, trace)):
        gap = o.get("min_gap")
        if gap is not None and gap < GAP_TIE:
            return i
        assert g["rank"] == o["rank"], (i, o["dir"], o["bond"])
        assert list(g["rows"]) == [int(x) for x in o["rows"]], (i, o["dir"], o["bond"])
        assert list(g["cols"]) == [int(x) for x in o["cols"]], (i, o["dir"], o["bond"])
    return len(trace)


CASES = [("random_pair", 3), ("random_pair", 12), ("random_pair", 40), ("fourier3d", 48),
         ("complex_pair", 20)]


@pytest.mark.parametrize("case,k", CASES)
def test_sketch_start_matches_oracle(case, k):
    print(f"case: sketch init {case} k={k}", flush=True)
    if case == "random_pair":
        x = W.random_pair(L=10, chi=5, seeds=(1001, 1002))
        tol, cap = 1e-12, 25
    elif case == "complex_pair":
        x = W.random_pair(L=9, chi=4, seeds=(1011, 1012), dtype=np.complex128)
        tol, cap = 1e-12, 16
    else:
        x = (_field(3, 3, 21, 16), _field(3, 3, 1021, 16))
        tol, cap = 1e-8, 48
    ref = oracle.aci(list(x), "product", tol, cap, maxiter=20, seed=77, sketch_rank=k, log_gaps=True)
    cores, info = aci.elementwise([to_dev(c) for c in x], "product", tol, cap, maxiter=20, seed=77, sketch_rank=k,
                                  trace=True)
    assert info.init_ranks[1:-1] == ref.init_ranks
    L = len(x[0])
    for rec in info.records[:L - 1]:
        assert rec["kind"] == "init" and list(rec["rows"]) == list(range(rec["m"]))
    n = _compare(info.records, ref.trace)
    print(f"{case}: {n} of {len(ref.trace)} records equal before any near tie", flush=True)
    if n == len(ref.trace):
        assert info.ranks[1:-1] == list(ref.ranks) and info.sweeps == ref.sweeps
        assert info.converged == ref.converged
        y = W.tt_full([c.cpu().numpy() for c in cores])
        assert rel_max_err(y, W.tt_full(ref.cores)) <= 1e-10
    f = W.tt_full(x[0]) * W.tt_full(x[1])
    assert rel_max_err(W.tt_full([c.cpu().numpy() for c in cores]), f) <= max(10 * tol / np.abs(f).max(), 1e-10)


def test_sketch_rank_is_validated():
    x = W.random_pair(L=6, chi=3, seeds=(1, 2))
    with pytest.raises(aci._lib.HipError, match="sketch_rank"):
        aci.elementwise([to_dev(c) for c in x], "product", 1e-12, 8, sketch_rank=-1)
