"""End-to-end parity of the HIP sweep (aci_elementwise) with the oracle:
identical pivot sets for every prrLU call of the run (initialisation and
both half sweeps), identical ranks, error estimates and convergence, and
output tensors within 1e-10 relative of the oracle's."""

import numpy as np
import pytest

import oracle
import workloads as W
from helpers import compare_records, rel_max_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
aci = pytest.importorskip("paper_2604_00037_amd")


def run_both(inputs, op, tol, maxrank, maxiter=20, init=None, seed=0, rule="exclusive"):
    ref = oracle.aci(inputs, op, tol, maxrank, maxiter=maxiter, init=init, seed=seed, rule=rule,
                     log_gaps=True)
    cores, info = aci.elementwise([to_dev(x) for x in inputs], op, tol, maxrank, maxiter=maxiter,
                                  init=None if init is None else to_dev(init), seed=seed,
                                  stop_rule=rule, trace=True)
    return ref, [c.cpu().numpy() for c in cores], info


def check(ref, cores, info, label, full=True):
    n = compare_records(info.records, ref.trace, label)
    assert n == len(ref.trace), f"{label}: pivots diverged at a near tie (record {n})"
    assert info.ranks[1:-1] == ref.ranks
    assert info.init_ranks[1:-1] == ref.init_ranks
    assert info.sweeps == ref.sweeps and info.converged == ref.converged
    np.testing.assert_allclose(info.eps, ref.eps, rtol=1e-9, atol=1e-14)
    for g, o in zip(cores, ref.cores):
        assert g.shape == o.shape
    # the nested index sets the result reports are the oracle's
    for l in range(1, len(cores)):
        assert info.I[l] == [tuple(int(v) for v in t) for t in ref.I[l]], f"{label}: I_{l}"
        assert info.J[l + 1] == [tuple(int(v) for v in t) for t in ref.J[l + 1]], f"{label}: J_{l + 1}"
    if full:
        y = W.tt_full(cores)
        yr = W.tt_full(ref.cores)
        assert rel_max_err(y, yr) <= 1e-10, label


def test_random_pair_default_init():
    x1, x2 = W.random_pair()
    ref, cores, info = run_both([x1, x2], "product", 1e-12, 64, seed=1003)
    check(ref, cores, info, "random pair L=12 chi=8")
    f = W.tt_full(x1) * W.tt_full(x2)
    assert rel_max_err(W.tt_full(cores), f) <= 1e-12
    assert info.ranks[1:-1] == [2, 4, 8, 16, 32, 64, 32, 16, 8, 4, 2]


def test_index_sets_without_trace():
    """Untraced runs keep the pivots of the last sweep per bond; the index
    sets built from them equal the oracle's."""
    x1, x2 = W.random_pair(L=10, chi=6, seeds=(1021, 1022))
    ref = oracle.aci([x1, x2], "product", 1e-12, 36, seed=1023, log_gaps=True)
    assert min(t["min_gap"] for t in ref.trace if t["min_gap"] is not None) > 1e-10
    cores, info = aci.elementwise([to_dev(x1), to_dev(x2)], "product", 1e-12, 36, seed=1023)
    assert info.ranks[1:-1] == ref.ranks
    for l in range(1, 10):
        assert info.I[l] == [tuple(int(v) for v in t) for t in ref.I[l]]
        assert info.J[l + 1] == [tuple(int(v) for v in t) for t in ref.J[l + 1]]
        assert len(info.I[l]) == len(info.J[l + 1]) == info.ranks[l]


def test_random_pair_explicit_init():
    x1, x2 = W.random_pair(L=10, chi=6, seeds=(1011, 1012))
    init = W.random_init(oracle.default_init_ranks([x1, x2], 36), 2, seed=1013)
    ref, cores, info = run_both([x1, x2], "product", 1e-12, 36, init=init)
    check(ref, cores, info, "explicit init")


@pytest.mark.parametrize("op,n_in", [("sum", 2), ("product", 3), ("product", 1), ("abs2_mul", 1)])
def test_ops_and_arity(op, n_in):
    xs = [W.left_orthogonalise(W.random_tt(9, 2, 4, seed=200 + i)) for i in range(n_in)]
    ref, cores, info = run_both(xs, op, 1e-12, 80, seed=7)
    check(ref, cores, info, f"{op} N={n_in}")


def test_rank_capped_not_converged():
    x1, x2 = W.random_pair(L=12, chi=8, seeds=(1021, 1022))
    ref, cores, info = run_both([x1, x2], "product", 1e-12, 12, maxiter=3, seed=3)
    check(ref, cores, info, "capped")
    assert not info.converged and info.status == 1


def test_literal_rule():
    x1, x2 = W.random_pair(L=9, chi=5, seeds=(1031, 1032))
    ref, cores, info = run_both([x1, x2], "product", 1e-10, 25, seed=4, rule="literal")
    check(ref, cores, info, "literal")


def test_ragged_local_dimensions_and_odd_ranks():
    rng = np.random.default_rng(8)
    L = 7
    dims = [2, 3, 2, 4, 3, 2, 3]
    xs = []
    for n in range(2):
        ranks = [1, 3, 5, 7, 5, 6, 2, 1]
        xs.append([rng.standard_normal((ranks[l], dims[l], ranks[l + 1])) for l in range(L)])
    ref, cores, info = run_both(xs, "product", 1e-12, 40, seed=9)
    check(ref, cores, info, "ragged")


def test_fourier3d_small_grid():
    """3D random Fourier fields (k^-5/3 spectrum) on a 16^3 quantics grid."""
    u, v = W.fourier3d_pair(R=4, kmax=4, chi=24, seeds=(2001, 2002))
    ref, cores, info = run_both([u, v], "product", 1e-8, 48, seed=11)
    check(ref, cores, info, "fourier3d R=4")


def test_nan_input_is_reported():
    x1, x2 = W.random_pair(L=6, chi=3, seeds=(1041, 1042))
    x1 = [c.copy() for c in x1]
    x1[2][0, 0, 0] = np.nan
    with pytest.raises(Exception, match="NUMERIC"):
        aci.elementwise([to_dev(x1), to_dev(x2)], "product", 1e-10, 16)


def test_invalid_arguments_are_rejected():
    x1, x2 = W.random_pair(L=6, chi=3, seeds=(1043, 1044))
    with pytest.raises(Exception, match="INVALID"):
        aci.elementwise([to_dev(x1), to_dev(x2)], "abs2_mul", 1e-10, 16)
    with pytest.raises(Exception, match="INVALID"):
        aci.elementwise([to_dev(x1)], "product", -1.0, 16)
    with pytest.raises(Exception, match="LIMIT"):
        aci.elementwise([to_dev(x1)], "product", 1e-10, 100000)


def test_repeat_runs_are_bitwise_identical():
    x1, x2 = W.random_pair(L=10, chi=6, seeds=(1051, 1052))
    a, ia = aci.elementwise([to_dev(x1), to_dev(x2)], "product", 1e-10, 30, seed=5)
    b, ib = aci.elementwise([to_dev(x1), to_dev(x2)], "product", 1e-10, 30, seed=5)
    assert ia.ranks == ib.ranks
    for p, q in zip(a, b):
        assert torch.equal(p, q)


def test_session_launch_log_matches_sweep_stats():
    """The per-launch log of a profiled sweep: one LDU, two contractions (the
    fresh environment and the two-site tensors) and one gather per local
    update, and per-class sums equal to the call's statistics."""
    x1, x2 = W.random_pair(L=10, chi=6, seeds=(1061, 1062))
    L = len(x1)
    s = aci.Session([to_dev(x1), to_dev(x2)], "product", 1e-10, 30, maxiter=3, seed=7,
                    fixed_sweeps=True, profile=True)
    try:
        st = s.sweep(2)
        log = s.launches()
    finally:
        s.close()
    assert len(log) == 2 * 4 * 2 * (L - 1)
    for sw in (st["sweeps_done"] - 2, st["sweeps_done"] - 1):
        for u in range(2 * (L - 1)):
            kinds = sorted((r["kind"], r["part"]) for r in log if r["sweep"] == sw and r["update"] == u)
            assert kinds == [("contract", 1), ("contract", 2), ("gather", 0), ("prrlu", 0)]
    for i, kind in enumerate(("prrlu", "contract")):
        assert sum(r["flops"] for r in log if r["kind"] == kind) == pytest.approx(st["flops"][i], rel=1e-12)
    for i, kind in enumerate(("prrlu", "contract", "gather")):
        assert sum(r["us"] for r in log if r["kind"] == kind) == pytest.approx(1e3 * st["kernel_ms"][i], rel=1e-4)
    assert all(r["kernel"].startswith("prrlu_kernel<") for r in log if r["kind"] == "prrlu")


# ------------------------------------------------------------ precision ladder
@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_mixed_precision_ladder_random_pair(precision):
    """Low-precision sweeps, then FP64 sweeps (the last allowed sweep is
    FP64): the converged result reconstructs the exact product like the FP64
    run, within 1e-10 of the oracle's output."""
    x1, x2 = W.random_pair()
    ref = oracle.aci([x1, x2], "product", 1e-12, 64, seed=1003)
    cores, info = aci.elementwise([to_dev(x1), to_dev(x2)], "product", 1e-12, 64, seed=1003,
                                  precision=precision)
    assert info.converged
    y = W.tt_full([c.cpu().numpy() for c in cores])
    assert rel_max_err(y, W.tt_full(ref.cores)) <= 1e-10
    assert rel_max_err(y, W.tt_full(x1) * W.tt_full(x2)) <= 1e-10
    assert info.ranks[1:-1] == ref.ranks


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_mixed_precision_ladder_gaussians_at_1e8(precision):
    """Product of two Gaussians (section 3.1) at tol 1e-8: the mixed-precision
    run converges and both it and the oracle are within 10 tol of the closed
    form; their outputs agree within 1e-7 relative."""
    L = 12
    gp, gm, h = W.gaussian_pair_full(L)
    tp = W.tt_svd(gp, 2, 64, rtol=1e-15)
    tm = W.tt_svd(gm, 2, 64, rtol=1e-15)
    ref = oracle.aci([tp, tm], "product", 1e-8, 64, seed=11)
    cores, info = aci.elementwise([to_dev(tp), to_dev(tm)], "product", 1e-8, 64, seed=11,
                                  precision=precision)
    assert info.converged
    y = W.tt_full([c.cpu().numpy() for c in cores]).reshape(-1)
    yr = W.tt_full(ref.cores).reshape(-1)
    assert np.abs(y - h).max() <= 10 * 1e-8
    assert np.abs(yr - h).max() <= 10 * 1e-8
    assert rel_max_err(y, yr) <= 1e-7


def test_session_ladder_switches_to_fp64():
    x1, x2 = W.random_pair(L=10, chi=6, seeds=(1071, 1072))
    s = aci.Session([to_dev(x1), to_dev(x2)], "product", 1e-10, 36, maxiter=10, seed=3,
                    precision="fp32", low_precision_sweeps=2, fixed_sweeps=True)
    try:
        precs = [s.sweep(1)["last_precision"] for _ in range(4)]
    finally:
        s.close()
    assert precs[0] == "fp32"
    assert precs[2:] == ["fp64", "fp64"]
    s = aci.Session([to_dev(x1), to_dev(x2)], "product", 1e-10, 36, maxiter=10, seed=3,
                    precision="bf16x3", low_precision_sweeps=-1, fixed_sweeps=True)
    try:
        precs = [s.sweep(1)["last_precision"] for _ in range(3)]
    finally:
        s.close()
    assert precs == ["bf16x3"] * 3
