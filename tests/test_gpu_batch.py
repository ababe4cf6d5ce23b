"""Batches (several products advanced together: joint mode with one LDU
launch per local update and every product on its own XCD, overlapped mode
with one stream per product, serial mode) and hipGraph replay of sweeps,
through the C ABI.

The kernels of a batch are the same as those of a single run and every
result element is produced by the same operations whatever the launch
placement, so batched outputs must equal separate runs bit for bit; separate
runs are in turn checked against the oracle (test_gpu_aci.py and below)."""

import numpy as np
import pytest

import oracle
import workloads as W
from helpers import rel_max_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
aci = pytest.importorskip("paper_2604_00037_amd")


def products_small():
    out = []
    for b, (chi, s) in enumerate([(4, 2101), (6, 2103), (5, 2105), (3, 2107)]):
        x1, x2 = W.random_pair(L=10, chi=chi, seeds=(s, s + 1))
        out.append([x1, x2])
    return out


def assert_same(a, b):
    assert len(a) == len(b)
    for p, q in zip(a, b):
        assert p.shape == q.shape
        assert torch.equal(p, q)


def test_batch_equals_separate_runs_and_oracle():
    prods = products_small()
    dev = [[to_dev(x) for x in p] for p in prods]
    res = aci.elementwise_batched(dev, "product", 1e-12, 40, seed=9)
    for b, (p, (cores, info)) in enumerate(zip(prods, res)):
        sc, si = aci.elementwise(dev[b], "product", 1e-12, 40, seed=9)
        assert info.ranks == si.ranks and info.sweeps == si.sweeps and info.converged == si.converged
        assert_same(cores, sc)
        ref = oracle.aci(p, "product", 1e-12, 40, seed=9)
        assert info.ranks[1:-1] == ref.ranks
        y = W.tt_full([c.cpu().numpy() for c in cores])
        assert rel_max_err(y, W.tt_full(ref.cores)) <= 1e-10


def test_batch_of_ten_shares_xcds_and_differs_in_length():
    """Ten overlapping products with a common group cap; one product has a
    different number of sites; the larger products need several
    cooperating groups per LDU."""
    prods = []
    for b in range(10):
        L = 12 if b != 3 else 9
        chi = 10 if b % 2 == 0 else 7
        x1, x2 = W.random_pair(L=L, chi=chi, seeds=(2200 + 2 * b, 2201 + 2 * b))
        prods.append([x1, x2])
    dev = [[to_dev(x) for x in p] for p in prods]
    B = aci.Batch(dev, "product", 1e-11, 100, maxiter=12, seed=4)
    try:
        B.sweep(12)
        got = [B.result(b) for b in range(10)]
        place = [B.info(b) for b in range(10)]
    finally:
        B.close()
    # overlapping products: groups spread over the XCDs, one cap for all,
    # small enough that every XCD holds all of them (ceil(cap/8) each)
    assert all(x == -1 for x, _ in place)
    caps = {g for _, g in place}
    assert len(caps) == 1
    cap = caps.pop()
    assert cap >= 8 and 10 * (-(-cap // 8)) <= 32
    for b in range(10):
        sc, si = aci.elementwise(dev[b], "product", 1e-11, 100, maxiter=12, seed=4)
        cores, info = got[b]
        assert info.ranks == si.ranks and info.converged == si.converged
        assert_same(cores, sc)
        if b in (0, 3):
            f = W.tt_full(prods[b][0]) * W.tt_full(prods[b][1])
            assert rel_max_err(W.tt_full([c.cpu().numpy() for c in cores]), f) <= 1e-9


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_session_graph_replays_match_eager(precision):
    """Every replay of a captured sweep, with eager work and synchronisation
    in between, gives the eager sweep's state bit for bit."""
    x1, x2 = W.random_pair(L=12, chi=9, seeds=(2301, 2302))
    d = [to_dev(x1), to_dev(x2)]
    kw = dict(maxiter=6, seed=5, fixed_sweeps=True, precision=precision, low_precision_sweeps=2)
    g = aci.Session(d, "product", 1e-11, 81, use_graph=True, **kw)
    e = aci.Session(d, "product", 1e-11, 81, use_graph=False, **kw)
    try:
        for it in range(6):
            sg = g.sweep(1)
            se = e.sweep(1)
            assert sg["ranks"] == se["ranks"] and sg["last_precision"] == se["last_precision"]
            cg, ig = g.result()
            ce, ie = e.result()
            assert ig.eps == ie.eps
            assert_same(cg, ce)
            # eager work of the program between replays
            t = torch.randn(1000, device="cuda")
            assert torch.isfinite((t * t).sum())
            torch.cuda.synchronize()
    finally:
        g.close()
        e.close()


def test_batch_graph_and_mixed_precision_match_separate_runs():
    prods = products_small()
    dev = [[to_dev(x) for x in p] for p in prods]
    res = aci.elementwise_batched(dev, "product", 1e-12, 40, seed=9, precision="fp32", use_graph=True)
    for b, (cores, info) in enumerate(res):
        sc, si = aci.elementwise(dev[b], "product", 1e-12, 40, seed=9, precision="fp32")
        assert info.ranks == si.ranks and info.converged and si.converged
        assert_same(cores, sc)
        f = W.tt_full(prods[b][0]) * W.tt_full(prods[b][1])
        assert rel_max_err(W.tt_full([c.cpu().numpy() for c in cores]), f) <= 1e-10


def test_tune_prrlu_picks_a_measured_candidate():
    best, tried = aci.tune_prrlu(384, 384, 192, 32)
    assert tried and all(us > 0 for _, us in tried)
    caps = [c for c, _ in tried]
    assert best in caps
    assert min(tried, key=lambda t: t[1])[0] == best
    again, _ = aci.tune_prrlu(384, 384, 192, 32)
    assert again == best


def test_tuned_batch_equals_separate_runs():
    prods = products_small()[:2]
    dev = [[to_dev(x) for x in p] for p in prods]
    res = aci.elementwise_batched(dev, "product", 1e-12, 40, seed=9, tune=True, mode="overlapped")
    for b, (cores, info) in enumerate(res):
        sc, si = aci.elementwise(dev[b], "product", 1e-12, 40, seed=9)
        assert_same(cores, sc)


def test_batch_rejects_explicit_init_and_bad_sizes():
    prods = products_small()[:1]
    dev = [[to_dev(x) for x in p] for p in prods]
    with pytest.raises(Exception, match="LIMIT"):
        aci.elementwise_batched(dev * 65, "product", 1e-12, 40)


def nine_products():
    prods = []
    for b in range(9):
        x1, x2 = W.random_pair(L=12, chi=10 - (b % 3), seeds=(2400 + 2 * b, 2401 + 2 * b))
        prods.append([x1, x2])
    return prods


def separate_fixed(dev, sweeps, **kw):
    out = []
    for d in dev:
        S = aci.Session(d, "product", 1e-11, 64, maxiter=sweeps, seed=4, fixed_sweeps=True, **kw)
        S.sweep(sweeps)
        out.append(S.result())
        S.close()
    return out


@pytest.mark.parametrize("mode,xcd", [("joint", -2), ("overlapped", -1), ("serial", 0)])
def test_batch_modes_equal_separate_runs(mode, xcd):
    """Nine products of one length whose two-site matrices reach 128 x 128
    (rank cap 64): in joint mode each LDU needs 16 cooperating groups and two
    products share an XCD.  Every placement gives the separate runs' outputs
    bit for bit."""
    prods = nine_products()
    dev = [[to_dev(x) for x in p] for p in prods]
    B = aci.Batch(dev, "product", 1e-11, 64, maxiter=5, seed=4, fixed_sweeps=True, mode=mode)
    try:
        st = B.sweep(5)
        got = [B.result(b) for b in range(9)]
        place = [B.info(b) for b in range(9)]
    finally:
        B.close()
    assert all(x == xcd for x, _ in place)
    assert st["sweeps_done"] == 5
    ref = separate_fixed(dev, 5)
    for b in range(9):
        cores, info = got[b]
        sc, si = ref[b]
        assert info.ranks == si.ranks and info.eps == si.eps
        assert_same(cores, sc)


def test_joint_batch_profiled_launches():
    """The launch log of a joint batch holds one batched LDU launch per local
    update (logged with the first product) and no single-product LDU."""
    prods = nine_products()[:3]
    dev = [[to_dev(x) for x in p] for p in prods]
    B = aci.Batch(dev, "product", 1e-11, 64, maxiter=2, seed=4, fixed_sweeps=True, mode="joint", profile=True)
    try:
        st = B.sweep(2)
    finally:
        B.close()
    L = 12
    assert st["launches"][0] == 2 * 2 * (L - 1)


def test_joint_graph_replays_match_eager():
    """Replays of the captured joint sweep, with eager work and
    synchronisation in between, track the eager joint batch bit for bit."""
    prods = nine_products()[:4]
    dev = [[to_dev(x) for x in p] for p in prods]
    kw = dict(maxiter=4, seed=4, fixed_sweeps=True, mode="joint")
    G = aci.Batch(dev, "product", 1e-11, 64, use_graph=True, **kw)
    E = aci.Batch(dev, "product", 1e-11, 64, use_graph=False, **kw)
    try:
        for it in range(4):
            sg = G.sweep(1)
            se = E.sweep(1)
            assert sg["ranks"] == se["ranks"] and sg["max_eps"] == se["max_eps"]
            for b in range(4):
                cg, ig = G.result(b)
                ce, ie = E.result(b)
                assert ig.eps == ie.eps
                assert_same(cg, ce)
            t = torch.randn(1000, device="cuda")
            assert torch.isfinite((t * t).sum())
            torch.cuda.synchronize()
    finally:
        G.close()
        E.close()


def test_joint_batch_complex_matches_separate_runs():
    fields = [W.gp_field(R=5, chi=32, seed=s, width_scale=2.0) for s in (5001, 5002)]
    dev = [[to_dev(f)] for f in fields]
    res = aci.elementwise_batched(dev, "abs2_mul", 1e-8, 64, seed=6, mode="joint")
    for b, (cores, info) in enumerate(res):
        sc, si = aci.elementwise(dev[b], "abs2_mul", 1e-8, 64, seed=6)
        assert info.ranks == si.ranks and info.converged == si.converged
        assert_same(cores, sc)


def test_joint_mode_rejected_when_impossible():
    x1, x2 = W.random_pair(L=10, chi=4, seeds=(2501, 2502))
    y1, y2 = W.random_pair(L=9, chi=4, seeds=(2503, 2504))
    dev = [[to_dev(x1), to_dev(x2)], [to_dev(y1), to_dev(y2)]]
    with pytest.raises(Exception, match="LIMIT"):
        aci.Batch(dev, "product", 1e-12, 40, mode="joint")
    B = aci.Batch(dev, "product", 1e-12, 40)      # auto: overlapped
    try:
        assert all(B.info(b)[0] == -1 for b in range(2))
    finally:
        B.close()


def test_graph_replays_match_eager_with_eight_wave_ldus():
    """Rank cap 192 on 18 sites: the interior two-site matrices are 384 x 384,
    factorised by the eight-wave LDU instance (a plain launch inside the
    graph, a cooperative one eagerly); the LINEAR_CUBIC epilogue's
    coefficients are captured with the launch.  Graph replays and eager
    sweeps agree bit for bit."""
    x1 = W.random_tt(18, 2, 20, 2401)
    x2 = W.random_tt(18, 2, 20, 2402)
    d = [to_dev(x1), to_dev(x2)]
    op = aci.linear_cubic((0.5, -1.25), 0.75)
    kw = dict(maxiter=3, seed=6, fixed_sweeps=True)
    g = aci.Session(d, op, 1e-12, 192, use_graph=True, **kw)
    e = aci.Session(d, op, 1e-12, 192, use_graph=False, **kw)
    try:
        for it in range(3):
            sg = g.sweep(1)
            se = e.sweep(1)
            assert sg["ranks"] == se["ranks"]
            cg, ig = g.result()
            ce, ie = e.result()
            assert ig.eps == ie.eps
            assert_same(cg, ce)
        assert max(sg["ranks"]) == 192
    finally:
        g.close()
        e.close()
