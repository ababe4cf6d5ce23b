"""Learned pivot proposal on the GPU against the oracle: row features, the
scoring network (forward bit for bit, one Adam step and its gradients), the
seeded rook search (bit for bit), its acceptance test and right factor; and
what a network trained on the GPU gains: fewer rook scans per pivot on
held-out fields than the search without scores or with an untrained
network.  Training rows and initial weights come from the library itself
(aci_proposal_dataset, aci_mlp_init); the oracle only checks them."""

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import proposal as P
from helpers import rel_max_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
aci = pytest.importorskip("paper_2604_00037_amd")


def dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def flat(net):
    return np.concatenate([p.reshape(-1) for p in net.params()]).astype(np.float32)


def unflat(v):
    sizes = [(7, 64), (64,), (64, 64), (64,), (64,), (1,)]
    out, off = [], 0
    for s in sizes:
        c = int(np.prod(s))
        out.append(np.array(v[off:off + c], dtype=np.float32).reshape(s))
        off += c
    return P.MLP(*out)


def test_features_match_oracle():
    rng = np.random.default_rng(1)
    M = rng.standard_normal((50, 40))
    A = [rng.standard_normal((50, 13)), rng.standard_normal((50, 9))]
    prev = np.array([3, 7, 49], dtype=np.int32)
    X = aci.proposal_features(dev(M), [dev(a) for a in A], dev(prev)).cpu().numpy()
    ref = P.row_features(M, A, prev)
    np.testing.assert_allclose(X, ref, rtol=1e-6, atol=1e-7)
    X1 = aci.proposal_features(dev(M), [dev(A[0])]).cpu().numpy()
    np.testing.assert_allclose(X1, P.row_features(M, A[:1], []), rtol=1e-6, atol=1e-7)


def test_network_forward_bitwise():
    net = P.mlp_init(31)
    X = np.random.default_rng(2).uniform(0, 1, (300, 7)).astype(np.float32)
    z = aci.mlp_forward(dev(flat(net)), dev(X)).cpu().numpy()
    zr, _ = P.mlp_forward(net, X)
    assert np.array_equal(z, zr.astype(np.float32))


def test_training_step_matches_oracle():
    net = P.mlp_init(37)
    rng = np.random.default_rng(3)
    X = rng.uniform(0, 1, (200, 7)).astype(np.float32)
    y = (rng.uniform(0, 1, 200) < 0.4).astype(np.float32)
    p = dev(flat(net))
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    st = {}
    for step in range(1, 6):
        gref, lref = P.mlp_grads(net, X, y)
        loss, g = aci.mlp_train_step(p, m, v, step, dev(X), dev(y), lr=1e-2, want_grads=True)
        np.testing.assert_allclose(g.cpu().numpy(), np.concatenate([a.reshape(-1) for a in gref]),
                                   rtol=1e-5, atol=1e-9)
        assert abs(loss - lref) <= 1e-5 * (1 + abs(lref))
        P.adam_step(net, gref, st, lr=1e-2)
        np.testing.assert_allclose(p.cpu().numpy(), flat(net), rtol=1e-5, atol=1e-7)


@pytest.mark.parametrize("m,n,maxrank,tol,seeded", [(30, 20, 20, 0.0, False), (30, 20, 20, 0.0, True),
                                                    (64, 80, 12, 0.0, True), (17, 33, 40, 1e-3, True),
                                                    (129, 70, 70, 0.0, False)])
def test_rook_search_bitwise(m, n, maxrank, tol, seeded):
    rng = np.random.default_rng(m * 7 + n)
    M = rng.standard_normal((m, n))
    if tol > 0:
        M = rng.standard_normal((m, 5)) @ rng.standard_normal((5, n)) + 1e-4 * M
    scores = rng.standard_normal(m).astype(np.float32) if seeded else None
    rk = aci.rook_lu(dev(M), tol, maxrank, scores=None if scores is None else dev(scores), max_iter=8)
    ref = P.rook_lu(M, tol, maxrank, scores=scores, max_iter=8)
    assert rk["rank"] == ref.rank
    assert np.array_equal(rk["rows"], ref.rows) and np.array_equal(rk["cols"], ref.cols)
    assert rk["scans"] == ref.scans
    assert rk["eps"] == ref.eps_rook
    assert np.array_equal(rk["L"].cpu().numpy(), ref.L)
    assert np.array_equal(rk["Up"].cpu().numpy(), ref.Up)
    ok, eps = aci.rook_check(dev(M), rk, max(tol, 1e-300))
    ok_ref, eps_ref = P.rook_accept(M, ref, max(tol, 1e-300))
    assert ok == ok_ref
    assert abs(eps - eps_ref) <= 1e-12 * np.abs(M).max() * m
    Y = aci.rook_right_factor(rk).cpu().numpy()
    Yr = P.rook_right_factor(ref)
    np.testing.assert_allclose(Y, Yr, rtol=1e-12, atol=1e-12)
    assert np.array_equal(Y[:, ref.cols], np.eye(ref.rank))


# ------------------------------------------------------------ training data
def _field(R, kmax, s, chi):
    g = W.fourier3d_full(R, kmax, s)
    q = np.ascontiguousarray(W.grid_to_quantics(g, R, 3)).reshape(-1)
    return W.tt_svd(q, 2, chi, rtol=1e-12)


def test_mlp_init_matches_oracle_definition():
    """aci_mlp_init against the oracle's SplitMix64 initialisation, bit for bit."""
    for seed in (7, 12345, 2 ** 63 + 5):
        p = aci.mlp_init(seed).cpu().numpy()
        assert np.array_equal(p, flat(P.mlp_init(seed)))


def _oracle_dataset(inputs, tol, maxrank, maxiter, seed):
    """Features and labels of every local update of the oracle's plain ACI,
    by the dataset's definition (oracle as the checker)."""
    rec = []
    res = oracle.aci(inputs, "product", tol, maxrank, maxiter=maxiter, seed=seed, record=rec, log_gaps=True)
    prev, Xs, ys = {}, [], []
    for r in rec:
        key = (r["bond"], r["dir"])
        pr = prev.get(key, np.zeros(0, np.int32))
        prev[key] = r["rows"]
        Xs.append(P.row_features(r["M"], r["A"], pr))
        y = np.zeros(r["M"].shape[0], np.float32)
        y[r["rows"][:max(1, len(r["rows"]) // 2)]] = 1
        ys.append(y)
    return np.concatenate(Xs), np.concatenate(ys), res


@pytest.mark.parametrize("case", ["random_pair", "fourier3d"])
def test_dataset_matches_oracle_records(case):
    """aci_proposal_dataset (features and pivot labels recorded from the
    library's own FP64 sweeps) against the same rows built from the oracle's
    sweeps: the same number of rows, labels equal where the oracle's pivot
    steps are tie-free, features within float32 rounding."""
    if case == "random_pair":
        x1, x2 = W.random_pair(L=10, chi=5, seeds=(1001, 1002))
        tol, cap, it, seed = 1e-12, 25, 3, 1003
    else:
        x1, x2 = _field(3, 3, 21, 16), _field(3, 3, 1021, 16)
        tol, cap, it, seed = 1e-8, 48, 3, 5
    print(f"case: proposal dataset vs oracle records, {case}", flush=True)
    X, y, sweeps = aci.proposal_dataset([to_dev(x1), to_dev(x2)], "product", tol, cap, maxiter=it, seed=seed)
    Xr, yr, res = _oracle_dataset([x1, x2], tol, cap, it, seed)
    gaps = [t["min_gap"] for t in res.trace if t["dir"] != "init" and t["min_gap"] is not None]
    assert sweeps == res.sweeps
    assert X.shape[0] == Xr.shape[0] and y.shape[0] == yr.shape[0]
    if min(gaps) > 1e-10:
        assert np.array_equal(y.cpu().numpy(), yr)
    else:
        print(f"near tie (min gap {min(gaps):.1e}): labels compared in count only")
        assert int(y.sum().item()) == int(yr.sum())
    np.testing.assert_allclose(X.cpu().numpy(), Xr, rtol=2e-6, atol=2e-7)


def test_dataset_capacity_is_reported():
    """A dataset that fills up stops at the last whole update and says so."""
    x1, x2 = W.random_pair(L=8, chi=4, seeds=(1011, 1012))
    d = [to_dev(x1), to_dev(x2)]
    X, y, _ = aci.proposal_dataset(d, "product", 1e-12, 16, maxiter=2, seed=3)
    full = X.shape[0]
    assert full > 0
    with pytest.raises(aci._lib.HipError, match="NOMEM"):
        aci.proposal_dataset(d, "product", 1e-12, 16, maxiter=2, seed=3, capacity=full - 1)


def _library_training_set(seeds, R=4, kmax=4, chi=24):
    """Training rows from the library's own plain FP64 sweeps on products
    of two 3D random Fourier fields (R bits per axis, |k| <= kmax, rank chi),
    tol 1e-8, rank cap 64, three sweeps each."""
    Xs, ys = [], []
    for s in seeds:
        X, y, _ = aci.proposal_dataset([to_dev(_field(R, kmax, s, chi)), to_dev(_field(R, kmax, s + 1000, chi))],
                                       "product", 1e-8, 64, maxiter=3, seed=s)
        Xs.append(X)
        ys.append(y)
    return torch.cat(Xs), torch.cat(ys)


def _train(X, y, steps, seed=0, init_seed=7):
    p = aci.mlp_init(init_seed)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    rng = np.random.default_rng(seed)
    losses = []
    for step in range(1, steps + 1):
        idx = torch.from_numpy(rng.choice(X.shape[0], 512, replace=False)).cuda()
        loss, _ = aci.mlp_train_step(p, m, v, step, X[idx].contiguous(), y[idx].contiguous(), lr=3e-3)
        losses.append(loss)
    return p, losses


# ------------------------------------------------------------ what it gains
def test_trained_network_reduces_rook_scans():
    """A network trained on the GPU from the library's own sweeps needs fewer
    rook scans per pivot inside held-out sweeps than the search started at
    the smallest free row (all-zero network: equal scores) and than the
    untrained network."""
    X, y = _library_training_set(range(1, 7))
    p, losses = _train(X, y, 300)
    assert np.mean(losses[-20:]) < 0.8 * np.mean(losses[:20])
    untrained = aci.mlp_init(7)
    zeros = torch.zeros_like(p)

    def scans(params):
        tot, piv, acc, tried = 0, 0, 0, 0
        for sd in (101, 102, 103):
            g1, g2 = _field(4, 4, sd, 24), _field(4, 4, sd + 1000, 24)
            s = aci.Session([to_dev(g1), to_dev(g2)], "product", 1e-8, 64, maxiter=3, seed=sd, proposal=params,
                            fixed_sweeps=True)
            try:
                st = s.sweep(3)
            finally:
                s.close()
            tot += st["proposal_scans"]
            piv += st["proposal_pivots"]
            acc += st["proposals_accepted"]
            tried += st["proposals_tried"]
        return tot / piv, acc, tried

    s_none, a_none, t = scans(zeros)
    s_untr, a_untr, _ = scans(untrained)
    s_trained, a_trained, _ = scans(p)
    print(f"rook scans per pivot in held-out sweeps: trained {s_trained:.3f}, untrained {s_untr:.3f}, "
          f"no scores {s_none:.3f}; accepted {a_trained}/{a_untr}/{a_none} of {t}")
    assert s_trained < s_none and s_trained < s_untr
    assert a_trained >= 0.9 * a_none


# ------------------------------------------------------------ inside the sweep


def test_sweep_with_proposal_reconstructs_exactly_and_accepts():
    """Exact-rank products at tol 1e-12: the rook proposals (untrained
    network) are accepted at least sometimes, and the result still
    reconstructs the product like the plain sweep."""
    x1, x2 = W.random_pair(L=10, chi=5, seeds=(4101, 4102))
    params = aci.mlp_init(41)
    s = aci.Session([to_dev(x1), to_dev(x2)], "product", 1e-12, 30, maxiter=8, seed=2, proposal=params)
    try:
        st = s.sweep(8)
        cores, info = s.result()
    finally:
        s.close()
    assert info.converged
    assert st["proposals_tried"] > 0 and st["proposals_accepted"] > 0
    f = W.tt_full(x1) * W.tt_full(x2)
    assert rel_max_err(W.tt_full([c.cpu().numpy() for c in cores]), f) <= 1e-10


def test_rejected_proposals_leave_the_sweep_unchanged():
    """Rank cap 1 on random inputs: no two-site matrix has rank 1, so no
    rank-1 rook result reaches the tolerance 1e-300, every proposal is
    rejected and the LDU's output is reproduced bit for bit (also when the
    sweep replays a captured graph)."""
    x1, x2 = W.random_pair(L=10, chi=6, seeds=(4111, 4112))
    d = [to_dev(x1), to_dev(x2)]
    params = aci.mlp_init(43)
    plain, pi = aci.elementwise(d, "product", 1e-300, 1, maxiter=4, seed=3, fixed_sweeps=True)
    for use_graph in (False, True):
        s = aci.Session(d, "product", 1e-300, 1, maxiter=4, seed=3, proposal=params, use_graph=use_graph,
                        fixed_sweeps=True)
        try:
            st = s.sweep(4)
            cores, info = s.result()
        finally:
            s.close()
        assert st["proposals_accepted"] == 0 and st["proposals_tried"] > 0
        assert info.ranks == pi.ranks and info.eps == pi.eps
        for a, b in zip(cores, plain):
            assert torch.equal(a, b)


def test_sweep_with_trained_proposal_on_held_out_fields():
    """Network trained on the GPU from the library's own sweeps, used inside
    the sweeps of a held-out 3D Fourier product: converged, within 10 tol
    of the exact product, and most proposals accepted."""
    X, y = _library_training_set(range(1, 5))
    p, _ = _train(X, y, 200, seed=1)
    g1, g2 = _field(4, 4, 151, 24), _field(4, 4, 1151, 24)
    s = aci.Session([to_dev(g1), to_dev(g2)], "product", 1e-8, 64, maxiter=6, seed=5, proposal=p)
    try:
        st = s.sweep(6)
        cores, info = s.result()
    finally:
        s.close()
    assert info.converged
    assert st["proposals_accepted"] >= 0.5 * st["proposals_tried"]
    f = W.tt_full(g1) * W.tt_full(g2)
    y = W.tt_full([c.cpu().numpy() for c in cores])
    assert np.abs(y - f).max() <= 10 * 1e-8 * max(1.0, np.abs(f).max())
    print(f"accepted {st['proposals_accepted']} of {st['proposals_tried']} proposals in the last sweeps")
