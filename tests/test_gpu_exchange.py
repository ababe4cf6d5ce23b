"""Failure handling and hygiene of the LDU pivot exchange (Alg. 2's global
argmax and pivot-row broadcast between cooperating workgroups).

The failures are forced from the host through aci_ctx_set_exchange_hooks:
a small spin limit on the kernels' own bounded waits, and a stall that makes
the readers wait for a step flag no workgroup ever publishes.  Every kernel
still exits (each wait ends at its spin limit); the calls must report
ACI_E_TIMEOUT and the context must work again once the hook is off.  The
other tests check that exchange words left in recycled memory, or before a
reset of a session's flags, never pass for current ones."""

import numpy as np
import pytest

import workloads as W
from oracle import prrlu as oprrlu

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
aci = pytest.importorskip("paper_2604_00037_amd")
from paper_2604_00037_amd import _lib  # noqa: E402


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _timeout(fn):
    with pytest.raises(_lib.HipError, match="ACI_E_TIMEOUT"):
        fn()


@pytest.mark.parametrize("stall_step", [0, 5, 150])
def test_stalled_ldu_times_out_and_the_context_recovers(stall_step):
    rng = np.random.default_rng(404 + stall_step)
    M = rng.standard_normal((384, 384))      # 24 cooperating workgroups on one XCD
    ctx = aci.Context()
    try:
        print(f"stall at step {stall_step}, 384 x 384 real", flush=True)
        ctx.set_exchange_hooks(spin_limit=2048, stall_step=stall_step)
        _timeout(lambda: aci.prrlu(dev(M), 0.0, 192, ctx=ctx))
        ctx.set_exchange_hooks()             # off: the same context works again
        got = aci.prrlu(dev(M), 0.0, 192, want_y=True, ctx=ctx)
    finally:
        ctx.close()
    ref = oprrlu(M, 0.0, 192)
    assert got["rank"] == ref.rank
    np.testing.assert_array_equal(got["rows"], ref.rows)
    np.testing.assert_array_equal(got["cols"], ref.cols)
    assert got["eps"] == ref.eps


def test_stalled_cross_xcd_complex_ldu_times_out():
    """1024 x 1024 complex: 128 groups over all eight XCDs, device-scope
    exchange, two candidate words per thread."""
    rng = np.random.default_rng(77)
    M = rng.standard_normal((1024, 1024)) + 1j * rng.standard_normal((1024, 1024))
    Md = dev(M)
    ctx = aci.Context()
    try:
        print("stall at step 3, 1024 x 1024 complex", flush=True)
        ctx.set_exchange_hooks(spin_limit=2048, stall_step=3)
        _timeout(lambda: aci.prrlu(Md, 0.0, 64, ctx=ctx))
        ctx.set_exchange_hooks()
        got = aci.prrlu(Md, 0.0, 64, ctx=ctx)
    finally:
        ctx.close()
    ref = aci.prrlu(Md, 0.0, 64)
    assert got["rank"] == ref["rank"] == 64
    np.testing.assert_array_equal(got["rows"], ref["rows"])
    np.testing.assert_array_equal(got["cols"], ref["cols"])


def _pair():
    x1, x2 = W.random_pair(L=10, chi=12, seeds=(611, 612))
    return [[dev(c) for c in x] for x in (x1, x2)]


def test_stalled_session_sweep_times_out_and_a_new_session_works():
    d = _pair()
    kw = dict(maxiter=3, seed=9, fixed_sweeps=True)
    ctx = aci.Context()
    try:
        S = aci.Session(d, "product", 1e-12, 64, ctx=ctx, **kw)
        print("session sweep with the exchange stalled", flush=True)
        ctx.set_exchange_hooks(spin_limit=2048, stall_step=0)
        _timeout(lambda: S.sweep(1))
        S.close()
        ctx.set_exchange_hooks()
        S2 = aci.Session(d, "product", 1e-12, 64, ctx=ctx, **kw)
        S2.sweep(3)
        c2, i2 = S2.result()
        S2.close()
    finally:
        ctx.close()
    S3 = aci.Session(d, "product", 1e-12, 64, **kw)
    S3.sweep(3)
    c3, i3 = S3.result()
    S3.close()
    assert i2.ranks == i3.ranks and i2.eps == i3.eps
    for a, b in zip(c2, c3):
        assert torch.equal(a, b)


def test_stalled_joint_batch_times_out():
    d = _pair()
    ctx = aci.Context()
    try:
        ctx.set_exchange_hooks(spin_limit=2048, stall_step=2)
        print("joint batch with the exchange stalled", flush=True)
        B = aci.Batch([d, d], "product", 1e-12, 64, maxiter=2, seed=3, fixed_sweeps=True, mode="joint", ctx=ctx)
        try:
            _timeout(lambda: B.sweep(1))
        finally:
            B.close()
    finally:
        ctx.close()


@pytest.mark.parametrize("use_graph", [False, True])
def test_epoch_reset_before_every_sweep_changes_nothing(use_graph):
    """A session's exchange words are cleared and its flags restarted before
    they could wrap; forcing that reset before every sweep (eager and graph
    replays) gives the default session's results bit for bit."""
    d = _pair()
    kw = dict(maxiter=4, seed=21, fixed_sweeps=True, use_graph=use_graph)
    ctx = aci.Context()
    try:
        ctx.set_exchange_hooks(epoch_launches=1)
        S = aci.Session(d, "product", 1e-12, 64, ctx=ctx, **kw)
        S.sweep(4)
        c1, i1 = S.result()
        S.close()
    finally:
        ctx.close()
    S = aci.Session(d, "product", 1e-12, 64, **kw)
    S.sweep(4)
    c2, i2 = S.result()
    S.close()
    assert i1.ranks == i2.ranks and i1.eps == i2.eps
    for a, b in zip(c1, c2):
        assert torch.equal(a, b)


def test_recycled_memory_with_flagged_words_does_not_leak_into_the_ldu():
    """The step exchange buffer of a new context comes from the caller's
    allocator.  A block whose words all carry flag 1 (the flag of the first
    pivot step of the context's first launch) and a huge key must not be
    taken for published candidates: the library clears the buffer after
    allocating it."""
    xwords = 2 * 128 * (4 + 2 * 2 * 64 * 16)   # words of the step exchange buffer
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    blk = torch.empty(xwords, dtype=torch.int64, device="cuda")
    blk.fill_((1 << 32) | 0x7FE00000)
    torch.cuda.synchronize()
    del blk                                    # back to torch's cache, contents kept
    rng = np.random.default_rng(31)
    M = rng.standard_normal((384, 384))
    ctx = aci.Context(allocator="torch")
    try:
        got = aci.prrlu(dev(M), 0.0, 96, ctx=ctx)
    finally:
        ctx.close()
    ref = oprrlu(M, 0.0, 96)
    np.testing.assert_array_equal(got["rows"], ref.rows)
    np.testing.assert_array_equal(got["cols"], ref.cols)
    assert got["eps"] == ref.eps


@pytest.mark.parametrize("m,n,cx", [(1024, 1024, True), (700, 1024, False)])
def test_row_publication_rule_changes_no_pivot(m, n, cx):
    """Groups spread over several XCDs publish their candidate's row with the
    candidate only above a fraction of the predicted pivot key; otherwise the
    winner publishes its row late.  All rows eager (0), the default mix (0.6)
    and all winners late from the third step (inf) give the same pivots and
    right factor bit for bit, and the oracle's pivots where no near tie
    decides them."""
    import math
    rng = np.random.default_rng(m + 7 * n)
    M = rng.standard_normal((m, n)) + (1j * rng.standard_normal((m, n)) if cx else 0.0)
    rank = min(m, n) // 2
    got = []
    for frac in (0.0, 0.6, math.inf):
        ctx = aci.Context()
        try:
            ctx.set_row_publication(frac)
            r = aci.prrlu(dev(M), 0.0, rank, want_y=True, ctx=ctx)
        finally:
            ctx.close()
        got.append((r["rows"], r["cols"], r["eps"], r["Y"].cpu().numpy()))
    for g in got[1:]:
        assert np.array_equal(g[0], got[0][0]) and np.array_equal(g[1], got[0][1]) and g[2] == got[0][2]
        assert np.array_equal(g[3].view(np.uint8), got[0][3].view(np.uint8))
    ref = oprrlu(M, 0.0, rank, log_gaps=True)
    if min(ref.gaps) > 1e-10:
        np.testing.assert_array_equal(got[0][0], ref.rows)
        np.testing.assert_array_equal(got[0][1], ref.cols)
        assert got[0][2] == ref.eps


def test_hook_arguments_are_checked():
    ctx = aci.Context()
    try:
        with pytest.raises(_lib.HipError, match="ACI_E_INVALID"):
            ctx.set_exchange_hooks(stall_step=-2)
        with pytest.raises(_lib.HipError, match="ACI_E_INVALID"):
            ctx.set_exchange_hooks(epoch_launches=1 << 40)
        with pytest.raises(_lib.HipError, match="ACI_E_INVALID"):
            ctx.set_row_publication(-0.5)
        with pytest.raises(_lib.HipError, match="ACI_E_INVALID"):
            ctx.set_row_publication(float("nan"))
    finally:
        ctx.close()
