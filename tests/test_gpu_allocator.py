"""Contexts whose device memory comes from torch's caching allocator
(aci_ctx_create_with_allocator): the workspaces show up in torch's
accounting while a session or batch lives and are given back when it
closes, and the results equal those of a default context bit for bit."""

import pytest

import workloads as W
from helpers import to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
aci = pytest.importorskip("paper_2604_00037_amd")


def test_session_and_batch_on_torch_allocator():
    x1, x2 = W.random_pair(L=10, chi=5, seeds=(2601, 2602))
    d = [to_dev(x1), to_dev(x2)]
    ref = aci.Session(d, "product", 1e-12, 40, maxiter=6, seed=3, fixed_sweeps=True)
    ref.sweep(6)
    rc, ri = ref.result()
    ref.close()

    ctx = aci.Context(allocator="torch")
    try:
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        S = aci.Session(d, "product", 1e-12, 40, maxiter=6, seed=3, fixed_sweeps=True, ctx=ctx)
        during = torch.cuda.memory_allocated()
        assert during > before
        S.sweep(6)
        cores, info = S.result()
        S.close()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() < during
        assert info.ranks == ri.ranks and info.eps == ri.eps
        for a, b in zip(cores, rc):
            assert torch.equal(a, b)

        y1, y2 = W.random_pair(L=10, chi=4, seeds=(2603, 2604))
        prods = [d, [to_dev(y1), to_dev(y2)]]
        B = aci.Batch(prods, "product", 1e-12, 40, maxiter=6, seed=3, fixed_sweeps=True, ctx=ctx)
        B.sweep(6)
        got = B.result(0)
        B.close()
        for a, b in zip(got[0], rc):
            assert torch.equal(a, b)
        # the single-step entry points draw their buffers from it as well
        M = torch.randn(64, 48, dtype=torch.float64, device="cuda")
        r = aci.prrlu(M, 0.0, 32, ctx=ctx)
        r0 = aci.prrlu(M, 0.0, 32)
        assert (r["rows"] == r0["rows"]).all() and r["eps"] == r0["eps"]
    finally:
        ctx.close()
