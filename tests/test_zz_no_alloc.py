"""aci_prrlu_noalloc (the LDU with its workspace in a static device array)
against aci_prrlu: two calls in a row, the second on a smaller matrix, with
identical pivots, rank, error estimate and right factor, and no allocation
through the context's allocator."""

import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

ACI_E_LIMIT = -6


def _call(ctx, fn, M, tol, maxrank, outs):
    m, n = (int(s) for s in M.shape)
    rows, cols, rank, eps, Y = outs
    st = fn(ctx.h, 1 if M.dtype == torch.complex128 else 0, C.c_void_p(M.data_ptr()), m, n, n, C.c_double(tol),
            maxrank, 0, C.c_void_p(rows.data_ptr()), C.c_void_p(cols.data_ptr()), C.c_void_p(rank.data_ptr()),
            C.c_void_p(eps.data_ptr()), C.c_void_p(Y.data_ptr()), n)
    torch.cuda.synchronize()
    return st


def _outs(M, maxrank):
    m, n = (int(s) for s in M.shape)
    k = max(1, min(m, n, maxrank))
    dev = M.device
    return (torch.full((k,), -1, dtype=torch.int32, device=dev), torch.full((k,), -1, dtype=torch.int32, device=dev),
            torch.zeros(1, dtype=torch.int32, device=dev), torch.zeros(1, dtype=torch.float64, device=dev),
            torch.zeros(k, n, dtype=M.dtype, device=dev))


def _matrix(m, n, seed, complex_=False):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((m, n))
    if complex_:
        a = a + 1j * rng.standard_normal((m, n))
    return torch.from_numpy(a).cuda()


@pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")
def test_noalloc_ldu_matches_aci_prrlu_on_two_calls():
    import paper_2604_00037_amd as aci
    from paper_2604_00037_amd import _lib
    print("case: aci_prrlu_noalloc vs aci_prrlu, 384x384 real then 200x150 real then 96x300 complex", flush=True)
    ref_ctx = aci.Context()
    ctx = aci.Context(allocator="torch")   # any library allocation would show in torch's counters
    lib = _lib.load()
    cases = [(384, 384, 11, False, 192, 1e-8), (200, 150, 12, False, 64, 1e-8), (96, 300, 13, True, 80, 1e-6)]
    for m, n, seed, cx, maxrank, tol in cases:
        M = _matrix(m, n, seed, cx)
        want = _outs(M, maxrank)
        assert _call(ref_ctx, lib.aci_prrlu, M, tol, maxrank, want) == 0
        got = _outs(M, maxrank)
        torch.cuda.synchronize()
        before = torch.cuda.memory_stats().get("allocation.all.allocated", 0)
        st = _call(ctx, lib.aci_prrlu_noalloc, M, tol, maxrank, got)
        after = torch.cuda.memory_stats().get("allocation.all.allocated", 0)
        assert st == 0, lib.aci_last_error(ctx.h)
        assert after == before, "the no-alloc entry point allocated through the context's allocator"
        r = int(want[2].item())
        assert r == int(got[2].item()) and r >= 1
        assert torch.equal(want[0][:r], got[0][:r]) and torch.equal(want[1][:r], got[1][:r])
        assert want[3].item() == got[3].item()
        assert torch.equal(want[4][:r], got[4][:r])
    ctx.close()
    ref_ctx.close()


@pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")
def test_noalloc_ldu_rejects_exchanges_beyond_its_scratch():
    import paper_2604_00037_amd as aci
    from paper_2604_00037_amd import _lib
    print("case: aci_prrlu_noalloc limit, 1024x1024 complex", flush=True)
    ctx = aci.Context()
    lib = _lib.load()
    M = torch.zeros(1024, 1024, dtype=torch.complex128, device="cuda")
    st = _call(ctx, lib.aci_prrlu_noalloc, M, 1e-8, 512, _outs(M, 512))
    assert st == ACI_E_LIMIT
    assert b"static scratch" in lib.aci_last_error(ctx.h)
    ctx.close()
