"""Patched ACI on the GPU against the oracle: the same tree of patches
(prefixes, level by level), and per patch the same ranks, convergence and
output values; the assembled patches against the exact product; levels of
more than twelve patches (batched without the joint LDU launch); and the
depth-0 case against the unpatched sweep."""

import numpy as np
import pytest

import oracle
from oracle import patched as P
import workloads as W
from helpers import rel_max_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
aci = pytest.importorskip("paper_2604_00037_amd")


def tt_add(a, b):
    """Cores of a + b (block-diagonal bonds)."""
    L = len(a)
    out = []
    for l, (x, y) in enumerate(zip(a, b)):
        if l == 0:
            out.append(np.concatenate([x, y], axis=2))
        elif l == L - 1:
            out.append(np.concatenate([x, y], axis=0))
        else:
            z = np.zeros((x.shape[0] + y.shape[0], x.shape[1], x.shape[2] + y.shape[2]), dtype=x.dtype)
            z[:x.shape[0], :, :x.shape[2]] = x
            z[x.shape[0]:, :, x.shape[2]:] = y
            out.append(z)
    return out


def half_rough(L, seed, dtype=np.float64):
    """Rank 2 where the first index is 0, rank 8 where it is 1."""
    smooth = W.random_tt(L, 2, 2, seed, dtype=dtype)
    rough = W.random_tt(L, 2, 6, seed + 1, dtype=dtype)
    rough[0] = rough[0].copy()
    rough[0][:, 0, :] = 0.0
    return tt_add(smooth, rough)


def check(inputs, op, tol, cap, depth, seed):
    ref = P.patched_aci(inputs, op, tol, cap, depth, seed=seed)
    got, status = aci.patched([to_dev(x) for x in inputs], op, tol, cap, depth, seed=seed)
    assert [p.prefix for p in got] == [p.prefix for p in ref]
    for g, r in zip(got, ref):
        assert g.ranks[1:-1] == r.result.ranks, g.prefix
        assert g.converged == r.result.converged and g.sweeps == r.result.sweeps
        y = W.tt_full([c.cpu().numpy() for c in g.cores])
        assert rel_max_err(y, W.tt_full(r.result.cores)) <= 1e-10, g.prefix
    return got, ref, status


@pytest.mark.parametrize("cplx", [False, True])
def test_mixed_depth_patches_match_oracle(cplx):
    dtype = np.complex128 if cplx else np.float64
    L = 10
    x1, x2 = half_rough(L, 3201, dtype), half_rough(L, 3211, dtype)
    got, ref, status = check([x1, x2], "product", 1e-10, 8, 4, 5)
    depths = sorted({len(p.prefix) for p in got})
    assert len(depths) > 1                     # the smooth half stops early
    assert status == 0 and all(p.converged for p in got)
    exact = W.tt_full(x1) * W.tt_full(x2)
    full = np.zeros_like(exact)
    for p in got:
        full[p.prefix] = W.tt_full([c.cpu().numpy() for c in p.cores])
    assert np.abs(full - exact).max() <= 1e-9 * np.abs(exact).max()


def test_wide_levels_and_unconverged_leaves():
    L = 9
    x1 = W.random_tt(L, 2, 6, 3221)
    x2 = W.random_tt(L, 2, 6, 3222)
    got, ref, status = check([x1, x2], "product", 1e-12, 3, 4, 2)   # 16 patches at the last level
    assert len(got) == 16 and status == 1
    assert not all(p.converged for p in got)


def test_depth_zero_is_elementwise():
    x1, x2 = W.random_pair(L=10, chi=4, seeds=(3231, 3232))
    got, _, _ = check([x1, x2], "product", 1e-12, 32, 0, 3)
    cores, info = aci.elementwise([to_dev(x1), to_dev(x2)], "product", 1e-12, 32, seed=3)
    assert len(got) == 1 and got[0].ranks == info.ranks
    for a, b in zip(got[0].cores, cores):
        assert torch.equal(a, b)


def test_patched_rejects_bad_depth():
    x1, x2 = W.random_pair(L=6, chi=3, seeds=(3241, 3242))
    with pytest.raises(aci._lib.HipError):
        aci.patched([to_dev(x1), to_dev(x2)], "product", 1e-12, 8, 5)


def test_patched_rejects_an_explicit_init():
    import ctypes as C
    from paper_2604_00037_amd import aci as mod
    x1, x2 = W.random_pair(L=6, chi=3, seeds=(3251, 3252))
    d1, d2 = to_dev(x1), to_dev(x2)
    ctx = mod.default_context()
    keep = []
    tts = mod._inputs([d1, d2], keep)
    opts = mod._options(keep, 4, 0, d1, "exclusive", "fp64", False, False, False)
    res = mod._lib.AciPatchedResult()
    status = ctx.lib.aci_patched(ctx.h, tts, 2, 0, 0, 1e-12, 8, 1, C.byref(opts), C.byref(res))
    assert status == -1
    assert b"init" in ctx.lib.aci_last_error(ctx.h)
    ctx.lib.aci_patched_free(ctx.h, C.byref(res))
