"""Step-level parity of the HIP kernels with the oracle, through the C ABI:
environment contractions, two-site tensors with f, LDU with full pivoting
(bit-identical pivots, error estimates and residual arithmetic), the
right-interpolative factor U_JJ^{-1} U, and frame gathers."""

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import prrlu as oprrlu
from oracle import cross_interpolate, apply_op
from helpers import gemm_bound

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
aci = pytest.importorskip("paper_2604_00037_amd")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


# ------------------------------------------------------------ contractions
@pytest.mark.parametrize("c,r0,d,r1", [(1, 1, 2, 1), (5, 3, 2, 7), (64, 64, 2, 64),
                                       (192, 128, 2, 128), (77, 129, 3, 65)])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_env_contractions_match_products(c, r0, d, r1, precision):
    rng = np.random.default_rng(c * 7 + r0)
    Ls = [rng.standard_normal((c, r0)) for _ in range(2)]
    Xs = [rng.standard_normal((r0, d, r1)) for _ in range(2)]
    outs = aci.env_contract("left", [dev(x) for x in Ls], [dev(x) for x in Xs], precision=precision)
    for Lf, X, o in zip(Ls, Xs, outs):
        A = Lf
        B = X.reshape(r0, d * r1)
        ref = A @ B
        assert np.all(np.abs(o.cpu().numpy() - ref) <= gemm_bound(A, B, precision) + 1e-300)
    Rs = [rng.standard_normal((r1, c)) for _ in range(2)]
    outs = aci.env_contract("right", [dev(x) for x in Rs], [dev(x) for x in Xs], precision=precision)
    for R, X, o in zip(Rs, Xs, outs):
        A = X.reshape(r0 * d, r1)
        ref = A @ R
        assert np.all(np.abs(o.cpu().numpy() - ref) <= gemm_bound(A, R, precision) + 1e-300)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_low_precision_products_are_not_fp64(precision):
    """The low-precision paths really round: their error is far above FP64's
    on a well-conditioned product (guards against a silent FP64 fallback)."""
    rng = np.random.default_rng(5)
    A = rng.standard_normal((128, 96))
    B = rng.standard_normal((96, 128))
    M = aci.pi_eval("product", [dev(A)], [dev(B)], precision=precision).cpu().numpy()
    err = np.abs(M - A @ B).max() / np.abs(A @ B).max()
    assert err > 1e-9


@pytest.mark.parametrize("op,N", [("product", 2), ("sum", 2), ("product", 3), ("abs2_mul", 1),
                                  ("product", 1)])
@pytest.mark.parametrize("m,n", [(2, 3), (64, 64), (130, 70), (384, 384)])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_two_site_tensor_with_f(op, N, m, n, precision):
    rng = np.random.default_rng(m + 31 * n + N)
    ks = [int(k) for k in rng.integers(1, 140, N)]
    A = [rng.standard_normal((m, k)) / np.sqrt(k) for k in ks]
    B = [rng.standard_normal((k, n)) for k in ks]
    M = aci.pi_eval(op, [dev(a) for a in A], [dev(b) for b in B], precision=precision).cpu().numpy()
    ref = apply_op(op, [a @ b for a, b in zip(A, B)])
    # first-order error bound of f applied to perturbed products
    errs = [gemm_bound(a, b, precision) for a, b in zip(A, B)]
    vals = [np.abs(a @ b) for a, b in zip(A, B)]
    if op == "sum":
        bound = sum(errs) + 4 * 2.0 ** -52 * sum(vals)
    elif op == "abs2_mul":
        bound = 3 * vals[0] ** 2 * errs[0] + 4 * 2.0 ** -52 * vals[0] ** 3
    else:
        bound = np.zeros_like(ref)
        for i in range(N):
            other = np.ones_like(ref)
            for j in range(N):
                if j != i:
                    other = other * (vals[j] + errs[j])
            bound = bound + errs[i] * other
        bound = bound + (N + 1) * 2.0 ** -52 * np.prod(vals, axis=0)
    assert np.all(np.abs(M - ref) <= 1.01 * bound + 1e-300)


def test_two_site_tensor_flags_nonfinite():
    A = np.ones((4, 3))
    A[1, 1] = np.nan
    B = np.ones((3, 5))
    with pytest.raises(Exception, match="NUMERIC"):
        aci.pi_eval("product", [dev(A)], [dev(B)])


# ------------------------------------------------------------------ prrLU
def _matrix(kind, m, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "gauss":
        return rng.standard_normal((m, n))
    if kind == "lowrank":
        r = max(1, min(m, n) // 3)
        M = (rng.standard_normal((m, r)) @ rng.standard_normal((r, n))) / np.sqrt(r)
        return M + 1e-9 * rng.standard_normal((m, n))
    if kind == "exactrank":
        r = max(1, min(m, n) // 4)
        return rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    if kind == "ties":
        return rng.integers(-2, 3, (m, n)).astype(np.float64)
    if kind == "zero":
        return np.zeros((m, n))
    raise ValueError(kind)


SHAPES = [(1, 1), (1, 9), (9, 1), (3, 5), (37, 61), (64, 64), (65, 129), (128, 200),
          (200, 384), (384, 384), (512, 256), (300, 512), (1000, 700)]


@pytest.mark.parametrize("m,n", SHAPES)
@pytest.mark.parametrize("kind", ["gauss", "lowrank", "ties"])
@pytest.mark.parametrize("rule", ["exclusive", "literal"])
def test_prrlu_bit_identical_to_oracle(m, n, kind, rule):
    M = _matrix(kind, m, n, seed=m * 131 + n * 7 + len(kind))
    maxrank = min(m, n, 192)
    tol = 1e-7 if kind == "lowrank" else 0.0
    ref = oprrlu(M, tol, maxrank, rule=rule)
    got = aci.prrlu(dev(M), tol, maxrank, stop_rule=rule)
    assert got["rank"] == ref.rank
    np.testing.assert_array_equal(got["rows"], ref.rows)
    np.testing.assert_array_equal(got["cols"], ref.cols)
    assert got["eps"] == ref.eps


@pytest.mark.parametrize("m,n,maxrank", [(3, 5, 5), (37, 61, 20), (128, 200, 128), (384, 384, 192),
                                         (300, 512, 160), (1000, 700, 100), (384, 300, 150), (480, 380, 190)])
def test_right_factor_matches_triangular_solve(m, n, maxrank):
    M = _matrix("lowrank", m, n, seed=m + n)
    A, B, ref = cross_interpolate(M, 1e-7, maxrank, "right")
    got = aci.prrlu(dev(M), 1e-7, maxrank, want_y=True)
    np.testing.assert_array_equal(got["cols"], ref.cols)
    Y = got["Y"].cpu().numpy()
    # B[:, J] is the identity exactly; elsewhere agreement to the solve's accuracy
    np.testing.assert_array_equal(Y[:, ref.cols], np.eye(ref.rank))
    assert np.abs(Y - B).max() <= 1e-10 * max(1.0, np.abs(B).max())
    # and the skeleton reproduces M on the pivot rows
    np.testing.assert_allclose(M[:, ref.cols] @ Y, A @ B, atol=1e-9 * np.abs(M).max())


@pytest.mark.parametrize("m,n", [(1, 1), (4, 6), (130, 70)])
def test_prrlu_zero_and_exact_rank(m, n):
    Z = np.zeros((m, n))
    got = aci.prrlu(dev(Z), 1e-12, 5, want_y=True)
    ref = oprrlu(Z, 1e-12, 5)
    assert got["rank"] == 1 and got["eps"] == 0.0
    np.testing.assert_array_equal(got["rows"], ref.rows)
    np.testing.assert_array_equal(got["cols"], ref.cols)
    Y = got["Y"].cpu().numpy()
    e = np.zeros((1, n))
    e[0, ref.cols[0]] = 1.0
    np.testing.assert_array_equal(Y, e)
    M = _matrix("exactrank", m, n, seed=5)
    ref = oprrlu(M, 1e-10, 1000)
    got = aci.prrlu(dev(M), 1e-10, 1000)
    assert got["rank"] == ref.rank
    np.testing.assert_array_equal(got["cols"], ref.cols)


def test_prrlu_first_pivot_and_cap():
    M = np.full((5, 5), 1e-20)
    M[3, 1] = -3e-20
    got = aci.prrlu(dev(M), 1e-8, 4)
    assert got["rank"] == 1 and list(got["rows"]) == [3] and list(got["cols"]) == [1]
    M = _matrix("gauss", 50, 40, 9)
    got = aci.prrlu(dev(M), 0.0, 7)
    ref = oprrlu(M, 0.0, 7)
    assert got["rank"] == 7 and got["eps"] == ref.eps


# ----------------------------------------------------------------- gathers
def test_gathers():
    rng = np.random.default_rng(3)
    S = rng.standard_normal((37, 53))
    idx = [5, 0, 36, 17]
    got = aci.gather("rows", dev(S), idx).cpu().numpy()
    np.testing.assert_array_equal(got, S[idx, :])
    idx = [52, 3, 3, 9, 0]
    got = aci.gather("cols", dev(S), idx).cpu().numpy()
    np.testing.assert_array_equal(got, S[:, idx])


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_contraction_tiles_give_identical_results(cplx, precision):
    """Every output tile shape accumulates each element in the same order,
    so all tiles give the default launch's result bit for bit (ragged
    sizes, two terms and the |z|^2 z epilogue)."""
    rng = np.random.default_rng(77)

    def mk(shape):
        x = rng.standard_normal(shape)
        return x + 1j * rng.standard_normal(shape) if cplx else x

    m, k, n = 130, 77, 70
    A = [torch.from_numpy(mk((m, k))).cuda(), torch.from_numpy(mk((m, k + 3))).cuda()]
    B = [torch.from_numpy(mk((k, n))).cuda(), torch.from_numpy(mk((k + 3, n))).cuda()]
    for op, a, b in (("product", A, B), ("abs2_mul", A[:1], B[:1])):
        ref = aci.pi_eval(op, a, b, precision=precision)
        for tile in aci.TILES:
            assert torch.equal(aci.pi_eval(op, a, b, precision=precision, tile=tile), ref), (op, tile)


def test_tune_contract_picks_the_fastest_tile():
    best, us = aci.tune_contract(384, 128, 384)
    assert set(us) == set(aci.TILES) and all(v > 0 for v in us.values())
    assert us[best] == min(us.values())
    best_c, us_c = aci.tune_contract(1024, 512, 1024, dtype="c128", precision="fp32")
    assert us_c[best_c] == min(us_c.values())


def test_tuned_session_equals_default():
    """A session whose contraction tiles come from the autotuner gives the
    default session's sweep bit for bit; its launch log names the tiles."""
    x1, x2 = W.random_pair(L=12, chi=9, seeds=(2701, 2702))
    d = [[torch.from_numpy(np.ascontiguousarray(c)).cuda() for c in x] for x in (x1, x2)]
    kw = dict(maxiter=4, seed=5, fixed_sweeps=True, profile=True)
    S1 = aci.Session(d, "product", 1e-11, 81, tune=True, **kw)
    S2 = aci.Session(d, "product", 1e-11, 81, **kw)
    try:
        S1.sweep(4)
        S2.sweep(4)
        c1, i1 = S1.result()
        c2, i2 = S2.result()
        names = {r["kernel"] for r in S1.launches() if r["kind"] == "contract"}
    finally:
        S1.close()
        S2.close()
    assert i1.ranks == i2.ranks and i1.eps == i2.eps
    for a, b in zip(c1, c2):
        assert torch.equal(a, b)
    assert names and all("Tile<" in n for n in names)
