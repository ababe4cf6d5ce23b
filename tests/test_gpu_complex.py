"""Complex (complex128 cores) HIP path against the oracle: contractions on
the real view with the operand expanded on the fly (FP64 and complex64
precision), the complex LDU with full pivoting (pivots bit for bit, keys
re^2 + im^2, complex arithmetic spelled out as in the oracle), gathers, and
whole sweeps including |psi|^2 psi of a Gross-Pitaevskii-like vortex field."""

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import prrlu as oprrlu
from oracle import apply_op
from helpers import compare_records, rel_max_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
aci = pytest.importorskip("paper_2604_00037_amd")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def crandn(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def cbound(A, B, unit):
    """Elementwise bound of a complex product computed as a real product of
    the real view: each real entry sums 2K real products."""
    K = A.shape[1]
    return 2 * (2 * K + 4) * unit * (np.abs(A) @ np.abs(B))


@pytest.mark.parametrize("m,k,n", [(3, 2, 5), (64, 40, 64), (130, 77, 70)])
@pytest.mark.parametrize("precision,unit", [("fp64", 2.0 ** -53), ("fp32", 2.0 ** -24)])
def test_complex_products_and_f(m, k, n, precision, unit):
    rng = np.random.default_rng(m + k + n)
    A = [crandn(rng, (m, k)) / np.sqrt(k), crandn(rng, (m, k + 3)) / np.sqrt(k)]
    B = [crandn(rng, (k, n)), crandn(rng, (k + 3, n))]
    P0, P1 = A[0] @ B[0], A[1] @ B[1]
    e0, e1 = cbound(A[0], B[0], unit), cbound(A[1], B[1], unit)
    M = aci.pi_eval("sum", [dev(a) for a in A], [dev(b) for b in B], precision=precision).cpu().numpy()
    assert np.all(np.abs(M - (P0 + P1)) <= 1.01 * (e0 + e1) + 4 * 2.0 ** -52 * np.abs(P0 + P1) + 1e-300)
    M = aci.pi_eval("product", [dev(a) for a in A], [dev(b) for b in B], precision=precision).cpu().numpy()
    bound = e0 * (np.abs(P1) + e1) + e1 * np.abs(P0) + 8 * 2.0 ** -52 * np.abs(P0) * np.abs(P1)
    assert np.all(np.abs(M - P0 * P1) <= 1.5 * bound + 1e-300)
    M = aci.pi_eval("abs2_mul", [dev(A[0])], [dev(B[0])], precision=precision).cpu().numpy()
    ref = apply_op("abs2_mul", [P0])
    bound = 3 * np.abs(P0) ** 2 * e0 * 1.5 + 8 * 2.0 ** -52 * np.abs(P0) ** 3
    assert np.all(np.abs(M - ref) <= bound + 1e-300)


def test_complex_environment_contraction():
    rng = np.random.default_rng(7)
    c, r0, d, r1 = 37, 21, 2, 19
    Lf = crandn(rng, (c, r0))
    X = crandn(rng, (r0, d, r1))
    out = aci.env_contract("left", [dev(Lf)], [dev(X)])[0].cpu().numpy()
    ref = Lf @ X.reshape(r0, d * r1)
    assert np.all(np.abs(out - ref) <= cbound(Lf, X.reshape(r0, d * r1), 2.0 ** -53) + 1e-300)
    R = crandn(rng, (r1, c))
    out = aci.env_contract("right", [dev(R)], [dev(X)])[0].cpu().numpy()
    ref = X.reshape(r0 * d, r1) @ R
    assert np.all(np.abs(out - ref) <= cbound(X.reshape(r0 * d, r1), R, 2.0 ** -53) + 1e-300)


@pytest.mark.parametrize("m,n,maxrank,tol", [(7, 9, 9, 0.0), (64, 64, 64, 0.0), (300, 200, 120, 0.0),
                                             (100, 130, 100, 1e-6), (513, 400, 64, 0.0),
                                             (600, 1000, 200, 0.0), (1024, 1024, 512, 0.0)])
def test_complex_ldu_pivots_bitwise(m, n, maxrank, tol):
    rng = np.random.default_rng(m * 3 + n)
    M = crandn(rng, (m, n))
    if tol > 0:
        M = crandn(rng, (m, 9)) @ crandn(rng, (9, n)) + 1e-7 * M
    ref = oprrlu(M, tol, maxrank, log_gaps=True)
    got = aci.prrlu(dev(M), tol, maxrank, want_y=True)
    if min(ref.gaps) > 1e-10:
        assert got["rank"] == ref.rank
        assert np.array_equal(got["rows"], ref.rows) and np.array_equal(got["cols"], ref.cols)
        assert got["eps"] == ref.eps
    U = ref.U
    J = ref.cols
    from scipy.linalg import solve_triangular
    Y = solve_triangular(U[:, J], U, unit_diagonal=True)
    np.testing.assert_allclose(got["Y"].cpu().numpy(), Y, rtol=0, atol=1e-9 * max(1.0, np.abs(Y).max()))


def test_complex_gathers():
    rng = np.random.default_rng(11)
    S = crandn(rng, (20, 30))
    idx = np.array([3, 0, 19, 7], dtype=np.int32)
    rows = aci.gather("rows", dev(S), dev(idx)).cpu().numpy()
    assert np.array_equal(rows, S[idx])
    cols = aci.gather("cols", dev(S), dev(np.array([29, 1, 4], dtype=np.int32))).cpu().numpy()
    assert np.array_equal(cols, S[:, [29, 1, 4]])


def run_both(inputs, op, tol, maxrank, seed, maxiter=12, precision="fp64"):
    ref = oracle.aci(inputs, op, tol, maxrank, maxiter=maxiter, seed=seed, log_gaps=True)
    cores, info = aci.elementwise([to_dev(x) for x in inputs], op, tol, maxrank, maxiter=maxiter, seed=seed,
                                  trace=True, precision=precision)
    return ref, [c.cpu().numpy() for c in cores], info


def test_complex_random_pair_sweep_matches_oracle():
    x1, x2 = W.random_pair(L=10, chi=5, seeds=(5101, 5102), dtype=np.complex128)
    ref, cores, info = run_both([x1, x2], "product", 1e-12, 40, seed=5)
    n = compare_records(info.records, ref.trace, "complex pair")
    assert n == len(ref.trace)
    assert info.ranks[1:-1] == ref.ranks and info.converged == ref.converged
    y = W.tt_full(cores)
    assert rel_max_err(y, W.tt_full(ref.cores)) <= 1e-10
    assert rel_max_err(y, W.tt_full(x1) * W.tt_full(x2)) <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_gross_pitaevskii_term_small(precision):
    """|psi|^2 psi of a vortex field on a 32 x 32 grid (2D quantics, L = 10):
    converged, the FP64 run identical to the oracle's pivots, and within 10 tol
    of the exact |psi|^2 psi."""
    R = 5
    psi = W.gp_field(R=R, chi=32, seed=5001, width_scale=2.0)
    ref, cores, info = run_both([psi], "abs2_mul", 1e-8, 64, seed=6, precision=precision)
    assert info.converged
    if precision == "fp64":
        n = compare_records(info.records, ref.trace, "gp")
        assert n == len(ref.trace)
    y = W.tt_full(cores)
    z = W.tt_full(psi)
    exact = (z.real * z.real + z.imag * z.imag) * z
    assert np.abs(y - exact).max() <= 10 * 1e-8 * max(1.0, np.abs(exact).max())
    assert rel_max_err(y, W.tt_full(ref.cores)) <= 1e-7
