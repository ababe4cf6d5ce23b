"""Pins of the whole oracle ACI (Alg. 1): brute force over all entries,
exact reconstruction at full rank, the Kronecker-delta product with SVD
rounding, closed-form Gaussian and Fourier products, special cases and the
interpolation property."""

import os

import numpy as np
import pytest

import workloads as W
from oracle import aci, default_init, splitmix64_stream, reference

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _full_f(xs, op):
    fs = [W.tt_full(x) for x in xs]
    if op == "product":
        out = fs[0]
        for f in fs[1:]:
            out = out * f
        return out
    if op == "sum":
        return sum(fs[1:], fs[0])
    raise ValueError(op)


def test_random_pair_bruteforce_all_entries():
    """Two random L=12, chi=8 TTs: the exact product has bond ranks
    min(2^l, 2^(L-l), 64) and ACI at maxrank 64 must reproduce all 4096
    entries to roundoff."""
    x1, x2 = W.random_pair()
    res = aci([x1, x2], "product", 1e-12, 64, maxiter=20, init=None, seed=1003)
    assert res.converged
    L = 12
    assert res.ranks == [min(2 ** l, 2 ** (L - l), 64) for l in range(1, L)]
    y = W.tt_full(res.cores)
    f = _full_f([x1, x2], "product")
    assert np.abs(y - f).max() <= 1e-13 * np.abs(f).max()


@pytest.mark.parametrize("pair", [(1003, 1004), (1005, 1006), (1007, 1008)])
def test_random_pairs_more_seeds(pair):
    x1, x2 = W.random_pair(L=10, chi=6, seeds=pair)
    res = aci([x1, x2], "product", 1e-12, 36, maxiter=20, seed=pair[0])
    f = _full_f([x1, x2], "product")
    assert res.converged
    assert np.abs(W.tt_full(res.cores) - f).max() <= 1e-13 * np.abs(f).max()


def test_matches_delta_product_with_svd_rounding():
    x1 = W.left_orthogonalise(W.random_tt(8, 2, 3, seed=31))
    x2 = W.left_orthogonalise(W.random_tt(8, 2, 4, seed=32))
    ref = reference.tt_round(reference.delta_product(x1, x2), rtol=1e-13)
    res = aci([x1, x2], "product", 1e-13, 64, maxiter=20, seed=33)
    assert res.converged
    assert res.ranks == W.tt_ranks(ref)[1:-1]
    yr = W.tt_full(ref)
    assert np.abs(W.tt_full(res.cores) - yr).max() <= 1e-12 * np.abs(yr).max()


def test_identity_single_input():
    x = W.left_orthogonalise(W.random_tt(9, 2, 5, seed=41))
    res = aci([x], "product", 1e-13, 50, seed=42)
    f = W.tt_full(x)
    assert np.abs(W.tt_full(res.cores) - f).max() <= 1e-13 * np.abs(f).max()
    exact = W.tt_ranks(reference.tt_round(x, rtol=1e-12))[1:-1]
    assert res.ranks == exact


def test_sum_rank_bound():
    x1 = W.left_orthogonalise(W.random_tt(9, 2, 3, seed=43))
    x2 = W.left_orthogonalise(W.random_tt(9, 2, 4, seed=44))
    res = aci([x1, x2], "sum", 1e-13, 50, seed=45)
    assert all(r <= 7 for r in res.ranks)
    f = _full_f([x1, x2], "sum")
    assert np.abs(W.tt_full(res.cores) - f).max() <= 1e-13 * np.abs(f).max()


def test_rank_one_inputs_give_rank_one_output():
    x1 = W.random_tt(10, 2, 1, seed=46)
    x2 = W.random_tt(10, 2, 1, seed=47)
    res = aci([x1, x2], "product", 1e-14, 10, seed=48)
    assert res.ranks == [1] * 9
    f = _full_f([x1, x2], "product")
    assert np.abs(W.tt_full(res.cores) - f).max() <= 1e-14 * np.abs(f).max()


def test_zero_result_path():
    x = W.random_tt(7, 2, 3, seed=49)
    neg = W.tt_scale(x, -1.0)
    res = aci([x, neg], "sum", 1e-12, 10, seed=50)
    assert res.ranks == [1] * 6 and res.converged
    assert np.all(W.tt_full(res.cores) == 0.0)


def test_complex_product_and_abs2_mul():
    x1 = W.left_orthogonalise(W.random_tt(8, 2, 3, seed=51, dtype=np.complex128))
    x2 = W.left_orthogonalise(W.random_tt(8, 2, 3, seed=52, dtype=np.complex128))
    res = aci([x1, x2], "product", 1e-13, 64, seed=53)
    f = W.tt_full(x1) * W.tt_full(x2)
    assert np.abs(W.tt_full(res.cores) - f).max() <= 1e-12 * np.abs(f).max()
    res = aci([x1], "abs2_mul", 1e-13, 64, seed=54)
    z = W.tt_full(x1)
    f = np.abs(z) ** 2 * z
    assert np.abs(W.tt_full(res.cores) - f).max() <= 1e-12 * np.abs(f).max()


def test_interpolation_property_on_bond1_cross():
    """After the final right-to-left sweep the TT equals f exactly on every
    point (s_1, j) with j in J_2, and the J sets are nested."""
    x1, x2 = W.random_pair(L=10, chi=5, seeds=(55, 56))
    res = aci([x1, x2], "product", 1e-6, 12, maxiter=3, seed=57)
    L = 10
    for l in range(2, L + 1):
        assert all(j[1:] in set(res.J[l + 1]) for j in res.J[l])
    pts = np.array([(s,) + j for s in range(2) for j in res.J[2]])
    y = W.tt_eval(res.cores, pts)
    f = W.tt_eval(x1, pts) * W.tt_eval(x2, pts)
    np.testing.assert_allclose(y, f, rtol=1e-12, atol=1e-14)


def test_not_converged_after_one_sweep():
    x1, x2 = W.random_pair()
    res = aci([x1, x2], "product", 1e-12, 64, maxiter=1, seed=1003)
    assert not res.converged and res.sweeps == 1


def test_literal_rule_also_reconstructs():
    x1, x2 = W.random_pair(L=10, chi=5, seeds=(58, 59))
    res = aci([x1, x2], "product", 1e-12, 25, rule="literal", seed=60)
    f = _full_f([x1, x2], "product")
    assert np.abs(W.tt_full(res.cores) - f).max() <= 1e-11 * np.abs(f).max()


@pytest.mark.parametrize("delta", [0.1, 0.4, 0.8])
def test_gaussian_product_closed_form(delta):
    """Eq. (gaussians): h = g+ g- = exp(-x^2/w^2) exp(-delta^2/(4 w^2)); the
    error decays with the output rank down to ~1e-14 (section 3.1)."""
    Lq = 18
    gp, gm, h = W.gaussian_pair_full(Lq, w=0.15, delta=delta)
    tp = W.tt_svd(gp, 2, 64, rtol=1e-15)
    tm = W.tt_svd(gm, 2, 64, rtol=1e-15)
    rng = np.random.default_rng(61)
    idx = rng.integers(0, 2 ** Lq, 1000)
    pts = ((idx[:, None] >> np.arange(Lq - 1, -1, -1)) & 1)
    errs = []
    for chi in (4, 8, 20):
        res = aci([tp, tm], "product", 1e-15, chi, maxiter=6, seed=62)
        errs.append(np.abs(W.tt_eval(res.cores, pts) - h[idx]).max())
    assert errs[0] > errs[1] > errs[2] or errs[2] < 1e-13
    assert errs[2] < 1e-12


def test_fourier_product_closed_form():
    """Eq. (fouriermultiplication): coefficients of g1 g2 are the
    convolution of the input coefficients."""
    Lq, K = 16, 12
    c1 = W.fourier1d_coeffs(K, 71)
    c2 = W.fourier1d_coeffs(K, 72)
    g1 = W.tt_svd(W.fourier1d_full(c1, Lq), 2, 64, rtol=1e-15)
    g2 = W.tt_svd(W.fourier1d_full(c2, Lq), 2, 64, rtol=1e-15)
    res = aci([g1, g2], "product", 1e-10, 64, maxiter=8, seed=73)
    assert res.converged
    h = W.fourier1d_full(W.fourier1d_product_coeffs(c1, c2), Lq)
    y = W.tt_full(res.cores).reshape(-1)
    assert np.abs(y - h).max() < 1e-8


def test_splitmix64_golden():
    with open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt")) as fh:
        vals = [int(line) for line in fh if line.strip() and not line.startswith("#")]
    assert splitmix64_stream(1234567, 5) == vals


def test_default_init_is_uniform_and_deterministic():
    cores = default_init([1, 2, 3, 1], [2, 2, 2], seed=99)
    assert [c.shape for c in cores] == [(1, 2, 2), (2, 2, 3), (3, 2, 1)]
    flat = np.concatenate([c.ravel() for c in cores])
    z = splitmix64_stream(99, flat.size)
    np.testing.assert_array_equal(flat, [(v >> 11) * 2.0 ** -53 * 2 - 1 for v in z])
    assert np.all(flat >= -1) and np.all(flat < 1)


def test_output_cores_solve_pivot_systems_at_labels():
    """For every bond l of the final right-to-left sweep, the pivot matrix
    P_l = f(x[I_l + J_{l+1}]) and the slice T_{l+1} = f(x[I_l + s + J_{l+2}]),
    both evaluated by brute force at the returned multi-index labels, satisfy
    P_l Y_{l+1} = T_{l+1} (Eq. ycicanonical with Y_{l+1} = P_l^{-1} T_{l+1});
    and Y_1 = T_1 = f(x[s + J_2])."""
    L = 9
    x1, x2 = W.random_pair(L=L, chi=4, seeds=(63, 64))
    res = aci([x1, x2], "product", 1e-10, 10, maxiter=4, seed=65)

    def f_at(pts):
        pts = np.array(pts)
        return W.tt_eval(x1, pts) * W.tt_eval(x2, pts)

    Y0 = res.cores[0]
    T1 = f_at([(s,) + j for s in range(2) for j in res.J[2]]).reshape(Y0.shape)
    np.testing.assert_allclose(Y0, T1, rtol=1e-12, atol=1e-14)
    for l in range(1, L):
        I, J1, J2 = res.I[l], res.J[l + 1], res.J[l + 2]
        P = f_at([i + j for i in I for j in J1]).reshape(len(I), len(J1))
        T = f_at([i + (s,) + j for i in I for s in range(2) for j in J2])
        Yn = res.cores[l].reshape(len(I), -1)
        np.testing.assert_allclose(P @ Yn, T.reshape(len(I), -1),
                                   atol=1e-11 * np.abs(T).max())
