"""Pins of cross interpolation (Alg. 3), the local reshape (Alg. 4) and the
frame recursion (Alg. 5 / Eq. framesrecursive) against direct definitions:
the CUR skeleton formula and brute-force products of core slices."""

import numpy as np
import pytest

import workloads as W
from oracle import cross_interpolate, left_frame, right_frame, local_update
from oracle.aci import _pi_tensors


@pytest.mark.parametrize("side", ["right", "left"])
@pytest.mark.parametrize("cplx", [False, True])
def test_skeleton_identity(side, cplx):
    rng = np.random.default_rng(21)
    M = rng.standard_normal((40, 9)) @ rng.standard_normal((9, 30))
    M = M + 1e-3 * rng.standard_normal((40, 30))
    if cplx:
        M = M + 1j * (rng.standard_normal((40, 9)) @ rng.standard_normal((9, 30)))
    A, B, lu = cross_interpolate(M, 0.0, 6, side)
    I, J = lu.rows, lu.cols
    skel = M[:, J] @ np.linalg.solve(M[np.ix_(I, J)], M[I, :])
    np.testing.assert_allclose(A @ B, skel, atol=1e-11 * np.abs(M).max())
    # interpolation: exact on pivot rows and columns
    np.testing.assert_allclose((A @ B)[I, :], M[I, :], atol=1e-12 * np.abs(M).max())
    np.testing.assert_allclose((A @ B)[:, J], M[:, J], atol=1e-12 * np.abs(M).max())
    if side == "right":
        np.testing.assert_array_equal(B[:, J], np.eye(len(J)))
    else:
        np.testing.assert_array_equal(A[I, :], np.eye(len(I)))
    # error estimate equals the largest entry of the CI residual
    assert abs(lu.eps - np.abs(M - A @ B).max()) <= 1e-11 * np.abs(M).max()


def _random_nested_sets(L, d, sizes, rng):
    """Nested I_0..I_L (I_l subset I_{l-1} x S_l) and J_1..J_{L+1}."""
    I = [[()]]
    for l in range(1, L + 1):
        cand = [i + (s,) for i in I[-1] for s in range(d)]
        k = min(sizes[l], len(cand))
        pick = rng.choice(len(cand), k, replace=False)
        I.append([cand[p] for p in pick])
    J = [None] * (L + 2)
    J[L + 1] = [()]
    for l in range(L, 0, -1):
        cand = [(s,) + j for s in range(d) for j in J[l + 1]]
        k = min(sizes[l - 1], len(cand))
        pick = rng.choice(len(cand), k, replace=False)
        J[l] = [cand[p] for p in pick]
    return I, J


def _brute_left(cores, i):
    v = np.ones((1, 1))
    for s, idx in enumerate(i):
        v = v @ cores[s][:, idx, :]
    return v[0]


def _brute_right(cores, j, start):
    v = np.ones((1, 1))
    for s in range(len(j) - 1, -1, -1):
        v = cores[start + s][:, j[s], :] @ v
    return v[:, 0]


def test_frames_match_brute_force_products():
    rng = np.random.default_rng(22)
    L, d = 7, 2
    X = W.random_tt(L, d, 5, seed=23)
    sizes = [1, 2, 4, 6, 6, 6, 4, 2, 1]
    I, J = _random_nested_sets(L, d, sizes, rng)
    Lf = np.ones((1, 1))
    for l in range(1, L):
        rows = [I[l - 1].index(i[:-1]) * d + i[-1] for i in I[l]]
        Lf = left_frame(X[l - 1], Lf, rows)
        ref = np.array([_brute_left(X, i) for i in I[l]])
        np.testing.assert_allclose(Lf, ref, rtol=1e-13, atol=1e-15)
    Rf = np.ones((1, 1))
    for l in range(L, 1, -1):
        cols = [j[0] * len(J[l + 1]) + J[l + 1].index(j[1:]) for j in J[l]]
        Rf = right_frame(X[l - 1], Rf, cols)
        ref = np.array([_brute_right(X, j, l - 1) for j in J[l]]).T
        np.testing.assert_allclose(Rf, ref, rtol=1e-13, atol=1e-15)


def test_two_site_tensor_matches_tt_evaluation():
    rng = np.random.default_rng(24)
    L, d = 8, 2
    Xs = [W.random_tt(L, d, 4, seed=25 + n) for n in range(2)]
    sizes = [1, 2, 4, 5, 5, 5, 5, 4, 2, 1]
    I, J = _random_nested_sets(L, d, sizes, rng)
    Lf = [[None] * (L + 1) for _ in Xs]
    Rf = [[None] * (L + 2) for _ in Xs]
    for n, X in enumerate(Xs):
        Lf[n][0] = np.ones((1, 1))
        Rf[n][L + 1] = np.ones((1, 1))
        for l in range(1, L + 1):
            rows = [I[l - 1].index(i[:-1]) * d + i[-1] for i in I[l]]
            Lf[n][l] = left_frame(X[l - 1], Lf[n][l - 1], rows)
        for l in range(L, 0, -1):
            cols = [j[0] * len(J[l + 1]) + J[l + 1].index(j[1:]) for j in J[l]]
            Rf[n][l] = right_frame(X[l - 1], Rf[n][l + 1], cols)
    for l in (1, 3, L - 1):
        Pis = _pi_tensors(Xs, Lf, Rf, l)
        for n, X in enumerate(Xs):
            pts = [i + (s, t) + j for i in I[l - 1] for s in range(d) for t in range(d)
                   for j in J[l + 2]]
            ref = W.tt_eval(X, np.array(pts)).reshape(Pis[n].shape)
            np.testing.assert_allclose(Pis[n], ref, rtol=1e-12, atol=1e-14)


def test_local_update_reshape_convention():
    rng = np.random.default_rng(26)
    Pi = rng.standard_normal((3, 2, 2, 5))
    Y, Y2, M, lu = local_update(Pi, 0.0, 100, "right")
    # row (a, s) = a*d + s, column (s', b) = s'*c_R + b
    assert M[1 * 2 + 1, 1 * 5 + 3] == Pi[1, 1, 1, 3]
    np.testing.assert_allclose(np.einsum("asr,rtb->astb", Y, Y2), Pi, atol=1e-12)
