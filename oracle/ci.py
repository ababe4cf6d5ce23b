"""Cross interpolation, local update and frame matrices.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* ``cross_interpolate`` -- Alg. 3.  "right": A = M[:, J], B = U_JJ^{-1} U
  (P^{-1} multiplied into the right factor); "left": A = L L_II^{-1},
  B = M[I, :].  A = M[:, J] equals L D U[:, J] in exact arithmetic (a cross
  interpolation reproduces its pivot columns), and the oracle uses the
  sampled columns directly (reading R6).
* ``local_update`` -- Alg. 4: Pi[a, s, s', b] -> M[(a, s), (s', b)] with
  row a*d + s and column s'*c_R + b.
* ``left_frame`` / ``right_frame`` -- Alg. 5 and Eq. (framesrecursive):
  L' = (L X)[I, :] and R' = (X R)[:, J].

Pins: the skeleton identity A B = M[:, J] M[I, J]^{-1} M[I, :] and the
exactness on pivot rows/columns; frames against brute-force products of
core slices along each multi-index (tests/test_oracle_ci.py).
"""

from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular

from .prrlu import prrlu


def cross_interpolate(M, tol, maxrank, leftorright="right", rule="exclusive", log_gaps=False):
    lu = prrlu(M, tol, maxrank, rule=rule, log_gaps=log_gaps)
    I, J = lu.rows, lu.cols
    if lu.zero_path:
        A = np.zeros((M.shape[0], 1), dtype=lu.L.dtype)
        B = lu.U.copy()
        return A, B, lu
    if leftorright == "right":
        A = np.array(M[:, J], copy=True)
        B = solve_triangular(lu.U[:, J], lu.U, lower=False, unit_diagonal=True)
    elif leftorright == "left":
        A = solve_triangular(lu.L[I, :].T, lu.L.T, lower=False, unit_diagonal=True).T
        B = np.array(M[I, :], copy=True)
    else:
        raise ValueError(leftorright)
    return A, B, lu


def local_update(Pi, tol, maxrank, leftorright, rule="exclusive", log_gaps=False):
    """Alg. 4.  ``Pi`` has shape (c_L, d, d', c_R).  Returns the two cores
    Y (c_L, d, r) and Y' (r, d', c_R), the matricised M and the LU record."""
    cL, d, d2, cR = Pi.shape
    M = Pi.reshape(cL * d, d2 * cR)
    A, B, lu = cross_interpolate(M, tol, maxrank, leftorright, rule, log_gaps)
    r = A.shape[1]
    Y = A.reshape(cL, d, r)
    Y2 = B.reshape(B.shape[0], d2, cR)
    return Y, Y2, M, lu


def left_frame(X, Lf, rows):
    """L'[(i, s), b] = sum_g L[i, g] X[g, s, b], truncated to ``rows``."""
    r0, d, r1 = X.shape
    T = Lf @ X.reshape(r0, d * r1)
    return T.reshape(-1, r1)[rows, :]


def right_frame(X, Rf, cols):
    """R'[a, (s, j)] = sum_g X[a, s, g] R[g, j], truncated to ``cols``."""
    r0, d, r1 = X.shape
    T = X.reshape(r0 * d, r1) @ Rf
    return T.reshape(r0, -1)[:, cols]
