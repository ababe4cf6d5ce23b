"""LDU factorisation with full pivoting (Alg. 2 of the paper, "LDU").

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Readings of the printed algorithm:

* the rank counter is advanced after every accepted pivot;
* the Schur complement update is the textbook one,
  S[k+1:, k+1:] -= S[k+1:, k] * S[k, k]^{-1} * S[k, k+1:], evaluated as
  ``l = S[i, k] / pivot`` followed by ``S[i, j] - l * S[k, j]`` (two
  roundings, no fused multiply-add);
* stop rule "exclusive" (default): a pivot whose magnitude is <= tol is
  never accepted, except the very first one; the returned error estimate is
  the largest remaining residual magnitude (0 once the matrix is exhausted).
  Rule "literal" reproduces the printed loop: the pivot is accepted first and
  the loop ends once |pivot| <= tol; the error is that pivot's magnitude
  (a pivot that is exactly zero is never accepted);
* argmax ties go to the smallest original row id, then the smallest
  original column id.  For complex matrices the search key is
  re*re + im*im and the reported magnitude is sqrt of that key;
* an all-zero matrix takes one pivot at the tie-break cell with value 0
  (the "zero path"): rank 1, error 0.

Complex arithmetic inside the elimination is spelled out in real operations
(products, sums, one division by |pivot|^2) so that every rounding step is
defined; the HIP kernel performs the same operations.

Pins: LAPACK ``?getc2`` (complete-pivoting LU) on tie-free full-rank
matrices, exact-rank products, the dense residual check of the error
estimate (tests/test_oracle_prrlu.py).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class PrrLU:
    rows: np.ndarray          # original row ids in pivot order (index set I)
    cols: np.ndarray          # original column ids in pivot order (index set J)
    rank: int
    eps: float                # error estimate
    pivots: np.ndarray        # pivot values pi_0 .. pi_{r-1}
    L: np.ndarray             # m x r, unit lower triangular in pivot order
    U: np.ndarray             # r x n, unit upper triangular in pivot order
    zero_path: bool = False
    gaps: list = field(default_factory=list)   # relative top-2 key gap per search

    @property
    def D(self):
        return np.diag(self.pivots)


def _search(Sr, Si, k, rows, cols):
    """argmax of the residual key over S[k:, k:] with the tie rule.
    Returns (p, q, key) with p, q positions in the (swapped) working array."""
    if Si is None:
        key = np.abs(Sr[k:, k:])
    else:
        a = Sr[k:, k:]
        b = Si[k:, k:]
        key = a * a + b * b
    best = key.max()
    ii, jj = np.nonzero(key == best)
    if len(ii) > 1:
        order = np.lexsort((cols[k + jj], rows[k + ii]))
        ii, jj = ii[order[0]], jj[order[0]]
    else:
        ii, jj = ii[0], jj[0]
    return k + int(ii), k + int(jj), best, key


def _gap(key, best):
    if key.size < 2 or best == 0.0:
        return 1.0
    second = np.partition(key.ravel(), -2)[-2]
    return float((best - second) / best)


def prrlu(M, tol, maxrank, rule="exclusive", log_gaps=False):
    """Factorise M ~ L D U with full pivoting; see module docstring."""
    M = np.asarray(M)
    is_complex = np.iscomplexobj(M)
    Sr = np.array(M.real, dtype=np.float64, copy=True)
    Si = np.array(M.imag, dtype=np.float64, copy=True) if is_complex else None
    m, n = Sr.shape
    rows = np.arange(m)
    cols = np.arange(n)
    kmax = min(m, n)
    if maxrank < 1:
        raise ValueError("maxrank must be >= 1")
    k = 0
    eps = 0.0
    piv_r, piv_i = [], []
    gaps = []
    zero_path = False
    while True:
        if k == kmax:
            if rule == "exclusive":
                eps = 0.0
            break
        p, q, best, key = _search(Sr, Si, k, rows, cols)
        v = float(np.sqrt(best)) if is_complex else float(best)
        if log_gaps:
            gaps.append(_gap(key, best))
        if rule == "exclusive":
            if k == maxrank:
                eps = v
                break
            if k >= 1 and v <= tol:
                eps = v
                break
        elif k >= 1 and v == 0.0:
            eps = 0.0
            break
        # swap row k <-> p and column k <-> q
        for S in (Sr, Si):
            if S is None:
                continue
            S[[k, p], :] = S[[p, k], :]
            S[:, [k, q]] = S[:, [q, k]]
        rows[[k, p]] = rows[[p, k]]
        cols[[k, q]] = cols[[q, k]]
        pr = Sr[k, k]
        pi = Si[k, k] if is_complex else 0.0
        if pr == 0.0 and pi == 0.0:
            # all-zero matrix: one pivot of value zero, nothing to eliminate
            zero_path = True
            piv_r.append(0.0)
            piv_i.append(0.0)
            k += 1
            eps = 0.0
            break
        if not is_complex:
            l = Sr[k + 1:, k] / pr
            Sr[k + 1:, k] = l
            Sr[k + 1:, k + 1:] -= np.outer(l, Sr[k, k + 1:])
        else:
            den = pr * pr + pi * pi
            cr = Sr[k + 1:, k].copy()
            ci = Si[k + 1:, k].copy()
            lr = (cr * pr + ci * pi) / den
            li = (ci * pr - cr * pi) / den
            Sr[k + 1:, k] = lr
            Si[k + 1:, k] = li
            ur = Sr[k, k + 1:]
            ui = Si[k, k + 1:]
            Sr[k + 1:, k + 1:] -= np.outer(lr, ur) - np.outer(li, ui)
            Si[k + 1:, k + 1:] -= np.outer(lr, ui) + np.outer(li, ur)
        piv_r.append(pr)
        piv_i.append(pi)
        k += 1
        if rule == "literal":
            eps = v
            if v <= tol or k == maxrank:
                break
    r = k
    dtype = np.complex128 if is_complex else np.float64
    pivots = np.array(piv_r) + (1j * np.array(piv_i) if is_complex else 0.0)
    pivots = pivots.astype(dtype)
    # unpack L (unit lower) and U (unit upper) in original row/column order
    Lsw = np.zeros((m, r), dtype=dtype)
    Usw = np.zeros((r, n), dtype=dtype)
    for t in range(r):
        Lsw[t, t] = 1.0
        if zero_path:
            Usw[t, t] = 1.0
            continue
        if is_complex:
            Lsw[t + 1:, t] = Sr[t + 1:, t] + 1j * Si[t + 1:, t]
            pr, pi = piv_r[t], piv_i[t]
            den = pr * pr + pi * pi
            sr = Sr[t, t + 1:]
            si = Si[t, t + 1:]
            Usw[t, t + 1:] = (sr * pr + si * pi) / den + 1j * ((si * pr - sr * pi) / den)
        else:
            Lsw[t + 1:, t] = Sr[t + 1:, t]
            Usw[t, t + 1:] = Sr[t, t + 1:] / piv_r[t]
        Usw[t, t] = 1.0
    L = np.zeros_like(Lsw)
    L[rows, :] = Lsw
    U = np.zeros_like(Usw)
    U[:, cols] = Usw
    return PrrLU(rows=rows[:r].copy(), cols=cols[:r].copy(), rank=r, eps=float(eps),
                 pivots=pivots, L=L, U=U, zero_path=zero_path, gaps=gaps)
