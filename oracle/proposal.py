"""Learned pivot proposal: features, a small MLP and a seeded rook search.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

This is an extension beyond the paper: the full-pivot LDU of Alg. 2 stays
the reference and the fallback.  A rook search (pivot = largest residual in
its row *and* its column, found by alternating row and column scans on
residuals evaluated on demand) can replace the full search when it is
started from good rows; a small network scores the rows of the two-site
matrix from cheap features, and the factorisation it produces is accepted
only if the true residual max |M - L U'| is within the tolerance.

Definitions (both sides implement exactly these):

* Row features of the m x n two-site matrix M at a local update, row i:
    f0, f1  ||A^n[i, :]||_2 / max_i' ||A^n[i', :]||_2 for inputs n = 0, 1
            (A^n the left environment, rows a*d + s; 0 for a missing input
            or an all-zero environment);
    f2      1 if row i was a pivot row of the previous update of the same
            bond and direction, else 0;
    f3..f6  |M[i, c_t]| / max_{i', t} |M[i', c_t]| at columns
            c_t = floor((2t + 1) n / 8), t = 0..3 (0 when that max is 0).
  Norms and ratios in float64, features rounded to float32.
* Network 7 -> 64 -> 64 -> 1 with ReLU: parameters float32 (master copy);
  each layer rounds its inputs and its weights to float16, accumulates the
  products in float32 in index order without fused multiply-add
  (acc = acc + fp32(x16 * w16), starting from 0), then adds the float32
  bias.  The score is the last layer's output z (a logit).
* Training: binary cross entropy with logits on pivot labels, mean over the
  minibatch; gradients in float32 (sums over the minibatch in sample order,
  same rounding rule; sigmoid evaluated in float64 and rounded); Adam in
  float32 with bias corrections 1 - beta^t computed in float64 and rounded.
* Rook search with lazy residuals: residual(i, j) = M[i, j] - sum_t L[i, t]
  Up[t, j], evaluated as acc = M[i, j]; acc = acc - fp(L[i, t] * Up[t, j])
  for t = 0, 1, ... (no FMA), and exactly 0 on pivot rows and pivot
  columns.  Step k starts at the best-scored non-pivot row (ties: smallest
  row; without scores: the smallest non-pivot row), scans its residual row
  for the largest |value| over non-pivot columns (ties: smallest column),
  then that column for the largest over non-pivot rows; it stops when the
  row does not change or after ``max_iter`` scans, and takes the last
  (row, column) pair as pivot pi.  Stop rule as the exclusive rule of Alg. 2
  on |pi|: never accept |pi| <= tol after the first pivot, stop at maxrank.
  L[:, k] = residual column / pi (1 at the pivot row), Up[k, :] = residual
  row.  Right factor B = T^{-1} Up with T = Up[:, J] taken upper triangular
  (back substitution in index order).
* Acceptance: eps = max |M - L Up| (dense product); accepted iff
  eps <= tol.  Otherwise the full search of Alg. 2 is used.

Pins: the rook property checked by brute force on small matrices; exact
recovery of exact-rank matrices; B[:, J] = I; the network's gradients
against central differences of a float64 copy of the network (roundings
switched off); the loss of a separable toy problem decreasing under Adam
(tests/test_oracle_proposal.py).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .splitmix import splitmix64_stream

NFEAT = 7
H = 64
SAMPLE_COLS = 4


# ------------------------------------------------------------------ features
def sample_columns(n):
    return [((2 * t + 1) * n) // 8 for t in range(SAMPLE_COLS)]


def row_features(M, A_list, prev_rows):
    """Features (m x 7, float32) of the rows of M, as defined above."""
    M = np.asarray(M, dtype=np.float64)
    m, n = M.shape
    F = np.zeros((m, NFEAT), dtype=np.float64)
    for t in range(2):
        if t < len(A_list):
            A = np.asarray(A_list[t], dtype=np.float64)
            nr = np.sqrt((A * A).sum(axis=1))
            mx = nr.max() if nr.size else 0.0
            if mx > 0.0:
                F[:, t] = nr / mx
    for i in prev_rows:
        if 0 <= i < m:
            F[i, 2] = 1.0
    cols = sample_columns(n)
    S = np.abs(M[:, cols])
    mx = S.max() if S.size else 0.0
    if mx > 0.0:
        F[:, 3:7] = S / mx
    return F.astype(np.float32)


# ------------------------------------------------------------------- network
@dataclass
class MLP:
    W1: np.ndarray   # 7 x 64   float32
    b1: np.ndarray   # 64
    W2: np.ndarray   # 64 x 64
    b2: np.ndarray   # 64
    w3: np.ndarray   # 64
    b3: np.ndarray   # 1

    def params(self):
        return [self.W1, self.b1, self.W2, self.b2, self.w3, self.b3]


def mlp_init(seed):
    """Uniform(-s, s) weights with s = sqrt(6 / fan_in) from one SplitMix64
    stream (W1, W2, w3 in C order, then nothing else); biases 0."""
    sizes = [(NFEAT, H), (H, H), (H,)]
    total = sum(int(np.prod(s)) for s in sizes)
    z = np.array(splitmix64_stream(seed, total), dtype=np.uint64)
    u = (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53 * 2.0 - 1.0
    out, off = [], 0
    for s, fan in zip(sizes, (NFEAT, H, H)):
        cnt = int(np.prod(s))
        out.append((u[off:off + cnt] * np.sqrt(6.0 / fan)).astype(np.float32).reshape(s))
        off += cnt
    return MLP(out[0], np.zeros(H, np.float32), out[1], np.zeros(H, np.float32), out[2],
               np.zeros(1, np.float32))


def _f16(x):
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float32)


def _layer(X, W, b, rounding=True):
    """acc[s, o] = sum_k fp32(x16[s, k] * w16[k, o]) in k order, then + b."""
    if rounding:
        X = _f16(X)
        W = _f16(W)
        acc = np.zeros((X.shape[0], W.shape[1]), dtype=np.float32)
        for k in range(W.shape[0]):
            acc = acc + (X[:, k:k + 1] * W[k:k + 1, :]).astype(np.float32)
        return acc + b.astype(np.float32)
    X = np.asarray(X, dtype=np.float64)
    return X @ np.asarray(W, dtype=np.float64) + np.asarray(b, dtype=np.float64)


def mlp_forward(net, X, rounding=True):
    """Logits (float32, or float64 without rounding) and the cache for the
    backward pass."""
    z1 = _layer(X, net.W1, net.b1, rounding)
    a1 = np.maximum(z1, 0)
    z2 = _layer(a1, net.W2, net.b2, rounding)
    a2 = np.maximum(z2, 0)
    z3 = _layer(a2, net.w3.reshape(H, 1), net.b3, rounding)[:, 0]
    return z3, (X, z1, a1, z2, a2, z3)


def _acc_outer(U, V, rounding):
    """G[k, o] = sum_s U[s, k] * V[s, o] in sample order (float32, no FMA)."""
    if not rounding:
        return np.asarray(U, np.float64).T @ np.asarray(V, np.float64)
    G = np.zeros((U.shape[1], V.shape[1]), dtype=np.float32)
    for s in range(U.shape[0]):
        G = G + (U[s][:, None] * V[s][None, :]).astype(np.float32)
    return G


def _acc_sum(V, rounding):
    if not rounding:
        return np.asarray(V, np.float64).sum(axis=0)
    g = np.zeros(V.shape[1], dtype=np.float32)
    for s in range(V.shape[0]):
        g = g + V[s]
    return g


def _acc_back(D, W, rounding):
    """da[s, k] = sum_o D[s, o] * W[k, o] in o order (float32, no FMA)."""
    if not rounding:
        return np.asarray(D, np.float64) @ np.asarray(W, np.float64).T
    acc = np.zeros((D.shape[0], W.shape[0]), dtype=np.float32)
    for o in range(W.shape[1]):
        acc = acc + (D[:, o:o + 1] * W[:, o][None, :]).astype(np.float32)
    return acc


def bce_loss(z, y):
    z = np.asarray(z, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return float(np.mean(np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def mlp_grads(net, X, y, rounding=True):
    """Gradients of the mean BCE-with-logits loss w.r.t. the parameters.

    dz3 = (sigmoid(z3) - y) / B; the layers' weights enter as the float16
    values used in the forward pass and the activations as their float16
    inputs (the straight-through convention for the roundings)."""
    z3, (X0, z1, a1, z2, a2, _) = mlp_forward(net, X, rounding)
    B = X0.shape[0]
    ft = np.float32 if rounding else np.float64
    y = np.asarray(y, dtype=ft)
    sig = (1.0 / (1.0 + np.exp(-z3.astype(np.float64)))).astype(ft)
    dz3 = ((sig - y) / ft(B)).astype(ft)
    cast = _f16 if rounding else (lambda v: np.asarray(v, np.float64))
    x16, a1_16, a2_16 = cast(X0), cast(a1), cast(a2)
    W2_16, w3_16 = cast(net.W2), cast(net.w3)
    g_w3 = _acc_outer(a2_16, dz3[:, None], rounding)[:, 0]
    g_b3 = _acc_sum(dz3[:, None], rounding)
    da2 = (dz3[:, None] * w3_16[None, :]).astype(ft)
    dz2 = np.where(z2 > 0, da2, ft(0)).astype(ft)
    g_W2 = _acc_outer(a1_16, dz2, rounding)
    g_b2 = _acc_sum(dz2, rounding)
    da1 = _acc_back(dz2, W2_16, rounding)
    dz1 = np.where(z1 > 0, da1, ft(0)).astype(ft)
    g_W1 = _acc_outer(x16, dz1, rounding)
    g_b1 = _acc_sum(dz1, rounding)
    return [g_W1, g_b1, g_W2, g_b2, g_w3, g_b3], bce_loss(z3, y)


def adam_step(net, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in float32 (state: dict with m, v lists and step t)."""
    f = np.float32
    if not state:
        state["m"] = [np.zeros_like(p) for p in net.params()]
        state["v"] = [np.zeros_like(p) for p in net.params()]
        state["t"] = 0
    state["t"] += 1
    t = state["t"]
    # bias corrections computed in float64, then rounded to float32
    c1 = f(1.0 - b1 ** t)
    c2 = f(1.0 - b2 ** t)
    for p, g, m, v in zip(net.params(), grads, state["m"], state["v"]):
        g = g.astype(f)
        m[...] = f(b1) * m + f(1.0 - b1) * g
        v[...] = f(b2) * v + f(1.0 - b2) * (g * g)
        mh = m / c1
        vh = v / c2
        p[...] = p - f(lr) * mh / (np.sqrt(vh) + f(eps))


# ----------------------------------------------------------------- rook LDU
@dataclass
class Rook:
    rows: np.ndarray
    cols: np.ndarray
    rank: int
    eps_rook: float      # |pi| that stopped the search (0 when exhausted)
    L: np.ndarray        # m x rank
    Up: np.ndarray       # rank x n (residual rows, = D U)
    scans: int           # row + column scans performed


def _residual_row(M, L, Up, k, i, prow, pcol):
    r = M[i, :].copy()
    for t in range(k):
        r = r - L[i, t] * Up[t, :]
    r[list(pcol)] = 0.0
    if i in prow:
        r[:] = 0.0
    return r


def _residual_col(M, L, Up, k, j, prow, pcol):
    c = M[:, j].copy()
    for t in range(k):
        c = c - L[:, t] * Up[t, j]
    c[list(prow)] = 0.0
    if j in pcol:
        c[:] = 0.0
    return c


def rook_lu(M, tol, maxrank, scores=None, max_iter=8):
    M = np.asarray(M, dtype=np.float64)
    m, n = M.shape
    kmax = min(m, n, maxrank)
    L = np.zeros((m, kmax), dtype=np.float64)
    Up = np.zeros((kmax, n), dtype=np.float64)
    prow, pcol = [], []
    scans = 0
    eps = 0.0
    k = 0
    while k < min(m, n):
        free = [i for i in range(m) if i not in prow]
        if scores is None:
            i0 = free[0]
        else:
            s = np.asarray(scores, dtype=np.float32)
            best = max(s[i] for i in free)
            i0 = min(i for i in free if s[i] == best)
        it = 0
        while True:
            r = _residual_row(M, L, Up, k, i0, prow, pcol)
            a = np.abs(r)
            j0 = int(np.flatnonzero(a == a.max())[0])
            c = _residual_col(M, L, Up, k, j0, prow, pcol)
            b = np.abs(c)
            i1 = int(np.flatnonzero(b == b.max())[0])
            scans += 2
            it += 1
            if i1 == i0 or it >= max_iter:
                break
            i0 = i1
        piv = r[j0]
        v = abs(piv)
        if k == maxrank:
            eps = v
            break
        if k >= 1 and v <= tol:
            eps = v
            break
        if v == 0.0:
            # all-zero matrix at k == 0: one pivot at (smallest row, col 0)
            prow.append(i0)
            pcol.append(j0)
            L[i0, k] = 1.0
            k += 1
            eps = 0.0
            break
        L[:, k] = c / piv
        L[i0, k] = 1.0
        Up[k, :] = r
        prow.append(i0)
        pcol.append(j0)
        k += 1
    return Rook(np.array(prow, dtype=np.int64), np.array(pcol, dtype=np.int64), k, float(eps),
                L[:, :k].copy(), Up[:k, :].copy(), scans)


def rook_right_factor(rk):
    """B = T^{-1} Up, T = Up[:, J] upper triangular, back substitution."""
    r = rk.rank
    T = rk.Up[:, rk.cols]
    Y = np.zeros_like(rk.Up)
    for t in range(r - 1, -1, -1):
        acc = rk.Up[t, :].copy()
        for s in range(t + 1, r):
            acc = acc - T[t, s] * Y[s, :]
        Y[t, :] = acc / T[t, t] if T[t, t] != 0.0 else 0.0
    return Y


def rook_accept(M, rk, tol):
    """(accepted, eps) with eps = max |M - L Up| (dense product)."""
    R = np.asarray(M, dtype=np.float64) - rk.L @ rk.Up
    eps = float(np.abs(R).max()) if R.size else 0.0
    return eps <= tol, eps
