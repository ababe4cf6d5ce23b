"""Alternating cross interpolation driver (Alg. 1 of the paper).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Conventions (reading R18): sites l = 1..L, cores C order (r_{l-1}, d, r_l).
At bond l the two-site tensor is matricised as M[(a, s), (s', b)] with row
a*d + s and column s'*c_R + b, where a indexes I_{l-1} and b indexes
J_{l+2}.  Index sets are lists of tuples (multi-indices); I_0 = J_{L+1} =
[()] and L_0 = R_{L+1} = [[1]] (Alg. 1, first loop).

Steps, in the order of Alg. 1:

1. Initialisation: Y_init (given, or ``default_init``) is brought into
   CI-canonical form right to left: at site l the core is matricised as
   r_{l-1} x (d |J_{l+1}|), cross-interpolated (right-interpolative,
   reading R9), its pivot columns define J_l, the left factor M[:, J_l] is
   multiplied into the core at l-1, and the right frames R^n_l are built
   with Alg. 5.
2. Sweeps: left-to-right local updates (Pi^n from frames, Eq.
   (pifromframes); Pi = f(Pi^1..Pi^N); Alg. 4 with "right"; Leftframe),
   then right-to-left (Alg. 4 with "left"; Rightframe).
3. Output cores come from the last right-to-left half sweep (reading R6):
   Y_{l+1} = U_JJ^{-1} U of the bond-l factorisation and Y_1 = M[:, J_2] at
   bond 1; this is T_1 P_1^{-1} T_2 P_2^{-1} ... T_L of Eq. (ycicanonical).
4. Convergence (reading R11): after each sweep, stop if no right-to-left
   rank exceeds the previous sweep's (the initial ranks for the first sweep)
   and the largest right-to-left error estimate is <= tol.

Pins: brute force over all entries of small products, exact full-rank
reconstruction, the interpolation property on the bond-1 cross points, the
Kronecker-delta product with SVD rounding, closed-form Gaussian and Fourier
products, and special cases (tests/test_oracle_aci.py).  Whether the global
max error stays below tol is not guaranteed by the method; tests only check
it empirically ("parity unpinned" beyond that).
"""

from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from .ci import local_update, left_frame, right_frame
from .prrlu import prrlu
from .sketch import sketch_init
from .splitmix import default_init

OPS = ("product", "sum", "abs2_mul")


def apply_op(op, Pis):
    """Elementwise f applied to the N two-site tensors (Eq. (localupdate)).
    product: ((P1 * P2) * P3)...; sum: ((P1 + P2) + P3)...;
    abs2_mul (N = 1): |z|^2 z with |z|^2 = re*re + im*im."""
    if callable(op):
        return op(*Pis)
    if op == "product":
        out = Pis[0]
        for P in Pis[1:]:
            out = out * P
        return out
    if op == "sum":
        out = Pis[0]
        for P in Pis[1:]:
            out = out + P
        return out
    if op == "abs2_mul":
        if len(Pis) != 1:
            raise ValueError("abs2_mul takes one input")
        z = Pis[0]
        if np.iscomplexobj(z):
            a = z.real * z.real + z.imag * z.imag
            return a * z.real + 1j * (a * z.imag)
        return (z * z) * z
    raise ValueError(f"unknown op {op!r}")


def default_init_ranks(inputs, maxrank):
    """Bond ranks min_n r^n_l capped at maxrank (section 2.6)."""
    L = len(inputs[0])
    r = [1]
    for s in range(L - 1):
        r.append(min(min(x[s].shape[2] for x in inputs), maxrank))
    r.append(1)
    return r


@dataclass
class ACIResult:
    cores: list
    ranks: list               # bond ranks r_1..r_{L-1} of the output
    eps: np.ndarray           # per-bond error estimate of the last R->L sweep
    sweeps: int
    converged: bool
    I: list                   # I_0..I_L as lists of tuples (I_l from the last update at l)
    J: list                   # J_1..J_{L+1} (index 0 unused)
    init_ranks: list
    trace: list = field(default_factory=list)
    times: list = field(default_factory=list)   # wall clock after init and after each sweep


def _pi_tensors(inputs, Lf, Rf, l):
    """Pi^n = L^n_{l-1} X^n_l X^n_{l+1} R^n_{l+2}, shape (c_L, d, d', c_R),
    evaluated as A^n = L X_l (c_L d x r_l) and B^n = X_{l+1} R (r_l x d' c_R)."""
    out = []
    for n, X in enumerate(inputs):
        Xl, Xr = X[l - 1], X[l]
        r0, d, r1 = Xl.shape
        _, d2, r2 = Xr.shape
        A = (Lf[n][l - 1] @ Xl.reshape(r0, d * r1)).reshape(-1, r1)
        B = (Xr.reshape(r1 * d2, r2) @ Rf[n][l + 2]).reshape(r1, -1)
        cL = Lf[n][l - 1].shape[0]
        cR = Rf[n][l + 2].shape[1]
        out.append((A @ B).reshape(cL, d, d2, cR))
    return out


def _left_envs(inputs, Lf, l):
    """A^n = L^n_{l-1} X^n_l as (c_L d) x r_l matrices (rows a*d + s)."""
    out = []
    for n, X in enumerate(inputs):
        Xl = X[l - 1]
        r0, d, r1 = Xl.shape
        out.append((Lf[n][l - 1] @ Xl.reshape(r0, d * r1)).reshape(-1, r1))
    return out


def aci(inputs, op, tol, maxrank, maxiter=20, init=None, seed=0,
        rule="exclusive", log_gaps=False, record=None, sketch_rank=0):
    """Approximate f(x^1, ..., x^N) as a TT (Alg. 1).  ``inputs`` is a list
    of N TTs (lists of cores).  Returns an ``ACIResult``.  If ``record`` is
    a list, every local update appends its two-site matrix M, the left
    environments A^n and its pivots (training data of the learned
    proposal).  ``sketch_rank`` k > 0 (with no ``init``) starts from the
    random index sketch of size k (``sketch.py``) instead of the default
    random Y_init."""
    N = len(inputs)
    if N < 1:
        raise ValueError("need at least one input")
    L = len(inputs[0])
    if L < 2:
        raise ValueError("need at least two sites")
    dims = [c.shape[1] for c in inputs[0]]
    for X in inputs:
        if len(X) != L or [c.shape[1] for c in X] != dims:
            raise ValueError("inputs differ in length or local dimensions")
    is_complex = any(np.iscomplexobj(c) for X in inputs for c in X)
    dtype = np.complex128 if is_complex else np.float64
    inputs = [[np.asarray(c, dtype=dtype) for c in X] for X in inputs]

    Lf = [[None] * (L + 1) for _ in range(N)]
    Rf = [[None] * (L + 2) for _ in range(N)]
    for n in range(N):
        Lf[n][0] = np.ones((1, 1), dtype=dtype)
        Rf[n][L + 1] = np.ones((1, 1), dtype=dtype)
    I = [None] * (L + 1)
    J = [None] * (L + 2)
    I[0] = [()]
    J[L + 1] = [()]
    trace = []

    # ---- initialisation: CI-canonical form of Y_init, right to left
    if init is None and sketch_rank > 0:
        init = sketch_init(dims, sketch_rank, maxrank, seed, dtype=dtype)
    if init is None:
        init = default_init(default_init_ranks(inputs, maxrank), dims, seed, dtype=dtype)
    G = [np.array(c, dtype=dtype, copy=True) for c in init]
    for l in range(L, 1, -1):
        g = G[l - 1]
        r0, d, c = g.shape
        M = g.reshape(r0, d * c)
        lu = prrlu(M, tol, maxrank, rule=rule, log_gaps=log_gaps)
        cols = lu.cols
        J[l] = [(int(q) // c,) + J[l + 1][int(q) % c] for q in cols]
        trace.append(dict(sweep=0, dir="init", bond=l, rank=lu.rank, eps=lu.eps,
                          rows=lu.rows.copy(), cols=lu.cols.copy(),
                          min_gap=min(lu.gaps) if lu.gaps else None, shape=M.shape))
        A = M[:, cols]
        gl = G[l - 2]
        G[l - 2] = (gl.reshape(-1, gl.shape[2]) @ A).reshape(gl.shape[0], gl.shape[1], len(cols))
        for n in range(N):
            Rf[n][l] = right_frame(inputs[n][l - 1], Rf[n][l + 1], cols)
    init_ranks = [len(J[l + 1]) for l in range(1, L)]
    rho_prev = list(init_ranks)
    times = [time.perf_counter()]

    Y = [None] * L
    eps_rl = np.zeros(L - 1)
    rho = list(init_ranks)
    converged = False
    sweeps = 0
    for it in range(1, maxiter + 1):
        sweeps = it
        # ---- left-to-right half sweep
        for l in range(1, L):
            Pis = _pi_tensors(inputs, Lf, Rf, l)
            Pi = apply_op(op, Pis)
            _, _, M, lu = local_update(Pi, tol, maxrank, "right", rule, log_gaps)
            if record is not None:
                record.append(dict(sweep=it, dir="LR", bond=l, M=M.copy(), A=_left_envs(inputs, Lf, l),
                                   rows=lu.rows.copy(), cols=lu.cols.copy(), rank=lu.rank, eps=lu.eps))
            d = dims[l - 1]
            cR = Pi.shape[3]
            I[l] = [I[l - 1][int(p) // d] + (int(p) % d,) for p in lu.rows]
            J[l + 1] = [(int(q) // cR,) + J[l + 2][int(q) % cR] for q in lu.cols]
            for n in range(N):
                Lf[n][l] = left_frame(inputs[n][l - 1], Lf[n][l - 1], lu.rows)
            trace.append(dict(sweep=it, dir="LR", bond=l, rank=lu.rank, eps=lu.eps,
                              rows=lu.rows.copy(), cols=lu.cols.copy(),
                              min_gap=min(lu.gaps) if lu.gaps else None,
                              shape=M.shape))
        # ---- right-to-left half sweep
        for l in range(L - 1, 0, -1):
            Pis = _pi_tensors(inputs, Lf, Rf, l)
            Pi = apply_op(op, Pis)
            Yl, Yr, M, lu = local_update(Pi, tol, maxrank, "right", rule, log_gaps)
            if record is not None:
                record.append(dict(sweep=it, dir="RL", bond=l, M=M.copy(), A=_left_envs(inputs, Lf, l),
                                   rows=lu.rows.copy(), cols=lu.cols.copy(), rank=lu.rank, eps=lu.eps))
            # The output factors are those of Alg. 3 with P^{-1} in the right
            # factor: B = U_JJ^{-1} U becomes Y_{l+1}; only at bond 1 is the
            # left factor M[:, J] kept (reading R6).
            d = dims[l - 1]
            cR = Pi.shape[3]
            I[l] = [I[l - 1][int(p) // d] + (int(p) % d,) for p in lu.rows]
            J[l + 1] = [(int(q) // cR,) + J[l + 2][int(q) % cR] for q in lu.cols]
            for n in range(N):
                Rf[n][l + 1] = right_frame(inputs[n][l], Rf[n][l + 2], lu.cols)
            Y[l] = Yr
            if l == 1:
                Y[0] = Yl
            rho[l - 1] = lu.rank
            eps_rl[l - 1] = lu.eps
            trace.append(dict(sweep=it, dir="RL", bond=l, rank=lu.rank, eps=lu.eps,
                              rows=lu.rows.copy(), cols=lu.cols.copy(),
                              min_gap=min(lu.gaps) if lu.gaps else None,
                              shape=M.shape))
        times.append(time.perf_counter())
        grew = any(rho[i] > rho_prev[i] for i in range(L - 1))
        rho_prev = list(rho)
        if not grew and eps_rl.max() <= tol:
            converged = True
            break
    return ACIResult(cores=Y, ranks=list(rho), eps=eps_rl.copy(), sweeps=sweeps,
                     converged=converged, I=I, J=J, init_ranks=init_ranks, trace=trace,
                     times=times)
