"""2-site tensor cross interpolation (TCI) of a function given point by
point: the construction the paper uses for its input TTs (Sec. 3), whose
index-set optimisation ACI follows step for step (Sec. 2.6).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The sweep is that of ``oracle.aci`` with one change: the two-site tensor of
bond l is not contracted from frames but evaluated directly,

    Pi[a, s, s', b] = f(I_{l-1}[a] + (s, s') + J_{l+2}[b]),

matricised with row a*d_l + s and column s'*|J_{l+2}| + b (reading R18).
Initialisation: the index sets are those of the given pivot multi-indices
(default: the all-zero index), I_l = distinct prefixes of length l and J_l
= distinct suffixes starting at site l (nested by construction).  Each
sweep is a left-to-right then a right-to-left half of Alg. 4 local updates
(LDU with full pivoting, Alg. 2, right-interpolative); the index sets take
the pivot rows and columns after every update as in Alg. 1; the output
cores come from the last right-to-left half (Y_{l+1} = U_JJ^{-1} U, Y_1 =
M[:, J_2], reading R6); the sweeps stop when no right-to-left rank grew and
the largest right-to-left error estimate is <= tol (reading R11; the
initial ranks are the pivot-set sizes).

Pins (tests/test_oracle_tci.py): exact recovery of random low-rank TTs and
of rank-1 product functions by brute force over all entries, the
interpolation property at the bond-1 crosses, and a quantics Gaussian
against its closed form within the tolerance.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .ci import local_update


@dataclass
class TCIResult:
    cores: list
    ranks: list               # bond ranks r_1..r_{L-1} of the output
    eps: np.ndarray           # per-bond error estimate of the last R->L half sweep
    sweeps: int
    converged: bool
    I: list                   # I_0..I_L (I_l from the last update at l)
    J: list                   # J_1..J_{L+1} (index 0 unused)
    evaluations: int          # points evaluated
    trace: list = field(default_factory=list)


def two_site_points(I_prev, J_next, l, dims):
    """All multi-indices I_{l-1}[a] + (s, s') + J_{l+2}[b] of bond l in the
    order (a, s, s', b), as an int array of shape (c_L d d', L)."""
    L = len(dims)
    d, d2 = dims[l - 1], dims[l]
    cL, cR = len(I_prev), len(J_next)
    pts = np.zeros((cL, d, d2, cR, L), dtype=np.int64)
    if l > 1:
        pts[..., :l - 1] = np.asarray(I_prev, dtype=np.int64).reshape(cL, 1, 1, 1, l - 1)
    pts[..., l - 1] = np.arange(d).reshape(1, d, 1, 1)
    pts[..., l] = np.arange(d2).reshape(1, 1, d2, 1)
    if l + 1 < L:
        pts[..., l + 1:] = np.asarray(J_next, dtype=np.int64).reshape(1, 1, 1, cR, L - l - 1)
    return pts.reshape(-1, L)


def tci(f, dims, tol, maxrank, maxiter=20, pivots=None, rule="exclusive", log_gaps=False):
    """2-site TCI of f: (P, L) int array of multi-indices -> (P,) values."""
    L = len(dims)
    if pivots is None:
        pivots = [tuple([0] * L)]
    pivots = [tuple(int(v) for v in p) for p in pivots]
    I = [None] * (L + 1)
    J = [None] * (L + 2)
    I[0] = [()]
    J[L + 1] = [()]
    for l in range(1, L):
        I[l] = list(dict.fromkeys(p[:l] for p in pivots))
    for l in range(2, L + 1):
        J[l] = list(dict.fromkeys(p[l - 1:] for p in pivots))
    Y = [None] * L
    rho_prev = [len(J[l + 1]) for l in range(1, L)]
    rho = list(rho_prev)
    eps_rl = np.zeros(L - 1)
    trace = []
    evals = 0
    converged = False
    sweeps = 0

    def update(l, direction):
        nonlocal evals
        pts = two_site_points(I[l - 1], J[l + 2], l, dims)
        vals = np.asarray(f(pts))
        evals += pts.shape[0]
        Pi = vals.reshape(len(I[l - 1]), dims[l - 1], dims[l], len(J[l + 2]))
        Yl, Yr, M, lu = local_update(Pi, tol, maxrank, "right", rule, log_gaps)
        d, cR = dims[l - 1], len(J[l + 2])
        I[l] = [I[l - 1][int(p) // d] + (int(p) % d,) for p in lu.rows]
        J[l + 1] = [(int(q) // cR,) + J[l + 2][int(q) % cR] for q in lu.cols]
        trace.append(dict(dir=direction, bond=l, rank=lu.rank, eps=lu.eps, rows=lu.rows.copy(),
                          cols=lu.cols.copy(), min_gap=min(lu.gaps) if lu.gaps else None, shape=M.shape))
        return Yl, Yr, lu

    for it in range(1, maxiter + 1):
        sweeps = it
        for l in range(1, L):
            update(l, "LR")
        for l in range(L - 1, 0, -1):
            Yl, Yr, lu = update(l, "RL")
            Y[l] = Yr
            if l == 1:
                Y[0] = Yl
            rho[l - 1] = lu.rank
            eps_rl[l - 1] = lu.eps
        grew = any(rho[i] > rho_prev[i] for i in range(L - 1))
        rho_prev = list(rho)
        if not grew and eps_rl.max() <= tol:
            converged = True
            break
    return TCIResult(cores=Y, ranks=list(rho), eps=eps_rl.copy(), sweeps=sweeps, converged=converged, I=I, J=J,
                     evaluations=evals, trace=trace)
