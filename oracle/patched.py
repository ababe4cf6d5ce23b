"""Patched ACI: f(x^1, ..., x^N) as a collection of tensor trains on patches
of the index space, refined where one TT of bounded rank does not reach the
tolerance (the patched elementwise scheme named in Sec. 4).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

A patch is a prefix p = (sigma_1, ..., sigma_k) of fixed leading indices;
its tensor is f restricted to those indices, a TT over sites k+1..L.  The
restriction of an input TT is exact: the prefix vector
v_p = X_1[:, sigma_1, :] ... X_k[:, sigma_k, :] (1 x r_k) is absorbed into
the first free core, X'_{k+1} = v_p X_{k+1} (1 x d x r_{k+1}).

Refinement (a reading; the paper gives the scheme by reference only):
breadth first from the empty prefix, ACI (Alg. 1) runs on every patch of a
level with the same tolerance, rank cap, sweep limit and seeded default
Y_init; a patch whose sweep converged (Alg. 1's test) is kept, the others
are split into their d children, up to ``max_depth`` fixed indices, where
patches are kept whatever their state.  At least two free sites remain
(max_depth <= L - 2).  Patches are returned level by level, in
lexicographic order of their prefixes within a level.

Parity status: pinned by the restriction of an input TT against brute-force
slicing, by max_depth = 0 reducing to the unpatched ACI, by the kept
prefixes partitioning the index space, and by the assembled patches against
the exact f on small inputs (tests/test_oracle_patched.py).
"""

from dataclasses import dataclass

import numpy as np

from .aci import aci


@dataclass
class Patch:
    prefix: tuple          # fixed leading indices
    result: object         # ACIResult of the patch (cores over sites k+1..L)


def restrict(X, prefix):
    """The TT of X with its leading indices fixed to ``prefix``."""
    v = np.ones((1, 1), dtype=X[0].dtype)
    for l, s in enumerate(prefix):
        v = v @ X[l][:, s, :]
    k = len(prefix)
    first = np.einsum("ab,bsc->asc", v, X[k])
    return [first] + [np.array(c, copy=True) for c in X[k + 1:]]


def patched_aci(inputs, op, tol, maxrank, max_depth, maxiter=20, seed=0, log_gaps=False):
    """Returns the kept patches as a list of ``Patch``."""
    L = len(inputs[0])
    if not 0 <= max_depth <= L - 2:
        raise ValueError("max_depth must lie in [0, L - 2]")
    d = [c.shape[1] for c in inputs[0]]
    kept = []
    level = [()]
    for depth in range(max_depth + 1):
        split = []
        for p in level:
            res = aci([restrict(X, p) for X in inputs], op, tol, maxrank, maxiter=maxiter, seed=seed,
                      log_gaps=log_gaps)
            if res.converged or depth == max_depth:
                kept.append(Patch(p, res))
            else:
                split.append(p)
        level = [p + (s,) for p in split for s in range(d[depth])]
        if not level:
            break
    return kept


def assemble(patches, dims):
    """Dense tensor of the patched result (small inputs only)."""
    full = None
    for pt in patches:
        cores = pt.result.cores
        t = np.asarray(cores[0]).reshape(cores[0].shape[1], -1)
        for c in cores[1:]:
            t = t.reshape(-1, c.shape[0]) @ c.reshape(c.shape[0], -1)
        t = t.reshape(dims[len(pt.prefix):])
        if full is None:
            full = np.zeros(dims, dtype=t.dtype)
        full[pt.prefix] = t
    return full
