"""Independent routes to a Hadamard product, used to pin the ACI oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* ``delta_product`` -- the prior-art construction the paper compares against
  (section 1 and Appendix A): attach a Kronecker delta to the cores, i.e.
  Z_l[(a, a'), s, (b, b')] = X^1_l[a, s, b] X^2_l[a', s, b'].  Exact, rank
  r^1 r^2.
* ``tt_round`` -- SVD truncation of a TT (right-orthogonalise, then truncated
  SVDs left to right); the standard compression that follows the delta
  product.  It uses singular value decompositions only, never the pivoted
  LU of the method under test.
"""

from __future__ import annotations

import numpy as np


def delta_product(*tts):
    out = [np.asarray(c) for c in tts[0]]
    for X in tts[1:]:
        nxt = []
        for a, b in zip(out, X):
            r0a, d, r1a = a.shape
            r0b, _, r1b = b.shape
            c = np.einsum("asb,csd->acsbd", a, np.asarray(b)).reshape(r0a * r0b, d, r1a * r1b)
            nxt.append(c)
        out = nxt
    return out


def tt_round(cores, rtol=1e-14, maxrank=None):
    cores = [np.array(c, copy=True) for c in cores]
    L = len(cores)
    # right-orthogonalise
    for s in range(L - 1, 0, -1):
        r0, d, r1 = cores[s].shape
        q, r = np.linalg.qr(cores[s].reshape(r0, d * r1).T)
        k = q.shape[1]
        cores[s] = q.T.reshape(k, d, r1)
        cores[s - 1] = np.einsum("asb,bc->asc", cores[s - 1], r.T)
    # truncated SVDs left to right
    for s in range(L - 1):
        r0, d, r1 = cores[s].shape
        u, sv, vh = np.linalg.svd(cores[s].reshape(r0 * d, r1), full_matrices=False)
        k = int(np.count_nonzero(sv > rtol * sv[0])) if sv[0] > 0 else 1
        k = max(1, k if maxrank is None else min(k, maxrank))
        cores[s] = u[:, :k].reshape(r0, d, k)
        cores[s + 1] = np.einsum("ab,bsc->asc", sv[:k, None] * vh[:k], cores[s + 1])
    return cores
