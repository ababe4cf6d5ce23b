"""Random index sketch as ACI's initial guess (RSI-style start).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. 2.8 describes recursive sketched interpolation (RSI): random sketches of
a user-chosen size k are contracted onto the input tensors to the right of
each site, so that one left-to-right pass forms two-site tensors to which f
is applied and factorises them.  For an elementwise f the sketch has to
select index points (f of random linear combinations of entries is not f of
the entries), so the sketch here is a random set of k nested right
multi-indices per bond, and the RSI pass is ACI's first left-to-right half
sweep started from those sets (reading R26).  It is realised as an initial
TT Y_init whose CI-canonical form (the initialisation of Alg. 1) selects
exactly the drawn index points:

* ranks rho_0 = rho_L = 1, rho_l = min(k, maxrank, d_1...d_l, d_{l+1}...d_L);
* one SplitMix64 stream (``splitmix.py``) seeded with ``seed``; for sites
  l = L, L-1, ..., 1 in this order: of the n = d_l rho_l columns (sigma, b)
  of the core matricised as rho_{l-1} x (d_l rho_l), column id sigma rho_l + b,
  draw rho_{l-1} without replacement by a partial Fisher-Yates shuffle
  (a = [0, n); for s = 0 .. rho_{l-1}-1: j = s + (z mod (n - s)) with z the
  next 64-bit output, swap a[s] and a[j], q_s = a[s]);
* core l is zero except core_l[s, q_s div rho_l, q_s mod rho_l] =
  (1 - s 2^-11) / (1 - b_s 2^-11) with b_s = q_s mod rho_l.

The initialisation factorises G_l = Y_l M_{l+1}[:, J_{l+1}], and
M_{l+1}[:, J_{l+1}] is diagonal with entries 1 - b 2^-11 (up to rounding), so
row s of G_l holds one non-zero of magnitude (1 - s 2^-11) (1 + O(2^-52)):
the pivots of Alg. 2 are (s, q_s) for s = 0, 1, ... in this order (all
magnitudes are at least 1/2, so a tolerance below 1/2 never stops the
initialisation early), and J_l = {(q_s div rho_l) ++ J_{l+1}[q_s mod rho_l]}
is the drawn random subset.

Pins (tests/test_oracle_sketch.py): the initialisation's pivots are the rows
in order at distinct columns and the index sets are nested and distinct;
over many seeds every column is drawn with the frequency a uniform draw
without replacement gives; ACI started from the sketch reproduces the exact
product at full rank (brute force over all entries).
"""

from __future__ import annotations

import numpy as np

from .splitmix import splitmix64_stream

_STEP = 2.0 ** -11


def sketch_ranks(dims, k, maxrank):
    L = len(dims)
    ranks = [1] * (L + 1)
    for l in range(1, L):
        left = int(np.prod(dims[:l], dtype=object))
        right = int(np.prod(dims[l:], dtype=object))
        ranks[l] = int(min(k, maxrank, left, right))
    return ranks


def sketch_init(dims, k, maxrank, seed, dtype=np.float64):
    """Cores of the random index sketch of size k (definition above)."""
    L = len(dims)
    rho = sketch_ranks(dims, k, maxrank)
    draws = iter(splitmix64_stream(seed, sum(rho[l - 1] for l in range(1, L + 1))))
    cores = [None] * L
    for l in range(L, 0, -1):
        d, r0, r1 = dims[l - 1], rho[l - 1], rho[l]
        n = d * r1
        a = list(range(n))
        core = np.zeros((r0, d, r1), dtype=dtype)
        for s in range(r0):
            j = s + int(next(draws) % (n - s))
            a[s], a[j] = a[j], a[s]
            q = a[s]
            b = q % r1
            core[s, q // r1, b] = (1.0 - s * _STEP) / (1.0 - b * _STEP)
        cores[l - 1] = core
    return cores
