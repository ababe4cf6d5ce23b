"""Default initial guess Y_init when the caller gives none.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper starts from a random TT whose bond dimensions are the smallest
of the inputs' (section 2.6) and names no distribution.
Reading R10: entries are uniform on [-1, 1), produced by SplitMix64
(S. Vigna's published generator: state += 0x9E3779B97F4A7C15, then the
xor-shift-multiply finaliser with constants 0xBF58476D1CE4E5B9 and
0x94D049BB133111EB and shifts 30, 27, 31).  Each 64-bit output z becomes
((z >> 11) * 2^-53) * 2 - 1, which is exact in binary64.  Entries are drawn
site by site, each core in C order, from one stream seeded with ``seed``.
The C library implements the same definition independently.

Pin: the published reference outputs of SplitMix64 for seed 1234567
(tests/golden/splitmix64_seed1234567.txt).
"""

from __future__ import annotations

import numpy as np

_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def splitmix64_stream(seed, count):
    """``count`` consecutive 64-bit outputs (Python ints)."""
    s = seed & _MASK
    out = []
    for _ in range(count):
        s = (s + _GAMMA) & _MASK
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        out.append(z ^ (z >> 31))
    return out


def default_init(ranks, dims, seed, dtype=np.float64):
    """Cores of shape (ranks[s], dims[s], ranks[s+1]) filled from one stream.
    Complex cores take two consecutive draws per entry (real, imaginary)."""
    is_complex = np.issubdtype(np.dtype(dtype), np.complexfloating)
    sizes = [ranks[s] * dims[s] * ranks[s + 1] for s in range(len(dims))]
    per = 2 if is_complex else 1
    z = np.array(splitmix64_stream(seed, per * sum(sizes)), dtype=np.uint64)
    u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) * 2.0 - 1.0
    cores = []
    pos = 0
    for s, sz in enumerate(sizes):
        chunk = u[pos:pos + per * sz]
        pos += per * sz
        if is_complex:
            c = chunk[0::2] + 1j * chunk[1::2]
        else:
            c = chunk
        cores.append(np.ascontiguousarray(c.reshape(ranks[s], dims[s], ranks[s + 1]), dtype=dtype))
    return cores
