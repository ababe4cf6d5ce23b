"""Plain CPU oracle for alternating cross interpolation (ACI).

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct
reference against which the HIP implementation is checked.  It may be
imported only by ``tests/``, by ``__graft_entry__.smoke()`` and by the
``cpu_baseline`` leg of ``bench.py``.  The product library never imports,
links or calls it, and it shares no code with the HIP path.

Everything is float64 (complex128 for complex inputs), written with NumPy
and SciPy primitives (matmul, triangular solve) as single steps, following
the algorithms of Appendix B of the paper in their order:

* ``prrlu``           -- Alg. 2 (LDU with full pivoting, greedy maxvol)
* ``cross_interpolate``, ``local_update`` -- Algs. 3 and 4
* ``left_frame``, ``right_frame``         -- Alg. 5 / Eq. (framesrecursive)
* ``aci``             -- Alg. 1 (initialisation, sweeps, convergence)
* ``splitmix64``      -- the counter-based generator of the default Y_init
* ``sketch``          -- random index sketch as the initial guess (the
                         RSI-style start of Sec. 2.8)
* ``reference``       -- exact Kronecker-delta product and SVD rounding,
                         an independent route to the Hadamard product
* ``proposal``        -- extension: row features, the small scoring network
                         (forward, gradients, Adam) and the seeded rook
                         search with its acceptance test
* ``tci``             -- 2-site TCI of a function given point by point (the
                         construction of the inputs, Sec. 3; the index-set
                         optimisation of Sec. 2.6 with Pi evaluated directly)
* ``patched``         -- patched ACI: f on patches of fixed leading indices,
                         refined where one TT at the rank cap does not
                         converge (the patched scheme named in Sec. 4)
* ``timestep``        -- TT operators on quantics grids (periodic stencil
                         MPOs, exact MPO-TT contraction) and one explicit
                         step of a cubic nonlinear equation with ACI started
                         from the current state (the use named in Sec. 4)

Parity status of each function is stated in its docstring.
"""

from .prrlu import prrlu, PrrLU
from .ci import cross_interpolate, local_update, left_frame, right_frame
from .aci import aci, ACIResult, apply_op, default_init_ranks
from .splitmix import splitmix64_stream, default_init
from .sketch import sketch_init, sketch_ranks
from . import reference
from . import proposal
from .tci import tci, TCIResult, two_site_points
from . import timestep
from . import patched

__all__ = [
    "prrlu", "PrrLU", "cross_interpolate", "local_update", "left_frame",
    "right_frame", "aci", "ACIResult", "apply_op", "default_init_ranks",
    "splitmix64_stream", "default_init", "sketch_init", "sketch_ranks", "reference", "proposal",
    "tci", "TCIResult", "two_site_points", "timestep", "patched",
]
