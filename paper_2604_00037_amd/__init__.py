"""MI355X implementation of alternating cross interpolation (ACI) for
elementwise operations on tensor trains (M. K. Ritter).

``elementwise`` runs the full sweep (Alg. 1) in the HIP library
``libaci.so``; ``env_contract``, ``pi_eval``, ``prrlu`` and ``gather`` expose
its single steps.  The library must be built (``python -m
paper_2604_00037_amd.build``); nothing falls back to the CPU.
"""

from .aci import (Context, Session, default_context, elementwise, env_contract, gather, pi_eval,
                  prrlu)

__all__ = ["Context", "Session", "default_context", "elementwise", "env_contract", "gather", "pi_eval",
           "prrlu"]
