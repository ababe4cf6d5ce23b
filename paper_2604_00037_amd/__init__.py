"""MI355X implementation of alternating cross interpolation (ACI) for
elementwise operations on tensor trains (M. K. Ritter).

``elementwise`` runs the full sweep (Alg. 1) in the HIP library
``libaci.so``; ``Session`` runs it sweep by sweep; ``elementwise_batched`` /
``Batch`` advance several products together; ``env_contract``, ``pi_eval``,
``prrlu`` and ``gather`` expose its single steps; ``tune_prrlu`` and
``tune_contract`` time the LDU launch shapes and the contraction tiles;
``tci`` builds a TT from point evaluations (2-site TCI); ``mpo_stencil``,
``mpo_apply`` and ``cubic_step`` apply TT operators and take an explicit step
of a cubic nonlinear equation (operator, then ACI of the nonlinearity);
``patched`` runs ACI on patches of fixed leading indices, refined where one
TT at the rank cap does not converge.  The library must be built (``python -m
paper_2604_00037_amd.build``); nothing falls back to the CPU.
"""

from .aci import (Batch, Context, Patch, Session, cubic_step, patched, default_context, elementwise, elementwise_batched,
                  env_contract, gather, linear_cubic, mlp_forward, mlp_init, mlp_train_step, mpo_apply, mpo_stencil,
                  pi_eval, proposal_dataset, proposal_features, prrlu, rook_check, rook_lu, rook_right_factor, tci,
                  tune_contract, tune_prrlu, TILES)

__all__ = ["Batch", "Context", "Session", "default_context", "elementwise", "elementwise_batched",
           "env_contract", "gather", "mlp_forward", "mlp_init", "mlp_train_step", "pi_eval", "proposal_dataset",
           "proposal_features",
           "prrlu", "rook_check", "rook_lu", "rook_right_factor", "tci", "tune_contract", "tune_prrlu", "TILES",
           "cubic_step", "linear_cubic", "mpo_apply", "mpo_stencil", "Patch", "patched"]
