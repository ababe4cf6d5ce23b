"""ctypes view of ``include/aci.h``.  Loads ``libaci.so`` from this package
directory and fails loudly when it is missing: there is no fallback."""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaci.so")

MAX_SITES = 128
MAX_INPUTS = 4
MAX_MATRIX = 1024

ACI_OK = 0
ACI_W_NOT_CONVERGED = 1
STATUS_NAMES = {
    0: "ACI_OK", 1: "ACI_W_NOT_CONVERGED", -1: "ACI_E_INVALID", -2: "ACI_E_DTYPE",
    -3: "ACI_E_HIP", -4: "ACI_E_NOMEM", -5: "ACI_E_NUMERIC", -6: "ACI_E_LIMIT",
    -7: "ACI_E_TIMEOUT",
}

EXPORTED = [
    "aci_ctx_create", "aci_ctx_create_with_allocator", "aci_ctx_destroy", "aci_last_error", "aci_elementwise",
    "aci_result_free", "aci_env_contract", "aci_pi_eval", "aci_prrlu", "aci_gather",
    "aci_session_create", "aci_session_sweep", "aci_session_result", "aci_session_launches",
    "aci_session_destroy", "aci_batch_create", "aci_batch_sweep", "aci_batch_result", "aci_batch_info",
    "aci_batch_destroy", "aci_elementwise_batched", "aci_tune_prrlu", "aci_tune_contract", "aci_tci",
    "aci_proposal_features", "aci_mlp_forward", "aci_mlp_train_step", "aci_rook_lu", "aci_rook_check",
    "aci_rook_right_factor", "aci_mpo_stencil", "aci_mpo_apply", "aci_cubic_step", "aci_patched",
    "aci_patched_free", "aci_ctx_set_exchange_hooks", "aci_ctx_set_row_publication", "aci_prrlu_noalloc",
    "aci_proposal_dataset", "aci_mlp_init",
]
MLP_PARAMS = 7 * 64 + 64 + 64 * 64 + 64 + 64 + 1


class AciTT(C.Structure):
    _fields_ = [
        ("L", C.c_int32),
        ("d", C.POINTER(C.c_int32)),
        ("ranks", C.POINTER(C.c_int32)),
        ("cores", C.POINTER(C.c_void_p)),
    ]


class AciPatchedResult(C.Structure):
    _fields_ = [
        ("n_patches", C.c_int32),
        ("L", C.c_int32),
        ("levels", C.c_int32),
        ("prefix_len", C.POINTER(C.c_int32)),
        ("prefix", C.POINTER(C.c_uint8)),
        ("ranks", C.POINTER(C.c_int32)),
        ("core_offset", C.POINTER(C.c_int64)),
        ("converged", C.POINTER(C.c_int32)),
        ("sweeps", C.POINTER(C.c_int32)),
        ("max_eps", C.POINTER(C.c_double)),
        ("cores", C.c_void_p),
        ("cores_elems", C.c_int64),
    ]


class AciMPO(C.Structure):
    _fields_ = [
        ("L", C.c_int32),
        ("d", C.POINTER(C.c_int32)),
        ("ranks", C.POINTER(C.c_int32)),
        ("cores", C.POINTER(C.c_void_p)),
    ]


class AciOptions(C.Structure):
    _fields_ = [
        ("maxiter", C.c_int32),
        ("seed", C.c_uint64),
        ("init", C.POINTER(AciTT)),
        ("stop_rule", C.c_int32),
        ("precision", C.c_int32),
        ("trace", C.c_int32),
        ("fixed_sweeps", C.c_int32),
        ("profile", C.c_int32),
        ("low_precision_sweeps", C.c_int32),
        ("use_graph", C.c_int32),
        ("tune", C.c_int32),
        ("proposal", C.c_void_p),
        ("proposal_scans", C.c_int32),
        ("batch_mode", C.c_int32),
        ("pointwise", C.c_void_p),
        ("pointwise_user", C.c_void_p),
        ("coef", C.POINTER(C.c_double)),
        ("sketch_rank", C.c_int32),
    ]


class AciResult(C.Structure):
    _fields_ = [
        ("L", C.c_int32),
        ("sweeps", C.c_int32),
        ("converged", C.c_int32),
        ("ranks", C.c_int32 * (MAX_SITES + 1)),
        ("eps", C.c_double * MAX_SITES),
        ("core_offset", C.c_int64 * MAX_SITES),
        ("out_elems", C.c_int64),
        ("init_ranks", C.c_int32 * (MAX_SITES + 1)),
        ("sweep_ms", C.c_double),
        ("n_records", C.c_int32),
        ("record_stride", C.c_int32),
        ("rec_meta", C.POINTER(C.c_int32)),
        ("rec_eps", C.POINTER(C.c_double)),
        ("rec_rows", C.POINTER(C.c_int32)),
        ("rec_cols", C.POINTER(C.c_int32)),
        ("I_off", C.c_int64 * MAX_SITES),
        ("J_off", C.c_int64 * MAX_SITES),
        ("I_idx", C.POINTER(C.c_uint8)),
        ("J_idx", C.POINTER(C.c_uint8)),
    ]


class AciSweepStats(C.Structure):
    _fields_ = [
        ("sweeps_done", C.c_int32),
        ("converged", C.c_int32),
        ("kernel_ms", C.c_double * 3),
        ("launches", C.c_int64 * 3),
        ("flops", C.c_double * 3),
        ("pivots", C.c_int32),
        ("ranks", C.c_int32 * (MAX_SITES + 1)),
        ("max_eps", C.c_double),
        ("last_precision", C.c_int32),
        ("proposals_tried", C.c_int32),
        ("proposals_accepted", C.c_int32),
        ("proposal_scans", C.c_int64),
        ("proposal_pivots", C.c_int64),
    ]


class AciLaunch(C.Structure):
    _fields_ = [
        ("kind", C.c_int32),
        ("variant", C.c_int32),
        ("part", C.c_int32),
        ("sweep", C.c_int32),
        ("update", C.c_int32),
        ("us", C.c_float),
        ("flops", C.c_double),
    ]


class HipError(RuntimeError):
    pass


_lib = None


# general elementwise f of ACI_OP_CUSTOM
POINTWISE_FN = C.CFUNCTYPE(C.c_int32, C.POINTER(C.c_void_p), C.c_int32, C.c_void_p, C.c_int64, C.c_int64,
                           C.c_int64, C.c_void_p, C.c_void_p)
# point evaluator of aci_tci
EVAL_FN = C.CFUNCTYPE(C.c_int32, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p)
# device allocator callbacks of aci_ctx_create_with_allocator
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


def load(path=LIB_PATH):
    """Load the library once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m paper_2604_00037_amd.build` "
            "(the HIP library is required; there is no CPU fallback)")
    lib = C.CDLL(path)
    vp = C.c_void_p
    i32 = C.c_int32
    lib.aci_ctx_create.argtypes = [C.POINTER(vp), vp]
    lib.aci_ctx_create.restype = C.c_int
    lib.aci_ctx_create_with_allocator.argtypes = [C.POINTER(vp), vp, ALLOC_FN, RELEASE_FN, vp]
    lib.aci_ctx_create_with_allocator.restype = C.c_int
    lib.aci_ctx_destroy.argtypes = [vp]
    lib.aci_ctx_destroy.restype = None
    lib.aci_ctx_set_exchange_hooks.argtypes = [vp, C.c_uint32, i32, C.c_int64]
    lib.aci_ctx_set_exchange_hooks.restype = C.c_int
    lib.aci_ctx_set_row_publication.argtypes = [vp, C.c_double]
    lib.aci_ctx_set_row_publication.restype = C.c_int
    lib.aci_last_error.argtypes = [vp]
    lib.aci_last_error.restype = C.c_char_p
    lib.aci_elementwise.argtypes = [vp, C.POINTER(AciTT), i32, i32, i32, C.c_double, i32,
                                    C.POINTER(AciOptions), vp, C.c_int64, C.POINTER(AciResult)]
    lib.aci_elementwise.restype = C.c_int
    lib.aci_result_free.argtypes = [C.POINTER(AciResult)]
    lib.aci_result_free.restype = None
    lib.aci_env_contract.argtypes = [vp, i32, i32, i32, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                     i32, i32, i32, i32, i32]
    lib.aci_env_contract.restype = C.c_int
    lib.aci_pi_eval.argtypes = [vp, i32, i32, i32, C.POINTER(vp), C.POINTER(vp), C.POINTER(i32),
                                i32, i32, vp, i32, i32, i32]
    lib.aci_pi_eval.restype = C.c_int
    lib.aci_prrlu.argtypes = [vp, i32, vp, i32, i32, i32, C.c_double, i32, i32, vp, vp, vp, vp, vp, i32]
    lib.aci_prrlu.restype = C.c_int
    lib.aci_prrlu_noalloc.argtypes = lib.aci_prrlu.argtypes
    lib.aci_prrlu_noalloc.restype = C.c_int
    lib.aci_gather.argtypes = [vp, i32, i32, vp, i32, i32, i32, vp, vp, vp, i32]
    lib.aci_gather.restype = C.c_int
    lib.aci_session_create.argtypes = [vp, C.POINTER(AciTT), i32, i32, i32, C.c_double, i32,
                                       C.POINTER(AciOptions), C.POINTER(vp)]
    lib.aci_session_create.restype = C.c_int
    lib.aci_session_sweep.argtypes = [vp, i32, C.POINTER(AciSweepStats)]
    lib.aci_session_sweep.restype = C.c_int
    lib.aci_session_result.argtypes = [vp, vp, C.c_int64, C.POINTER(AciResult)]
    lib.aci_session_result.restype = C.c_int
    lib.aci_session_launches.argtypes = [vp, C.POINTER(AciLaunch), i32, C.POINTER(i32)]
    lib.aci_session_launches.restype = C.c_int
    lib.aci_batch_create.argtypes = [vp, C.POINTER(AciTT), C.POINTER(i32), i32, i32, i32, C.c_double, i32,
                                     C.POINTER(AciOptions), C.POINTER(vp)]
    lib.aci_batch_create.restype = C.c_int
    lib.aci_batch_sweep.argtypes = [vp, i32, C.POINTER(AciSweepStats)]
    lib.aci_batch_sweep.restype = C.c_int
    lib.aci_batch_result.argtypes = [vp, i32, vp, C.c_int64, C.POINTER(AciResult)]
    lib.aci_batch_result.restype = C.c_int
    lib.aci_batch_info.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(i32)]
    lib.aci_batch_info.restype = C.c_int
    lib.aci_batch_destroy.argtypes = [vp]
    lib.aci_batch_destroy.restype = None
    lib.aci_elementwise_batched.argtypes = [vp, C.POINTER(AciTT), C.POINTER(i32), i32, i32, i32, C.c_double,
                                            i32, C.POINTER(AciOptions), C.POINTER(vp), C.POINTER(C.c_int64),
                                            C.POINTER(AciResult)]
    lib.aci_elementwise_batched.restype = C.c_int
    lib.aci_tune_prrlu.argtypes = [vp, i32, i32, i32, i32, C.POINTER(i32), C.POINTER(i32),
                                   C.POINTER(C.c_float), i32, C.POINTER(i32)]
    lib.aci_tune_prrlu.restype = C.c_int
    lib.aci_tune_contract.argtypes = [vp, i32, i32, i32, i32, i32, i32, C.POINTER(i32), C.POINTER(C.c_float)]
    lib.aci_tune_contract.restype = C.c_int
    lib.aci_tci.argtypes = [vp, i32, C.POINTER(i32), i32, EVAL_FN, vp, vp, vp, C.c_int64, vp, i32, C.c_double,
                            i32, C.POINTER(AciOptions), vp, C.c_int64, C.POINTER(AciResult)]
    lib.aci_tci.restype = C.c_int
    f32p = C.POINTER(C.c_float)
    i32p = C.POINTER(i32)
    lib.aci_proposal_features.argtypes = [vp, vp, i32, i32, i32, C.POINTER(vp), i32p, i32p, i32, vp, i32, vp]
    lib.aci_proposal_features.restype = C.c_int
    lib.aci_proposal_dataset.argtypes = [vp, C.POINTER(AciTT), i32, i32, C.c_double, i32, C.POINTER(AciOptions),
                                         vp, vp, C.c_int64, C.POINTER(C.c_int64), i32p]
    lib.aci_proposal_dataset.restype = C.c_int
    lib.aci_mlp_init.argtypes = [vp, C.c_uint64, vp]
    lib.aci_mlp_init.restype = C.c_int
    lib.aci_mlp_forward.argtypes = [vp, vp, vp, i32, vp]
    lib.aci_mlp_forward.restype = C.c_int
    lib.aci_mlp_train_step.argtypes = [vp, vp, vp, vp, i32, vp, vp, i32, C.c_float, vp, f32p]
    lib.aci_mlp_train_step.restype = C.c_int
    lib.aci_rook_lu.argtypes = [vp, vp, i32, i32, i32, C.c_double, i32, vp, i32, vp, vp, vp, vp, vp, i32, vp, i32, vp]
    lib.aci_rook_lu.restype = C.c_int
    lib.aci_rook_check.argtypes = [vp, vp, i32, i32, i32, vp, i32, vp, i32, vp, C.c_double, vp, vp]
    lib.aci_rook_check.restype = C.c_int
    lib.aci_rook_right_factor.argtypes = [vp, vp, i32, vp, vp, i32, vp, i32]
    lib.aci_rook_right_factor.restype = C.c_int
    lib.aci_mpo_stencil.argtypes = [i32, i32, i32, C.POINTER(C.c_double), C.POINTER(C.c_double), i32p]
    lib.aci_mpo_stencil.restype = C.c_int
    lib.aci_mpo_apply.argtypes = [vp, C.POINTER(AciMPO), C.POINTER(AciTT), i32, C.POINTER(vp), C.POINTER(C.c_float)]
    lib.aci_mpo_apply.restype = C.c_int
    lib.aci_cubic_step.argtypes = [vp, C.POINTER(AciTT), i32, i32, C.POINTER(C.c_double), C.c_double, i32,
                                   C.POINTER(AciOptions), vp, C.c_int64, C.POINTER(AciResult)]
    lib.aci_cubic_step.restype = C.c_int
    lib.aci_patched.argtypes = [vp, C.POINTER(AciTT), i32, i32, i32, C.c_double, i32, i32, C.POINTER(AciOptions),
                                C.POINTER(AciPatchedResult)]
    lib.aci_patched.restype = C.c_int
    lib.aci_patched_free.argtypes = [vp, C.POINTER(AciPatchedResult)]
    lib.aci_patched_free.restype = None
    lib.aci_session_destroy.argtypes = [vp]
    lib.aci_session_destroy.restype = None
    _lib = lib
    return lib
