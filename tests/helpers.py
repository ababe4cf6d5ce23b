"""Shared helpers of the GPU parity tests."""

import numpy as np

GAP_TIE = 1e-10   # a pivot step is tie-free when its relative top-2 key gap exceeds this


def to_dev(cores, device="cuda"):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(c)).to(device) for c in cores]


def to_host(cores):
    return [c.detach().cpu().numpy() for c in cores]


def gemm_bound(A, B):
    """Elementwise forward error bound of a float64 product computed in any
    summation order: K * 2^-52 * (|A| @ |B|), K the inner dimension."""
    K = A.shape[1]
    return (K + 2) * 2.0 ** -52 * (np.abs(A) @ np.abs(B))


def compare_records(gpu_records, oracle_trace, label=""):
    """Pivot sets must agree record by record.  A mismatch is accepted only at
    a step the oracle logged as a near tie (relative top-2 gap < GAP_TIE);
    comparison stops there because later steps depend on the choice.
    Returns the number of records compared."""
    assert len(gpu_records) == len(oracle_trace), (label, len(gpu_records), len(oracle_trace))
    for i, (g, o) in enumerate(zip(gpu_records, oracle_trace)):
        kind = {"init": "init", "LR": "LR", "RL": "RL"}[o["dir"]]
        assert g["kind"] == kind and g["bond"] == o["bond"], (label, i, g["kind"], g["bond"], o)
        same = (g["rank"] == o["rank"] and list(g["rows"]) == [int(x) for x in o["rows"]]
                and list(g["cols"]) == [int(x) for x in o["cols"]])
        if not same:
            gap = o.get("min_gap")
            assert gap is not None and gap < GAP_TIE, (
                f"{label} record {i} ({kind} bond {o['bond']}): pivots differ at a tie-free step "
                f"(min gap {gap}); gpu rank {g['rank']} oracle rank {o['rank']}")
            return i
    return len(gpu_records)


def rel_max_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    scale = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / scale)
