"""Shared helpers of the GPU parity tests."""

import numpy as np

GAP_TIE = 1e-10   # a pivot step is tie-free when its relative top-2 key gap exceeds this


def to_dev(cores, device="cuda"):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(c)).to(device) for c in cores]


def to_host(cores):
    return [c.detach().cpu().numpy() for c in cores]


def gemm_bound(A, B, precision="fp64"):
    """Elementwise forward error bound of a product computed in any summation
    order, from float64 operands:
      fp64:   (K + 2) u64 |A||B|;
      fp32:   operands rounded to fp32 (2 u32) and fp32 accumulation
              ((K + 2) u32): (K + 4) u32 |A||B|;
      bf16x3: x = hi + lo + r with hi = bf16(x), lo = bf16(x - hi), so
              |r| <= 2^-17 |x| (two bf16 roundings of 2^-9 each, plus the
              fp32 rounding); the dropped lo*lo term and the r terms add at
              most 2^-15 |a||b| per product, then fp32 accumulation.
    K is the inner dimension, |A||B| = |A| @ |B|."""
    K = A.shape[1]
    AB = np.abs(A) @ np.abs(B)
    if precision == "fp64":
        return (K + 2) * 2.0 ** -52 * AB
    if precision == "fp32":
        return (K + 4) * 2.0 ** -24 * AB
    if precision == "bf16x3":
        return (2.0 ** -15 + (K + 4) * 2.0 ** -24) * AB
    raise ValueError(precision)


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
