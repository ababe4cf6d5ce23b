"""Tensor-train containers and helpers used to build and check inputs.

A TT is a list of cores; core ``s`` (site s+1) has shape ``(r_s, d, r_{s+1})``
in C order with ``r_0 = r_L = 1`` (the layout of the problem statement,
section 2.1 of the paper).  Cores are float64 or complex128 numpy arrays.
"""

from __future__ import annotations

import numpy as np


def tt_ranks(cores):
    """Bond ranks ``[r_0, r_1, ..., r_L]``."""
    return [cores[0].shape[0]] + [c.shape[2] for c in cores]


def random_tt(L, d, maxrank, seed, scale=None, dtype=np.float64):
    """Cores with i.i.d. N(0, scale^2) entries, drawn site by site in C order
    from ``numpy.random.Generator(PCG64(seed))``.  Interior ranks are
    ``maxrank`` (ranks 1 at both ends).  ``scale`` defaults to
    ``1/sqrt(maxrank)`` (variance 1/chi)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if scale is None:
        scale = 1.0 / np.sqrt(maxrank)
    ranks = [1] + [maxrank] * (L - 1) + [1]
    cores = []
    for s in range(L):
        shape = (ranks[s], d, ranks[s + 1])
        if np.issubdtype(np.dtype(dtype), np.complexfloating):
            re = rng.standard_normal(shape)
            im = rng.standard_normal(shape)
            c = (re + 1j * im) * (scale / np.sqrt(2.0))
        else:
            c = rng.standard_normal(shape) * scale
        cores.append(np.ascontiguousarray(c, dtype=dtype))
    return cores


def left_orthogonalise(cores):
    """Left-orthogonalise with reduced Householder QR, pushing R into the next
    core.  Represents the same tensor; ranks become min(r_{s-1} d, r_s)."""
    out = []
    carry = None
    L = len(cores)
    for s, c in enumerate(cores):
        c = np.asarray(c)
        if carry is not None:
            c = np.einsum("ab,bsc->asc", carry, c)
        r0, d, r1 = c.shape
        if s == L - 1:
            out.append(np.ascontiguousarray(c))
            break
        q, r = np.linalg.qr(c.reshape(r0 * d, r1), mode="reduced")
        out.append(np.ascontiguousarray(q.reshape(r0, d, q.shape[1])))
        carry = r
    return out


def tt_round(cores, maxrank, rtol=0.0):
    """TT rounding by QR and truncated SVD (I. Oseledets, TT-decomposition,
    2011): right-to-left orthogonalisation, then a left-to-right sweep that
    keeps at most ``maxrank`` singular values per bond and drops those below
    ``rtol`` times the largest.  Returns new cores (the same tensor when no
    value is dropped)."""
    cores = [np.asarray(c) for c in cores]
    L = len(cores)
    out = [c.copy() for c in cores]
    for s in range(L - 1, 0, -1):
        r0, d, r1 = out[s].shape
        q, r = np.linalg.qr(out[s].reshape(r0, d * r1).T, mode="reduced")
        out[s] = np.ascontiguousarray(q.T.reshape(q.shape[1], d, r1))
        out[s - 1] = np.einsum("asb,bc->asc", out[s - 1], r.T)
    for s in range(L - 1):
        r0, d, r1 = out[s].shape
        u, sv, vt = np.linalg.svd(out[s].reshape(r0 * d, r1), full_matrices=False)
        keep = int(min(maxrank, max(1, np.count_nonzero(sv > rtol * sv[0])))) if sv[0] > 0 else 1
        out[s] = np.ascontiguousarray(u[:, :keep].reshape(r0, d, keep))
        out[s + 1] = np.einsum("ab,bsc->asc", sv[:keep, None] * vt[:keep], out[s + 1])
    out[-1] = np.ascontiguousarray(out[-1])
    return out


def tt_scale(cores, factor):
    out = [c.copy() for c in cores]
    out[0] = out[0] * factor
    return out


def tt_full(cores):
    """Brute-force contraction of the whole TT into a dense array of shape
    ``(d_1, ..., d_L)``.  Only for small L."""
    t = np.asarray(cores[0])
    t = t.reshape(t.shape[1], t.shape[2])
    for c in cores[1:]:
        c = np.asarray(c)
        r0, d, r1 = c.shape
        t = t.reshape(-1, r0) @ c.reshape(r0, d * r1)
    dims = [c.shape[1] for c in cores]
    return t.reshape(dims)


def tt_eval(cores, points):
    """Evaluate the TT at integer multi-indices ``points`` (shape P x L) by
    multiplying the selected core slices left to right: at each site the
    points sharing a digit value take one matrix product."""
    points = np.asarray(points)
    P = points.shape[0]
    dtype = np.result_type(*[c.dtype for c in cores])
    v = np.ones((P, 1), dtype=dtype)
    for s, c in enumerate(cores):
        c = np.asarray(c)
        nxt = np.empty((P, c.shape[2]), dtype=dtype)
        for sigma in range(c.shape[1]):
            sel = points[:, s] == sigma
            if sel.any():
                nxt[sel] = v[sel] @ c[:, sigma, :]
        v = nxt
    return v[:, 0]


def tt_svd(full, d, maxrank, rtol=0.0, method="auto"):
    """Left-to-right TT-SVD of a dense array with ``d**L`` entries (given in
    C order over the sites).  Each bond keeps at most ``maxrank`` singular
    vectors and drops those below ``rtol * sigma_max``.

    ``full`` may be a numpy array or a torch tensor (any device).  With
    ``method="gram"`` the bond SVD is computed from the eigen-decomposition
    of the small Gram matrix W W^H, which needs one pass over W per bond and
    is the only practical route at 2^30 entries; ``"svd"`` uses a dense
    LAPACK SVD (accurate down to roundoff, for small arrays).
    """
    is_torch = not isinstance(full, np.ndarray)
    n_total = full.numel() if is_torch else full.size
    L = int(round(np.log(n_total) / np.log(d)))
    assert d ** L == n_total, "size is not a power of d"
    if method == "auto":
        method = "svd" if n_total <= (1 << 22) else "gram"
    cores = []
    W = full.reshape(1, -1)
    r = 1
    for s in range(L - 1):
        W = W.reshape(r * d, -1)
        if method == "svd":
            Wn = W if not is_torch else W.cpu().numpy()
            u, sv, vh = np.linalg.svd(Wn, full_matrices=False)
            k = _keep(sv, maxrank, rtol)
            core = u[:, :k]
            Wn = sv[:k, None] * vh[:k]
            W = Wn
        else:
            if is_torch:
                G = _gram_fixed_order(W).cpu().numpy()
            else:
                G = W @ W.conj().T
            lam, U = np.linalg.eigh(G)
            lam = lam[::-1]
            U = U[:, ::-1]
            sv = np.sqrt(np.maximum(lam, 0.0))
            # Gram eigenvalues carry round-off of order eps * lambda_max, so
            # singular values below ~sqrt(eps) sigma_max are not resolved; the
            # rank can never exceed the smaller side of W
            k = _keep(sv, min(maxrank, W.shape[0], W.shape[1]), max(rtol, 1e-7))
            core = np.ascontiguousarray(U[:, :k])
            if is_torch:
                import torch
                Ut = torch.from_numpy(core.conj().T.copy()).to(W.device)
                W = Ut @ W
            else:
                W = core.conj().T @ W
        cores.append(np.ascontiguousarray(core.reshape(r, d, k)))
        r = k
    last = W.reshape(r, d, 1)
    if is_torch:
        last = last.cpu().numpy()
    cores.append(np.ascontiguousarray(last))
    return cores


def _gram_fixed_order(W, chunk=8192):
    """W W^H for a device matrix W (m x K, K large) with a fixed summation
    order: the products of K-chunks of ``chunk`` columns as one batched
    product, then a sum over the chunks.  A single library GEMM may split a
    long K across workgroups and accumulate the parts atomically, so its
    result can differ in the last bits from run to run, and the
    eigenvectors of nearly equal eigenvalues (hence the TT cores) with it."""
    import torch
    m, K = W.shape
    if K <= chunk or K % chunk:
        return W @ W.conj().T.contiguous()
    B = K // chunk
    Wb = W.reshape(m, B, chunk).permute(1, 0, 2).contiguous()      # B x m x chunk
    Wh = Wb.conj().transpose(1, 2).contiguous()                     # B x chunk x m
    G = torch.bmm(Wb, Wh)
    del Wb, Wh
    return G.sum(dim=0)


def _keep(sv, maxrank, rtol):
    if sv.size == 0 or sv[0] == 0.0:
        return 1
    k = int(np.count_nonzero(sv > rtol * sv[0]))
    return max(1, min(k, maxrank))
