"""Python binding of the ACI library: argument marshalling over the C ABI.

Device memory and streams come from PyTorch (HIP build); every step of the
computation runs in the library's HIP kernels.  All tensors passed in must be
contiguous float64 (or complex128) tensors on the current HIP device.
"""

from __future__ import annotations

import atexit
import ctypes as C
import weakref

import numpy as np
from dataclasses import dataclass, field

import torch

from . import _lib

# Library objects still alive, released explicitly at interpreter exit
# (sessions and batches before the contexts they use), while the HIP runtime
# and the torch allocator a context may call back into are still up.
_live_children = weakref.WeakSet()
_live_contexts = weakref.WeakSet()


def _teardown():
    global _default_ctx
    if torch.cuda.is_available() and torch.cuda.is_initialized():
        torch.cuda.synchronize()
    for obj in list(_live_children):
        obj.close()
    for ctx in list(_live_contexts):
        ctx.close()
    _default_ctx = None


atexit.register(_teardown)

OPS = {"product": 0, "sum": 1, "abs2_mul": 2}
RULES = {"exclusive": 0, "literal": 1}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2}
F64 = 0
C128 = 1


def _code(t):
    """aci_dtype of a tensor."""
    return C128 if t.dtype == torch.complex128 else F64


def _check(lib, ctx, status, allow_warning=True):
    if status == 0 or (allow_warning and status > 0):
        return status
    msg = lib.aci_last_error(ctx).decode(errors="replace")
    name = _lib.STATUS_NAMES.get(status, str(status))
    raise _lib.HipError(f"{name}: {msg}")


def _dev_tensor(t, name, dtype=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    want = (dtype,) if dtype is not None else (torch.float64, torch.complex128)
    if t.dtype not in want:
        raise TypeError(f"{name} must be " + " or ".join(str(w).replace("torch.", "") for w in want))
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Context:
    """Owns an ``aci_ctx`` bound to the current device and torch stream.
    ``allocator="torch"`` gives the library's device memory to torch's
    caching allocator (aci_ctx_create_with_allocator) instead of hipMalloc."""

    def __init__(self, stream=None, allocator=None):
        self.lib = _lib.load()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        if allocator is None:
            st = self.lib.aci_ctx_create(C.byref(h), C.c_void_p(stream.cuda_stream))
        elif allocator == "torch":
            device = torch.cuda.current_device()

            def alloc(nbytes, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream)
                except RuntimeError:
                    return None

            def release(ptr, user):
                torch.cuda.caching_allocator_delete(ptr)

            # the callbacks must outlive the context
            self._alloc = _lib.ALLOC_FN(alloc)
            self._release = _lib.RELEASE_FN(release)
            st = self.lib.aci_ctx_create_with_allocator(C.byref(h), C.c_void_p(stream.cuda_stream), self._alloc,
                                                        self._release, None)
        else:
            raise ValueError("allocator must be None or 'torch'")
        _check(self.lib, None, st)
        self.h = h
        _live_contexts.add(self)

    def set_exchange_hooks(self, spin_limit=0, stall_step=-1, epoch_launches=0):
        """aci_ctx_set_exchange_hooks: spin limit of the LDU exchange waits,
        a test stall from pivot step ``stall_step`` on (-1: off), and the
        session epoch reset period (0: default)."""
        _check(self.lib, self.h, self.lib.aci_ctx_set_exchange_hooks(self.h, int(spin_limit), int(stall_step),
                                                                     int(epoch_launches)))

    def set_row_publication(self, eager_frac=0.6):
        """aci_ctx_set_row_publication: eager row publication of LDUs across
        XCDs above this fraction of the predicted pivot key (0: always,
        math.inf: winners publish late)."""
        _check(self.lib, self.h, self.lib.aci_ctx_set_row_publication(self.h, float(eager_frac)))

    def close(self):
        if getattr(self, "h", None):
            self.lib.aci_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx = None


def default_context():
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context()
    return _default_ctx


def _tt_struct(cores, keep):
    L = len(cores)
    d = (C.c_int32 * L)(*[int(c.shape[1]) for c in cores])
    ranks = (C.c_int32 * (L + 1))(*([int(cores[0].shape[0])] + [int(c.shape[2]) for c in cores]))
    ptrs = (C.c_void_p * L)(*[c.data_ptr() for c in cores])
    keep.extend([d, ranks, ptrs])
    return _lib.AciTT(L, d, ranks, ptrs)


@dataclass
class Info:
    status: int
    sweeps: int
    converged: bool
    ranks: list
    eps: list
    init_ranks: list
    sweep_ms: float
    records: list = field(default_factory=list)
    I: list = field(default_factory=list)    # I_0..I_L as lists of tuples (I_0, I_L empty)
    J: list = field(default_factory=list)    # J_1..J_{L+1} at index 1..L+1 (J_1, J_{L+1} empty)


class _DevArray:
    """A device buffer of the library seen by torch without a copy."""

    def __init__(self, ptr, shape, typestr):
        self.__cuda_array_interface__ = {"data": (int(ptr), False), "shape": tuple(shape), "typestr": typestr,
                                         "version": 3, "strides": None}


def linear_cubic(alpha, beta):
    """The op a_1 x_1 + ... + a_N x_N + b |x_1|^2 x_1 (ACI_OP_LINEAR_CUBIC)
    with alpha = (a_1, ..., a_N) and beta = b, for ``elementwise``,
    ``Session`` and ``Batch``."""
    return ("linear_cubic", tuple(alpha), beta)


def _coef_array(values, complex_, keep):
    vals = []
    for v in values:
        v = complex(v)
        if not complex_ and v.imag != 0.0:
            raise ValueError("complex coefficient for real inputs")
        vals.extend([v.real, v.imag] if complex_ else [v.real])
    arr = (C.c_double * len(vals))(*vals)
    keep.append(arr)
    return arr


def _op_code(op, opts, keep, complex_, n_inputs=None):
    """The aci_op of ``op``; a callable f(*tensors) -> tensor becomes
    ACI_OP_CUSTOM with options.pointwise applying it (torch ops on the
    library's stream, on (rows, ld) views of the two-site tensors);
    ``linear_cubic(alpha, beta)`` sets options.coef."""
    if isinstance(op, tuple) and op and op[0] == "linear_cubic":
        _, alpha, beta = op
        if n_inputs is not None and len(alpha) != n_inputs:
            raise ValueError("linear_cubic needs one coefficient per input")
        opts.coef = _coef_array(list(alpha) + [beta], complex_, keep)
        return 4
    if not callable(op):
        return OPS[op]
    typestr = "<c16" if complex_ else "<f8"
    dev = torch.device("cuda", torch.cuda.current_device())
    failures = []

    def apply(pis, n, out, rows, cols, ld, user, stream):
        try:
            st = torch.cuda.ExternalStream(stream) if stream else torch.cuda.default_stream(dev)
            with torch.cuda.stream(st):
                xs = [torch.as_tensor(_DevArray(pis[i], (rows, ld), typestr), device=dev) for i in range(n)]
                o = torch.as_tensor(_DevArray(out, (rows, ld), typestr), device=dev)
                o.copy_(op(*xs))
            return 0
        except Exception as exc:       # reported by the caller after the call returns
            failures.append(exc)
            return 1

    cb = _lib.POINTWISE_FN(apply)
    keep.extend([cb, failures])
    opts.pointwise = C.cast(cb, C.c_void_p)
    return 3


def _raise_pointwise(keep):
    for k in keep:
        if isinstance(k, list) and k and isinstance(k[0], Exception):
            raise k[0]


def _options(keep, maxiter, seed, init, stop_rule, precision, trace, fixed_sweeps, profile,
             low_precision_sweeps=0, use_graph=False, proposal=None, proposal_scans=0, sketch_rank=0):
    opts = _lib.AciOptions()
    opts.sketch_rank = int(sketch_rank)
    opts.low_precision_sweeps = int(low_precision_sweeps)
    opts.use_graph = 1 if use_graph else 0
    if proposal is not None:
        _dev_tensor(proposal, "proposal", torch.float32)
        if proposal.numel() != _lib.MLP_PARAMS:
            raise ValueError(f"proposal must be {_lib.MLP_PARAMS} float32 network parameters")
        keep.append(proposal)
        opts.proposal = C.c_void_p(proposal.data_ptr())
    opts.proposal_scans = int(proposal_scans)
    opts.maxiter = maxiter
    opts.seed = seed
    opts.stop_rule = RULES[stop_rule]
    opts.precision = PRECISIONS[precision]
    opts.trace = 1 if trace else 0
    opts.fixed_sweeps = 1 if fixed_sweeps else 0
    opts.profile = 1 if profile else 0
    if init is not None:
        for l, c in enumerate(init):
            _dev_tensor(c, f"init[{l}]")
        init_tt = _tt_struct(init, keep)
        keep.append(init_tt)
        opts.init = C.pointer(init_tt)
    return opts


def _inputs(inputs, keep):
    if len(inputs) < 1:
        raise ValueError("need at least one input TT")
    dt = inputs[0][0].dtype
    for n, X in enumerate(inputs):
        for l, c in enumerate(X):
            _dev_tensor(c, f"inputs[{n}][{l}]")
            if c.dim() != 3:
                raise ValueError("cores must be 3-dimensional")
            if c.dtype != dt:
                raise TypeError("all input cores must share one dtype")
    return (_lib.AciTT * len(inputs))(*[_tt_struct(X, keep) for X in inputs])


def _out_buffer(inputs, maxrank):
    L = len(inputs[0])
    dmax = max(int(c.shape[1]) for c in inputs[0])
    # capacity for every admissible rank profile (maxrank above the compiled
    # limit is rejected by the library itself)
    mr = min(int(maxrank), 512)
    cap = L * dmax * mr * mr
    return torch.empty(cap, dtype=inputs[0][0].dtype, device=inputs[0][0].device), cap


def _unpack(res, out, dims, status, trace):
    L = len(dims)
    ranks = [res.ranks[i] for i in range(L + 1)]
    cores = []
    for l in range(L):
        off = res.core_offset[l]
        cnt = ranks[l] * dims[l] * ranks[l + 1]
        cores.append(out[off:off + cnt].view(ranks[l], dims[l], ranks[l + 1]))
    records = []
    if trace:
        stride = res.record_stride
        for r in range(res.n_records):
            meta = [res.rec_meta[6 * r + i] for i in range(6)]
            rank = meta[3]
            records.append(dict(
                kind=("init", "LR", "RL")[meta[0]], sweep=meta[1], bond=meta[2], rank=rank,
                m=meta[4], n=meta[5], eps=res.rec_eps[r],
                rows=[res.rec_rows[stride * r + i] for i in range(rank)],
                cols=[res.rec_cols[stride * r + i] for i in range(rank)]))
    I = [[()]] + [[] for _ in range(L)]
    J = [[] for _ in range(L + 1)] + [[()]]
    for l in range(1, L):
        oi, oj, w = res.I_off[l - 1], res.J_off[l - 1], L - l
        I[l] = [tuple(res.I_idx[oi + k * l + t] for t in range(l)) for k in range(ranks[l])]
        J[l + 1] = [tuple(res.J_idx[oj + k * w + t] for t in range(w)) for k in range(ranks[l])]
    info = Info(status=status, sweeps=res.sweeps, converged=bool(res.converged),
                ranks=ranks, eps=[res.eps[i] for i in range(L - 1)],
                init_ranks=[res.init_ranks[i] for i in range(L + 1)],
                sweep_ms=res.sweep_ms, records=records, I=I, J=J)
    return cores, info


def elementwise(inputs, op="product", tol=1e-12, maxrank=64, *, maxiter=20, seed=0, init=None,
                stop_rule="exclusive", precision="fp64", trace=False, fixed_sweeps=False,
                low_precision_sweeps=0, proposal=None, proposal_scans=0, sketch_rank=0, ctx=None):
    """Alg. 1: returns (cores, info) with cores a list of device tensors of
    shape (r_{l-1}, d_l, r_l) approximating op(inputs) elementwise."""
    ctx = ctx or default_context()
    lib = ctx.lib
    keep = []
    tts = _inputs(inputs, keep)
    opts = _options(keep, maxiter, seed, init, stop_rule, precision, trace, fixed_sweeps, False,
                    low_precision_sweeps, False, proposal, proposal_scans, sketch_rank)
    code = _op_code(op, opts, keep, _code(inputs[0][0]) == 1, len(inputs))
    out, cap = _out_buffer(inputs, maxrank)
    res = _lib.AciResult()
    status = lib.aci_elementwise(ctx.h, tts, len(inputs), _code(inputs[0][0]), code, float(tol), int(maxrank),
                                 C.byref(opts), C.c_void_p(out.data_ptr()), cap, C.byref(res))
    try:
        _raise_pointwise(keep)
        _check(lib, ctx.h, status)
        return _unpack(res, out, [int(c.shape[1]) for c in inputs[0]], status, trace)
    finally:
        lib.aci_result_free(C.byref(res))


def kernel_name(kind, variant):
    """Kernel instance behind a launch-log entry, spelled as in the device
    profiler's kernel names."""
    b = {0: "false", 1: "true"}
    if kind == 0 and variant >= 2000000:
        rs, cs = divmod(variant - 2000000, 100)
        return f"prrlu_batch_kernel<{rs}, {cs}, false, 8>"
    if kind == 0 and variant >= 1000000:
        rs, cs = divmod(variant - 1000000, 100)
        return f"prrlu_kernel<{rs}, {cs}, false, false, 8>"
    if kind == 0 and variant >= 200000:
        cx, rest = divmod(variant - 200000, 100000)
        rs, cs = divmod(rest, 100)
        return f"prrlu_batch_kernel<{rs}, {cs}, {b[cx]}, 4>"
    if kind == 0 and 20000 <= variant < 30000:
        return {20001: "features_kernel", 20002: "mlp_forward_kernel", 20003: "rook_kernel",
                20004: "contract_kernel<-1, false>", 20005: "check_kernel", 20006: "commit_kernel",
                20007: "copy_rows_kernel", 20008: "rook_solve_kernel"}[variant]
    if kind == 0:
        cx, rest = divmod(variant, 100000)
        solo, rest = divmod(rest, 10000)
        rs, cs = divmod(rest, 100)
        return f"prrlu_kernel<{rs}, {cs}, {b[solo]}, {b[cx]}, 4>"
    if kind == 1:
        tile, rest = divmod(variant, 10000)
        cx, rest = divmod(rest, 1000)
        prec, op = divmod(rest, 100)
        op -= 1
        tl = "Tile<%d, %d> " % ((64, 64), (32, 64), (32, 32))[tile]
        return (f"contract_kernel<{op}, {b[cx]}, {tl}>" if prec == 0
                else f"contract_lp_kernel<{op}, {prec}, {b[cx]}, {tl}>")
    return "gather_kernel"


class Session:
    """Alg. 1 one sweep at a time: the constructor runs the initialisation,
    ``sweep(n)`` runs n sweeps, ``result()`` returns the current output."""

    def __init__(self, inputs, op="product", tol=1e-12, maxrank=64, *, maxiter=20, seed=0, init=None,
                 stop_rule="exclusive", precision="fp64", trace=False, fixed_sweeps=False,
                 profile=False, low_precision_sweeps=0, use_graph=False, proposal=None, proposal_scans=0,
                 tune=False, sketch_rank=0, ctx=None):
        self.ctx = ctx or default_context()
        self.inputs = inputs            # the library reads these until close()
        self.maxrank = maxrank
        self.trace = trace
        self._keep = []
        tts = _inputs(inputs, self._keep)
        opts = _options(self._keep, maxiter, seed, init, stop_rule, precision, trace, fixed_sweeps,
                        profile, low_precision_sweeps, use_graph, proposal, proposal_scans, sketch_rank)
        opts.tune = 1 if tune else 0
        self._init = init
        h = C.c_void_p()
        code = _op_code(op, opts, self._keep, _code(inputs[0][0]) == 1, len(inputs))
        st = self.ctx.lib.aci_session_create(self.ctx.h, tts, len(inputs), _code(inputs[0][0]), code, float(tol),
                                             int(maxrank), C.byref(opts), C.byref(h))
        _check(self.ctx.lib, self.ctx.h, st, allow_warning=False)
        self.h = h
        _live_children.add(self)

    def sweep(self, n=1):
        stats = _lib.AciSweepStats()
        st = self.ctx.lib.aci_session_sweep(self.h, int(n), C.byref(stats))
        _raise_pointwise(self._keep)
        _check(self.ctx.lib, self.ctx.h, st)
        L = len(self.inputs[0])
        return dict(status=st, sweeps_done=stats.sweeps_done, converged=bool(stats.converged),
                    kernel_ms=list(stats.kernel_ms), launches=list(stats.launches),
                    flops=list(stats.flops), pivots=stats.pivots,
                    ranks=[stats.ranks[i] for i in range(L + 1)], max_eps=stats.max_eps,
                    last_precision=[k for k, v in PRECISIONS.items() if v == stats.last_precision][0],
                    proposals_tried=stats.proposals_tried, proposals_accepted=stats.proposals_accepted,
                    proposal_scans=stats.proposal_scans, proposal_pivots=stats.proposal_pivots)

    def launches(self):
        """Launch log of the last ``sweep`` call (needs ``profile=True``): one
        dict per kernel launch with the kernel instance name as the device
        profiler reports it, the update it belongs to, its device time (us)
        and its algorithmic flops."""
        lib = self.ctx.lib
        n = C.c_int32(0)
        _check(lib, self.ctx.h, lib.aci_session_launches(self.h, None, 0, C.byref(n)))
        buf = (_lib.AciLaunch * max(1, n.value))()
        _check(lib, self.ctx.h, lib.aci_session_launches(self.h, buf, n.value, C.byref(n)))
        out = []
        for r in buf[:n.value]:
            out.append(dict(kind=("prrlu", "contract", "gather")[r.kind], kernel=kernel_name(r.kind, r.variant),
                            part=r.part, sweep=r.sweep, update=r.update, us=float(r.us), flops=r.flops))
        return out

    def result(self):
        out, cap = _out_buffer(self.inputs, self.maxrank)
        res = _lib.AciResult()
        st = self.ctx.lib.aci_session_result(self.h, C.c_void_p(out.data_ptr()), cap, C.byref(res))
        try:
            _check(self.ctx.lib, self.ctx.h, st)
            return _unpack(res, out, [int(c.shape[1]) for c in self.inputs[0]], st, self.trace)
        finally:
            self.ctx.lib.aci_result_free(C.byref(res))

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.aci_session_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ single steps
def env_contract(side, frames, cores, precision="fp64", ctx=None):
    """side "left": A = L X (c x d r1); side "right": B = X R (r0 d x c)."""
    ctx = ctx or default_context()
    n = len(frames)
    outs = []
    for F, X in zip(frames, cores):
        _dev_tensor(F, "frame")
        _dev_tensor(X, "core")
    r0, d, r1 = (int(s) for s in cores[0].shape)
    if side == "left":
        c = int(frames[0].shape[0])
        outs = [torch.empty(c, d * r1, dtype=cores[0].dtype, device=cores[0].device) for _ in range(n)]
    else:
        c = int(frames[0].shape[1])
        outs = [torch.empty(r0 * d, c, dtype=cores[0].dtype, device=cores[0].device) for _ in range(n)]
    fp = (C.c_void_p * n)(*[f.data_ptr() for f in frames])
    cp = (C.c_void_p * n)(*[x.data_ptr() for x in cores])
    op_ = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
    st = ctx.lib.aci_env_contract(ctx.h, _code(cores[0]), 0 if side == "left" else 1, n, fp, cp, op_, c, r0, d, r1,
                                  PRECISIONS[precision])
    _check(ctx.lib, ctx.h, st, allow_warning=False)
    return outs


def pi_eval(op, A, B, precision="fp64", tile=None, ctx=None):
    """M = op(A[0] @ B[0], A[1] @ B[1], ...) on the matrix cores; tile: one of
    TILES, or None for the default of the shape."""
    ctx = ctx or default_context()
    n = len(A)
    for a, b in zip(A, B):
        _dev_tensor(a, "A")
        _dev_tensor(b, "B")
    m = int(A[0].shape[0])
    ncol = int(B[0].shape[1])
    M = torch.empty(m, ncol, dtype=A[0].dtype, device=A[0].device)
    ap = (C.c_void_p * n)(*[a.data_ptr() for a in A])
    bp = (C.c_void_p * n)(*[b.data_ptr() for b in B])
    ks = (C.c_int32 * n)(*[int(a.shape[1]) for a in A])
    st = ctx.lib.aci_pi_eval(ctx.h, _code(A[0]), OPS[op], n, ap, bp, ks, m, ncol, C.c_void_p(M.data_ptr()), ncol,
                             PRECISIONS[precision], -1 if tile is None else TILES.index(tile))
    _check(ctx.lib, ctx.h, st, allow_warning=False)
    return M


def prrlu(M, tol, maxrank, stop_rule="exclusive", want_y=False, ctx=None, noalloc=False):
    """Alg. 2 on the device matrix M.  Returns dict(rows, cols, rank, eps, Y).
    noalloc: call aci_prrlu_noalloc (library workspace in a static device
    array) instead of aci_prrlu."""
    ctx = ctx or default_context()
    _dev_tensor(M, "M")
    m, n = (int(s) for s in M.shape)
    dev = M.device
    kcap = max(1, min(m, n, maxrank))
    rows = torch.full((kcap,), -1, dtype=torch.int32, device=dev)
    cols = torch.full((kcap,), -1, dtype=torch.int32, device=dev)
    rank = torch.zeros(1, dtype=torch.int32, device=dev)
    eps = torch.zeros(1, dtype=torch.float64, device=dev)
    Y = torch.zeros(kcap, n, dtype=M.dtype, device=dev) if want_y else None
    fn = ctx.lib.aci_prrlu_noalloc if noalloc else ctx.lib.aci_prrlu
    st = fn(ctx.h, _code(M), C.c_void_p(M.data_ptr()), m, n, n, float(tol), int(maxrank),
            RULES[stop_rule], C.c_void_p(rows.data_ptr()), C.c_void_p(cols.data_ptr()),
            C.c_void_p(rank.data_ptr()), C.c_void_p(eps.data_ptr()),
            C.c_void_p(Y.data_ptr() if Y is not None else 0), n)
    _check(ctx.lib, ctx.h, st, allow_warning=False)
    r = int(rank.item())
    return dict(rows=rows[:r].cpu().numpy(), cols=cols[:r].cpu().numpy(), rank=r,
                eps=float(eps.item()), Y=(Y[:r] if Y is not None else None))


def gather(side, src, idx, ld_out=None, ctx=None):
    """side "rows": out = src[idx, :]; side "cols": out = src[:, idx]."""
    ctx = ctx or default_context()
    _dev_tensor(src, "src")
    h, w = (int(s) for s in src.shape)
    idx_t = torch.as_tensor(idx, dtype=torch.int32, device=src.device).contiguous()
    r = int(idx_t.numel())
    rank = torch.tensor([r], dtype=torch.int32, device=src.device)
    if side == "rows":
        out = torch.zeros(r, w, dtype=src.dtype, device=src.device)
        ld = w
    else:
        out = torch.zeros(h, r, dtype=src.dtype, device=src.device)
        ld = r
    st = ctx.lib.aci_gather(ctx.h, _code(src), 0 if side == "rows" else 1, C.c_void_p(src.data_ptr()), h, w, w,
                            C.c_void_p(idx_t.data_ptr()), C.c_void_p(rank.data_ptr()),
                            C.c_void_p(out.data_ptr()), max(ld, 1))
    _check(ctx.lib, ctx.h, st, allow_warning=False)
    return out


def _stats_dict(stats, L):
    return dict(sweeps_done=stats.sweeps_done, converged=bool(stats.converged),
                kernel_ms=list(stats.kernel_ms), launches=list(stats.launches),
                flops=list(stats.flops), pivots=stats.pivots,
                ranks=[stats.ranks[i] for i in range(L + 1)], max_eps=stats.max_eps,
                last_precision=[k for k, v in PRECISIONS.items() if v == stats.last_precision][0])


def _batch_inputs(products, keep):
    counts = [len(p) for p in products]
    flat = [X for p in products for X in p]
    return _inputs(flat, keep), (C.c_int32 * len(counts))(*counts)


BATCH_MODES = {"auto": 0, "joint": 1, "overlapped": 2, "serial": 3}


class Batch:
    """Several elementwise operations advanced together; see aci_batch_create.
    ``mode``: "joint" (update by update, one LDU launch per update with every
    product on its own XCD), "overlapped" (one stream per product, LDUs spread
    over the XCDs), "serial", or "auto" (joint when possible)."""

    def __init__(self, products, op="product", tol=1e-12, maxrank=64, *, maxiter=20, seed=0,
                 stop_rule="exclusive", precision="fp64", fixed_sweeps=False, profile=False,
                 low_precision_sweeps=0, use_graph=False, tune=False, mode="auto", ctx=None):
        self.ctx = ctx or default_context()
        self.products = products
        self.maxrank = maxrank
        self._keep = []
        tts, counts = _batch_inputs(products, self._keep)
        opts = _options(self._keep, maxiter, seed, None, stop_rule, precision, False, fixed_sweeps,
                        profile, low_precision_sweeps, use_graph)
        opts.tune = 1 if tune else 0
        opts.batch_mode = BATCH_MODES[mode]
        h = C.c_void_p()
        code = _op_code(op, opts, self._keep, _code(products[0][0][0]) == 1)
        st = self.ctx.lib.aci_batch_create(self.ctx.h, tts, counts, len(products), _code(products[0][0][0]), code,
                                           float(tol),
                                           int(maxrank), C.byref(opts), C.byref(h))
        _check(self.ctx.lib, self.ctx.h, st, allow_warning=False)
        self.h = h
        _live_children.add(self)

    def sweep(self, n=1):
        stats = _lib.AciSweepStats()
        st = self.ctx.lib.aci_batch_sweep(self.h, int(n), C.byref(stats))
        _raise_pointwise(self._keep)
        _check(self.ctx.lib, self.ctx.h, st)
        d = _stats_dict(stats, len(self.products[0][0]))
        d["status"] = st
        return d

    def result(self, b):
        inputs = self.products[b]
        out, cap = _out_buffer(inputs, self.maxrank)
        res = _lib.AciResult()
        st = self.ctx.lib.aci_batch_result(self.h, int(b), C.c_void_p(out.data_ptr()), cap, C.byref(res))
        try:
            _check(self.ctx.lib, self.ctx.h, st)
            return _unpack(res, out, [int(c.shape[1]) for c in inputs[0]], st, False)
        finally:
            self.ctx.lib.aci_result_free(C.byref(res))

    def info(self, b):
        x, g = C.c_int32(0), C.c_int32(0)
        _check(self.ctx.lib, self.ctx.h, self.ctx.lib.aci_batch_info(self.h, int(b), C.byref(x), C.byref(g)))
        return x.value, g.value

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.aci_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def elementwise_batched(products, op="product", tol=1e-12, maxrank=64, *, maxiter=20, seed=0,
                        stop_rule="exclusive", precision="fp64", low_precision_sweeps=0,
                        use_graph=False, tune=False, mode="auto", ctx=None):
    """aci_elementwise_batched: returns [(cores, info)] per product."""
    ctx = ctx or default_context()
    lib = ctx.lib
    keep = []
    tts, counts = _batch_inputs(products, keep)
    opts = _options(keep, maxiter, seed, None, stop_rule, precision, False, False, False,
                    low_precision_sweeps, use_graph)
    opts.tune = 1 if tune else 0
    opts.batch_mode = BATCH_MODES[mode]
    bufs = [_out_buffer(p, maxrank) for p in products]
    outs = (C.c_void_p * len(products))(*[C.c_void_p(b.data_ptr()) for b, _ in bufs])
    caps = (C.c_int64 * len(products))(*[c for _, c in bufs])
    res = (_lib.AciResult * len(products))()
    code = _op_code(op, opts, keep, _code(products[0][0][0]) == 1)
    status = lib.aci_elementwise_batched(ctx.h, tts, counts, len(products), _code(products[0][0][0]), code,
                                         float(tol),
                                         int(maxrank), C.byref(opts), outs, caps, res)
    try:
        _raise_pointwise(keep)
        _check(lib, ctx.h, status)
        return [_unpack(res[b], bufs[b][0], [int(c.shape[1]) for c in products[b][0]], status, False)
                for b in range(len(products))]
    finally:
        for b in range(len(products)):
            lib.aci_result_free(C.byref(res[b]))


def tci(f, dims, tol=1e-12, maxrank=64, *, dtype=None, maxiter=20, pivots=None, stop_rule="exclusive",
        fixed_sweeps=False, ctx=None):
    """aci_tci: 2-site TCI of ``f``, a callable taking a device int32 tensor of
    multi-indices (count x L) and returning ``count`` values (float64 or,
    with ``dtype=torch.complex128``, complex).  ``pivots``: multi-indices
    seeding the index sets.  Returns (cores, info) as ``elementwise``."""
    ctx = ctx or default_context()
    dtype = dtype or torch.float64
    if dtype not in (torch.float64, torch.complex128):
        raise TypeError("dtype must be float64 or complex128")
    L = len(dims)
    dev = torch.device("cuda", torch.cuda.current_device())
    side = min(max(dims) * maxrank, _lib.MAX_MATRIX)
    P = side * side
    idx_t = torch.zeros((P, L), dtype=torch.int32, device=dev)
    val_t = torch.zeros(P, dtype=dtype, device=dev)
    failure = []

    def evaluate(count, L_, user, stream):
        try:
            with torch.cuda.stream(ctx.stream):
                vals = f(idx_t[:count])
                val_t[:count].copy_(torch.as_tensor(vals, device=dev).reshape(-1).to(dtype))
            return 0
        except Exception as exc:     # reported after the call returns
            failure.append(exc)
            return 1

    cb = _lib.EVAL_FN(evaluate)
    keep = []
    opts = _options(keep, maxiter, 0, None, stop_rule, "fp64", False, fixed_sweeps, False)
    d = (C.c_int32 * L)(*[int(x) for x in dims])
    if pivots is not None:
        piv = np.ascontiguousarray(np.asarray(pivots, dtype=np.int32).reshape(-1, L))
        pv, npv = piv.ctypes.data_as(C.c_void_p), piv.shape[0]
    else:
        piv, pv, npv = None, None, 0
    cap = sum(maxrank * int(x) * maxrank for x in dims)
    out = torch.zeros(cap, dtype=dtype, device=dev)
    res = _lib.AciResult()
    st = ctx.lib.aci_tci(ctx.h, L, d, 1 if dtype == torch.complex128 else 0, cb, None,
                         C.c_void_p(idx_t.data_ptr()), C.c_void_p(val_t.data_ptr()), P, pv, npv, float(tol),
                         int(maxrank), C.byref(opts), C.c_void_p(out.data_ptr()), cap, C.byref(res))
    try:
        if failure:
            raise failure[0]
        _check(ctx.lib, ctx.h, st)
        return _unpack(res, out, [int(x) for x in dims], st, False)
    finally:
        ctx.lib.aci_result_free(C.byref(res))


TILES = ["64x64", "32x64", "32x32"]


def tune_contract(m, k, n, dtype="f64", precision="fp64", ngroup=1, ctx=None):
    """aci_tune_contract: (best tile name, {tile name: mean us per launch})."""
    ctx = ctx or default_context()
    best = C.c_int32(0)
    us = (C.c_float * 3)()
    st = ctx.lib.aci_tune_contract(ctx.h, {"f64": 0, "c128": 1}[dtype], PRECISIONS[precision], int(ngroup),
                                   int(m), int(k), int(n), C.byref(best), us)
    _check(ctx.lib, ctx.h, st, allow_warning=False)
    return TILES[best.value], {TILES[t]: float(us[t]) for t in range(3)}


def tune_prrlu(m, n, maxrank, cap=0, ctx=None):
    """aci_tune_prrlu: (best group cap, [(cap, mean us), ...])."""
    ctx = ctx or default_context()
    best = C.c_int32(0)
    cand = (C.c_int32 * 16)()
    us = (C.c_float * 16)()
    cnt = C.c_int32(0)
    st = ctx.lib.aci_tune_prrlu(ctx.h, int(m), int(n), int(maxrank), int(cap), C.byref(best), cand, us, 16,
                                C.byref(cnt))
    _check(ctx.lib, ctx.h, st, allow_warning=False)
    return best.value, [(cand[i], us[i]) for i in range(cnt.value)]


# ------------------------------------------------------------ learned proposal
def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def proposal_features(M, env, prev_rows=None, ctx=None):
    """Row features (m x 7 float32) of the two-site matrix M (device, m x n)
    from the left environments env (list of <= 2 device matrices with m rows)
    and the previous pivot rows (device int32 tensor or None)."""
    ctx = ctx or default_context()
    _dev_tensor(M, "M", torch.float64)
    m, n = M.shape
    X = torch.empty((m, 7), dtype=torch.float32, device=M.device)
    envp = (C.c_void_p * 2)(*[_p(e) for e in env] + [None] * (2 - len(env)))
    ew = (C.c_int32 * 2)(*[int(e.shape[1]) for e in env] + [0] * (2 - len(env)))
    el = (C.c_int32 * 2)(*[int(e.stride(0)) for e in env] + [0] * (2 - len(env)))
    npv = 0 if prev_rows is None else int(prev_rows.numel())
    st = ctx.lib.aci_proposal_features(ctx.h, _p(M), m, n, int(M.stride(0)), envp, ew, el, len(env),
                                       _p(prev_rows) if npv else None, npv, _p(X))
    _check(ctx.lib, ctx.h, st, allow_warning=False)
    return X


def proposal_dataset(inputs, op="product", tol=1e-12, maxrank=64, *, capacity=1 << 20, maxiter=20, seed=0,
                     init=None, stop_rule="exclusive", fixed_sweeps=False, ctx=None):
    """aci_proposal_dataset: training rows (features X, labels y) recorded
    from the library's own plain FP64 sweeps of op(inputs).  Returns
    (X, y, sweeps) with X (count x 7) and y (count) device float32 views."""
    ctx = ctx or default_context()
    keep = []
    tts = _inputs(inputs, keep)
    if _code(inputs[0][0]) != F64:
        raise TypeError("the dataset is recorded from real inputs")
    opts = _options(keep, maxiter, seed, init, stop_rule, "fp64", False, fixed_sweeps, False)
    code = _op_code(op, opts, keep, False, len(inputs))
    dev = inputs[0][0].device
    X = torch.empty((capacity, 7), dtype=torch.float32, device=dev)
    y = torch.empty(capacity, dtype=torch.float32, device=dev)
    count = C.c_int64(0)
    sweeps = C.c_int32(0)
    st = ctx.lib.aci_proposal_dataset(ctx.h, tts, len(inputs), code, float(tol), int(maxrank), C.byref(opts),
                                      _p(X), _p(y), int(capacity), C.byref(count), C.byref(sweeps))
    _check(ctx.lib, ctx.h, st)
    return X[:count.value], y[:count.value], sweeps.value


def mlp_init(seed, device=None, ctx=None):
    """aci_mlp_init: initial network parameters (ACI_MLP_PARAMS float32 on
    the device) from SplitMix64(seed)."""
    ctx = ctx or default_context()
    p = torch.empty(_lib.MLP_PARAMS, dtype=torch.float32, device=device or torch.cuda.current_device())
    _check(ctx.lib, ctx.h, ctx.lib.aci_mlp_init(ctx.h, int(seed) & ((1 << 64) - 1), _p(p)), allow_warning=False)
    return p


def mlp_forward(params, X, ctx=None):
    ctx = ctx or default_context()
    out = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    st = ctx.lib.aci_mlp_forward(ctx.h, _p(params), _p(X), int(X.shape[0]), _p(out))
    _check(ctx.lib, ctx.h, st, allow_warning=False)
    return out


def mlp_train_step(params, adam_m, adam_v, step, X, y, lr=1e-3, want_grads=False, ctx=None):
    """One Adam step in place; returns (mean loss before the step, grads or None)."""
    ctx = ctx or default_context()
    g = torch.empty_like(params) if want_grads else None
    loss = C.c_float(0.0)
    st = ctx.lib.aci_mlp_train_step(ctx.h, _p(params), _p(adam_m), _p(adam_v), int(step), _p(X), _p(y),
                                    int(X.shape[0]), float(lr), _p(g), C.byref(loss))
    _check(ctx.lib, ctx.h, st, allow_warning=False)
    return loss.value, g


def rook_lu(M, tol, maxrank, scores=None, max_iter=8, ctx=None):
    """Rook search: dict(rows, cols, rank, eps, L (m x rank), Up (rank x n), scans)."""
    ctx = ctx or default_context()
    _dev_tensor(M, "M", torch.float64)
    m, n = M.shape
    dev = M.device
    rows = torch.zeros(maxrank, dtype=torch.int32, device=dev)
    cols = torch.zeros(maxrank, dtype=torch.int32, device=dev)
    ib = torch.zeros(4, dtype=torch.int32, device=dev)
    eps = torch.zeros(1, dtype=torch.float64, device=dev)
    L = torch.zeros((m, maxrank), dtype=torch.float64, device=dev)
    Up = torch.zeros((maxrank, n), dtype=torch.float64, device=dev)
    st = ctx.lib.aci_rook_lu(ctx.h, _p(M), m, n, int(M.stride(0)), float(tol), int(maxrank), _p(scores),
                             int(max_iter), _p(rows), _p(cols), C.c_void_p(ib.data_ptr()), _p(eps), _p(L),
                             maxrank, _p(Up), n, C.c_void_p(ib.data_ptr() + 4))
    _check(ctx.lib, ctx.h, st, allow_warning=False)
    r = int(ib[0].item())
    return dict(rows=rows[:r].cpu().numpy(), cols=cols[:r].cpu().numpy(), rank=r, eps=float(eps.item()),
                L=L[:, :r], Up=Up[:r], scans=int(ib[1].item()), _L=L, _Up=Up, _rows=rows, _cols=cols,
                _rank=ib[:1])


def rook_check(M, rk, tol, ctx=None):
    """(accepted, eps) of a rook_lu result against M."""
    ctx = ctx or default_context()
    m, n = M.shape
    eps = torch.zeros(1, dtype=torch.float64, device=M.device)
    acc = torch.zeros(1, dtype=torch.int32, device=M.device)
    st = ctx.lib.aci_rook_check(ctx.h, _p(M), m, n, int(M.stride(0)), _p(rk["_L"]), int(rk["_L"].shape[1]),
                                _p(rk["_Up"]), n, _p(rk["_rank"]), float(tol), _p(eps), _p(acc))
    _check(ctx.lib, ctx.h, st, allow_warning=False)
    return bool(acc.item()), float(eps.item())


def rook_right_factor(rk, ctx=None):
    ctx = ctx or default_context()
    Up = rk["_Up"]
    n = Up.shape[1]
    Y = torch.zeros_like(Up)
    st = ctx.lib.aci_rook_right_factor(ctx.h, _p(Up), n, _p(rk["_cols"]), _p(rk["_rank"]), n, _p(Y), n)
    _check(ctx.lib, ctx.h, st, allow_warning=False)
    return Y[:rk["rank"]]


# ------------------------------------------------------------ TT operators
def mpo_stencil(R, ndim, axis, weights, device=None):
    """Periodic stencil sum_delta w_delta S^delta along ``axis`` (weights =
    (w_-1, w_0, w_+1), (S^delta psi)(x) = psi(x + delta h)) of a box with 2^R
    points per axis, as MPO cores (w_{l-1}, 2, 2, w_l) on the device
    (aci_mpo_stencil builds them on the host)."""
    lib = _lib.load()
    L = int(R) * int(ndim)
    cores = (C.c_double * (36 * max(L, 1)))()
    ranks = (C.c_int32 * (L + 1))()
    w = (C.c_double * 3)(*[float(x) for x in weights])
    status = lib.aci_mpo_stencil(int(R), int(ndim), int(axis), w, cores, ranks)
    if status != 0:
        raise _lib.HipError(f"{_lib.STATUS_NAMES.get(status, status)}: aci_mpo_stencil")
    flat = np.ctypeslib.as_array(cores)
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    out = []
    for l in range(L):
        shape = (ranks[l], 2, 2, ranks[l + 1])
        out.append(torch.from_numpy(flat[36 * l:36 * l + int(np.prod(shape))].reshape(shape).copy()).to(dev))
    return out


def mpo_apply(mpo, x, ctx=None, timing=False):
    """Exact MPO-TT contraction (aci_mpo_apply): returns the cores of W x,
    shapes (w_{l-1} r_{l-1}, d_l, w_l r_l), bond index a r + c; with
    ``timing`` also the device milliseconds of its launches."""
    ctx = ctx or default_context()
    lib = ctx.lib
    keep = []
    L = len(x)
    if len(mpo) != L:
        raise ValueError("operator and TT differ in length")
    for l, c in enumerate(x):
        _dev_tensor(c, f"x[{l}]")
    for l, w in enumerate(mpo):
        _dev_tensor(w, f"mpo[{l}]", torch.float64)
        if w.dim() != 4:
            raise ValueError("operator cores must be 4-dimensional")
    tt = _tt_struct(x, keep)
    d = (C.c_int32 * L)(*[int(w.shape[1]) for w in mpo])
    wr = (C.c_int32 * (L + 1))(*([int(mpo[0].shape[0])] + [int(w.shape[3]) for w in mpo]))
    wp = (C.c_void_p * L)(*[w.data_ptr() for w in mpo])
    op = _lib.AciMPO(L, d, wr, wp)
    out = [torch.empty((wr[l] * int(x[l].shape[0]), int(x[l].shape[1]), wr[l + 1] * int(x[l].shape[2])),
                       dtype=x[0].dtype, device=x[0].device) for l in range(L)]
    optr = (C.c_void_p * L)(*[o.data_ptr() for o in out])
    ms = C.c_float(0.0)
    _check(lib, ctx.h, lib.aci_mpo_apply(ctx.h, C.byref(op), C.byref(tt), _code(x[0]), optr,
                                         C.byref(ms) if timing else None), False)
    return (out, ms.value) if timing else out


def cubic_step(psi, ndim, c0, c_lap, c3, tol=1e-12, maxrank=64, *, maxiter=20, init=None,
               stop_rule="exclusive", precision="fp64", trace=False, fixed_sweeps=False, ctx=None):
    """One explicit step y = c0 psi + c_lap sum_a D_a psi + c3 |psi|^2 psi on a
    periodic quantics grid (aci_cubic_step): the second differences D_a psi
    by exact MPO application, then ACI started from psi (or ``init``).
    Returns (cores, info) like ``elementwise``."""
    ctx = ctx or default_context()
    lib = ctx.lib
    keep = []
    for l, c in enumerate(psi):
        _dev_tensor(c, f"psi[{l}]")
    tt = _tt_struct(psi, keep)
    cx = _code(psi[0]) == 1
    coef = _coef_array([c0, c_lap, c3], cx, keep)
    opts = _options(keep, maxiter, 0, init, stop_rule, precision, trace, fixed_sweeps, False)
    out, cap = _out_buffer([psi], maxrank)
    res = _lib.AciResult()
    status = lib.aci_cubic_step(ctx.h, C.byref(tt), _code(psi[0]), int(ndim), coef, float(tol), int(maxrank),
                                C.byref(opts), C.c_void_p(out.data_ptr()), cap, C.byref(res))
    try:
        _check(lib, ctx.h, status)
        return _unpack(res, out, [int(c.shape[1]) for c in psi], status, trace)
    finally:
        lib.aci_result_free(C.byref(res))


# ------------------------------------------------------------ patched ACI
@dataclass
class Patch:
    prefix: tuple            # fixed leading indices
    cores: list              # TT over the remaining sites (device tensors)
    ranks: list
    converged: bool
    sweeps: int
    max_eps: float


def patched(inputs, op="product", tol=1e-12, maxrank=64, max_depth=2, *, maxiter=20, seed=0,
            stop_rule="exclusive", precision="fp64", ctx=None):
    """Patched ACI (aci_patched): f on patches of fixed leading indices,
    split where one TT at the rank cap does not converge.  Returns the kept
    patches (level by level, prefixes in lexicographic order) and the
    status."""
    ctx = ctx or default_context()
    lib = ctx.lib
    keep = []
    tts = _inputs(inputs, keep)
    opts = _options(keep, maxiter, seed, None, stop_rule, precision, False, False, False)
    cx = _code(inputs[0][0]) == 1
    code = _op_code(op, opts, keep, cx, len(inputs))
    res = _lib.AciPatchedResult()
    status = lib.aci_patched(ctx.h, tts, len(inputs), _code(inputs[0][0]), code, float(tol), int(maxrank),
                             int(max_depth), C.byref(opts), C.byref(res))
    try:
        _raise_pointwise(keep)
        _check(lib, ctx.h, status)
        L = res.L
        dims = [int(c.shape[1]) for c in inputs[0]]
        typestr = "<c16" if cx else "<f8"
        dev = inputs[0][0].device
        allc = torch.as_tensor(_DevArray(res.cores, (max(res.cores_elems, 1),), typestr), device=dev)
        out = []
        for i in range(res.n_patches):
            k = res.prefix_len[i]
            prefix = tuple(int(res.prefix[i * L + j]) for j in range(k))
            ranks = [int(res.ranks[i * (L + 1) + j]) for j in range(L - k + 1)]
            cores = []
            for j in range(L - k):
                off = res.core_offset[i * L + j]
                cnt = ranks[j] * dims[k + j] * ranks[j + 1]
                cores.append(allc[off:off + cnt].view(ranks[j], dims[k + j], ranks[j + 1]).clone())
            out.append(Patch(prefix, cores, ranks, bool(res.converged[i]), int(res.sweeps[i]),
                             float(res.max_eps[i])))
        torch.cuda.current_stream().synchronize()
        return out, status
    finally:
        lib.aci_patched_free(ctx.h, C.byref(res))
