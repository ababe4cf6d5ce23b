/*
 * aci.h -- C ABI of the MI355X alternating cross interpolation (ACI) library.
 *
 * ACI (M. K. Ritter, "Fast elementwise operations on tensor trains with
 * alternating cross interpolation") approximates an elementwise function
 * f(x^1, ..., x^N) of N tensor trains directly as a tensor train y with
 * ||y - f(x)||_max <= tol (section 2.1, Eq. ydef:maxnorm), by sweeping
 * two-site local updates (Alg. 1).  Every step of the sweep runs in the
 * library's own HIP kernels for gfx950.
 *
 * Conventions shared by every entry point:
 *  - All tensors are row-major (C order).  A TT core of site l has shape
 *    (r_{l-1}, d_l, r_l); r_0 = r_L = 1.
 *  - Pointers documented as "device" must point to device memory of the
 *    device that was current when the context was created; "host" pointers
 *    point to host memory.  The library never takes ownership of caller
 *    memory and never frees it.
 *  - All work is ordered on the stream given to aci_ctx_create.  Entry
 *    points return after the work they enqueue has completed.
 *  - Every function returns an int status: ACI_OK (0), a positive warning
 *    or a negative error.  No C++ exception crosses the ABI.  The text of
 *    the last error is available from aci_last_error().
 *  - Real data is IEEE binary64 (double).  Complex data is interleaved
 *    binary64 pairs (re, im), i.e. C99 double complex.
 */
#ifndef ACI_H
#define ACI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define ACI_OK 0
#define ACI_W_NOT_CONVERGED 1   /* maxiter reached, or error estimate > tol at the rank cap */
#define ACI_E_INVALID (-1)      /* bad argument: null pointer, shape mismatch, tol < 0, ... */
#define ACI_E_DTYPE (-2)        /* unsupported dtype / precision combination */
#define ACI_E_HIP (-3)          /* a HIP runtime call failed (text in aci_last_error) */
#define ACI_E_NOMEM (-4)        /* device allocation failed, or output buffer too small */
#define ACI_E_NUMERIC (-5)      /* NaN or Inf met in a two-site tensor */
#define ACI_E_LIMIT (-6)        /* size beyond the compiled limits (see ACI_MAX_*) */
#define ACI_E_TIMEOUT (-7)      /* a device-side wait exceeded its spin limit */

/* ---- compiled limits ------------------------------------------------------ */
#define ACI_MAX_SITES 128       /* L */
#define ACI_MAX_DIM 4           /* local dimension d_l */
#define ACI_MAX_RANK 512        /* maxrank (output bond dimension cap) */
#define ACI_MAX_INPUTS 4        /* N */
#define ACI_MAX_MATRIX 1024     /* rows and columns of a matricised two-site tensor */
#define ACI_MAX_INPUT_RANK 2048 /* bond ranks of the input TTs (and of Y_init: ACI_MAX_MATRIX) */
#define ACI_MAX_BATCH 64        /* products of one batch */
#define ACI_MAX_MLP_BATCH 4096  /* samples of one training step of the scoring network */
#define ACI_MLP_FEATURES 7
#define ACI_MLP_HIDDEN 64
#define ACI_MLP_PARAMS (7 * 64 + 64 + 64 * 64 + 64 + 64 + 1)

typedef enum { ACI_F64 = 0, ACI_C128 = 1 } aci_dtype;

/* f of Eq. (localupdate), applied elementwise to the N two-site tensors:
 * PRODUCT: ((x1*x2)*x3)...; SUM: ((x1+x2)+x3)...; ABS2_MUL (N = 1): |x|^2 x;
 * CUSTOM: any f, applied by the caller's aci_pointwise_fn (options);
 * LINEAR_CUBIC: a1 x1 + a2 x2 + ... + aN xN + b |x1|^2 x1, coefficients from
 * options.coef, the right-hand side of an explicit step of a cubic
 * nonlinear equation (aci_cubic_step); evaluated as
 * (((a1 x1 + b (|x1|^2 x1)) + a2 x2) + ...) with |z|^2 = re*re + im*im. */
typedef enum { ACI_OP_PRODUCT = 0, ACI_OP_SUM = 1, ACI_OP_ABS2_MUL = 2, ACI_OP_CUSTOM = 3,
               ACI_OP_LINEAR_CUBIC = 4 } aci_op;

/* A general elementwise f (the problem statement's f: C^N -> C, Sec. 2):
 * for every i < rows, j < cols, out[i ld + j] = f(pis[0][i ld + j], ...,
 * pis[n-1][i ld + j]), where pis are device pointers to the N two-site
 * tensors Pi^n of the local update (elements of the dtype) and out is the
 * matrix the LDU then factorises.  rows x cols bounds the update's two-site
 * tensor (its exact extent lives on the device); entries outside it hold
 * arbitrary values and their results are never read.  Called from the host
 * once per local update while the sweep is enqueued; the work must be
 * ordered on `stream` (a hipStream_t) and must not wait for the device.
 * Returns 0 on success. */
typedef int32_t (*aci_pointwise_fn)(void* const* pis, int32_t n, void* out, int64_t rows, int64_t cols,
                                    int64_t ld, void* user, void* stream);

/* Precision of the contractions that form the two-site tensors.  The pivot
 * search, the Schur updates, the pivot-matrix solve and the error estimate are
 * always binary64. */
typedef enum { ACI_PREC_FP64 = 0, ACI_PREC_FP32 = 1, ACI_PREC_BF16X3 = 2 } aci_precision;

typedef struct aci_ctx aci_ctx;

/* A tensor train held in caller device memory (the inputs x^n of section 2.1). */
typedef struct {
  int32_t L;                 /* number of sites, 2 <= L <= ACI_MAX_SITES */
  const int32_t* d;          /* host, L local dimensions */
  const int32_t* ranks;      /* host, L+1 bond ranks, ranks[0] = ranks[L] = 1 */
  const void* const* cores;  /* host array of L device pointers; core l is
                                ranks[l] x d[l] x ranks[l+1], C order */
} aci_tt;

typedef struct {
  int32_t maxiter;       /* sweeps (Alg. 1 "maxiter"); <= 0 selects 20 */
  uint64_t seed;         /* SplitMix64 seed of the default Y_init */
  const aci_tt* init;    /* Y_init (section 2.6); NULL: random TT with ranks
                            min_n r^n_l (capped at maxrank), entries uniform on
                            [-1,1) drawn from SplitMix64(seed) site by site in
                            C order (two draws re, im per complex entry) */
  int32_t stop_rule;     /* 0: exclusive (default; never accept |pivot| <= tol
                            after the first, error = largest remaining
                            residual); 1: literal Alg. 2 (accept, then stop) */
  int32_t precision;     /* aci_precision of the contractions (environments and
                            two-site tensors); the LDU, the solve and the error
                            estimate are FP64 in every mode.  FP32 / BF16X3
                            start a precision ladder: low-precision sweeps
                            never count as converged; the sweeps switch to FP64
                            after a low-precision sweep that kept the
                            right-to-left ranks, or after low_precision_sweeps
                            of them.  In a low-precision sweep the LDU stops at
                            max(tol, floor |first pivot|) with floor
                            32 x 2^-24 (FP32) or 4 x 2^-15 (BF16X3), the
                            noise of its two-site matrix.  aci_elementwise
                            always ends with an FP64 sweep. */
  int32_t trace;         /* 1: record the pivots of every local update */
  int32_t fixed_sweeps;  /* 1: run exactly maxiter sweeps, no early exit */
  int32_t profile;       /* 1: time every kernel launch with HIP events
                            (aci_sweep_stats.kernel_ms) */
  int32_t low_precision_sweeps; /* ladder limit: 0 selects 4; < 0 never leaves
                            the low precision (sessions only, for timing) */
  int32_t use_graph;     /* 1: capture a sweep's launches once into a hipGraph
                            and replay it (ignored with profile or trace) */
  int32_t tune;          /* 1 = pick the tile of every contraction launch
                            with aci_tune_contract, and in overlapped batches
                            each product's LDU group count with
                            aci_tune_prrlu (both cached per context);
                            launch shapes beyond ACI_MAX_MATRIX keep the
                            default tile */
  const float* proposal; /* learned pivot proposal (extension): device array of
                            ACI_MLP_PARAMS network parameters, or NULL.  Every
                            local update then scores the rows, runs the seeded
                            rook search and keeps it if max |M - L Up| <= tol;
                            otherwise the LDU of Alg. 2 runs as usual */
  int32_t proposal_scans; /* rook scan-pair limit per pivot; 0 selects 8 */
  int32_t batch_mode;    /* batches: 0 = joint when possible, else overlapped;
                            1 = joint (error if not possible): the products
                            advance update by update together and the LDUs of
                            one update run as one launch, each product's
                            groups on one XCD; needs at most 12 products of
                            one length and no proposal; 2 = overlapped: every
                            product sweeps on its own stream, LDU groups
                            spread over the XCDs; 3 = one product after
                            another */
  aci_pointwise_fn pointwise;   /* f of ACI_OP_CUSTOM (NULL otherwise); sweeps
                                   with it are never captured into graphs */
  void* pointwise_user;         /* passed to pointwise */
  const double* coef;           /* host, ACI_OP_LINEAR_CUBIC only: a1..aN, b;
                                   N+1 doubles for ACI_F64, N+1 (re, im)
                                   pairs for ACI_C128; copied at the call */
  int32_t sketch_rank;          /* k > 0 with init NULL: start from a random
                                   index sketch of size k (the RSI-style start
                                   of Sec. 2.8) instead of the default Y_init:
                                   bond ranks rho_l = min(k, maxrank,
                                   d_1..d_l, d_{l+1}..d_L); for sites
                                   l = L..1, rho_{l-1} of the d_l rho_l
                                   columns (sigma, b), id sigma rho_l + b, are
                                   drawn without replacement from one
                                   SplitMix64(seed) stream by a partial
                                   Fisher-Yates shuffle (j = s + z mod (n - s),
                                   swap, take a[s]), and core l is zero except
                                   (1 - s 2^-11) / (1 - b 2^-11) at row s and
                                   its drawn column, so that the initialisation
                                   selects exactly the drawn index points;
                                   0: off */
} aci_options;

/* Result of aci_elementwise.  Output cores are written compactly, site after
 * site, into the caller's output buffer: core l starts at element
 * core_offset[l] and has shape ranks[l] x d_l x ranks[l+1]. */
typedef struct {
  int32_t L;
  int32_t sweeps;                       /* sweeps performed */
  int32_t converged;                    /* 1 if the convergence test of Alg. 1 passed */
  int32_t ranks[ACI_MAX_SITES + 1];     /* output bond ranks chi'_l */
  double eps[ACI_MAX_SITES];            /* eps[l-1]: error estimate of the last
                                           right-to-left update at bond l */
  int64_t core_offset[ACI_MAX_SITES];   /* element offsets in the output buffer */
  int64_t out_elems;                    /* elements written */
  int32_t init_ranks[ACI_MAX_SITES + 1];/* |J_{l+1}| after the CI-canonical init */
  double sweep_ms;                      /* device time of all sweeps (hipEvents) */
  /* trace (options.trace = 1): one record per prrLU call, in call order:
   * first the L-1 initialisation calls (sites L..2), then 2(L-1) per sweep. */
  int32_t n_records;
  int32_t record_stride;                /* = maxrank */
  int32_t* rec_meta;                    /* host, n_records x 6:
                                           kind (0 init, 1 L->R, 2 R->L), sweep,
                                           bond (site for init), rank, m, n */
  double* rec_eps;                      /* host, n_records */
  int32_t* rec_rows;                    /* host, n_records x record_stride */
  int32_t* rec_cols;                    /* host, n_records x record_stride */
  /* Nested index sets after the last sweep (Alg. 1, the pivots of its
   * right-to-left half): for bond l = 1..L-1, I_l holds ranks[l]
   * multi-indices of l digits (sigma_1..sigma_l, each < d), row-major at
   * I_idx + I_off[l-1]; J_{l+1} holds ranks[l] multi-indices of L-l digits
   * (sigma_{l+1}..sigma_L) at J_idx + J_off[l-1].  I_l is built from the
   * row pivots of the right-to-left update at bond l through the I_{l-1} of
   * the left-to-right half; J_{l+1} from its column pivots through J_{l+2}.
   * Host memory, released by aci_result_free. */
  int64_t I_off[ACI_MAX_SITES];
  int64_t J_off[ACI_MAX_SITES];
  uint8_t* I_idx;
  uint8_t* J_idx;
} aci_result;

/* Per-call statistics of aci_session_sweep.  Kernel classes: 0 = LDU with
 * full pivoting (including the pivot-matrix solve), 1 = contractions
 * (environments and two-site tensors with f), 2 = frame gathers.
 * Algorithmic flops of the sweeps of this call, from the shapes and ranks
 * actually met:
 *   class 0: sum over updates of sum_{k<r} 2 (m-k-1)(n-k-1), plus
 *            r (r-1) (n-r) for the right-to-left solve U_JJ^{-1} U;
 *   class 1: 2 m k n for every matrix product (k the inner dimension). */
typedef struct {
  int32_t sweeps_done;               /* sweeps of the session so far */
  int32_t converged;                 /* convergence test after the last sweep */
  double kernel_ms[3];               /* device time per class (options.profile) */
  int64_t launches[3];
  double flops[3];
  int32_t pivots;                    /* prrLU steps (pivots accepted) in this call */
  int32_t ranks[ACI_MAX_SITES + 1];  /* right-to-left ranks after the last sweep */
  double max_eps;                    /* largest right-to-left error estimate */
  int32_t last_precision;            /* aci_precision of the last sweep run */
  int32_t proposals_tried;           /* local updates with a learned proposal */
  int32_t proposals_accepted;        /* of which the rook result was kept */
  int64_t proposal_scans;            /* rook row/column scans of all proposals */
  int64_t proposal_pivots;           /* pivots of all rook searches (kept or not) */
} aci_sweep_stats;

/* One kernel launch of a profiled aci_session_sweep call (options.profile).
 * kind: 0 LDU with full pivoting, 1 contraction, 2 frame gather.
 * variant: kind 0: 100000*complex + 10000*solo + 100*RS + CS, the instance
 *          prrlu_kernel<RS, CS, solo, complex, 4> (RS row slots per wave, CS
 *          column slots per lane, solo = one workgroup, four waves), or
 *          1000000 + 100*RS + CS for the eight-wave instance
 *          prrlu_kernel<RS, CS, false, false, 8> of real multi-group
 *          factorisations with 16 or more rows per group, CS < 16 and
 *          RS CS <= 32, 200000 + 100000*complex + 100*RS + CS for the joint
 *          batch LDU prrlu_batch_kernel<RS, CS, complex, 4>, 2000000 +
 *          100*RS + CS for its eight-wave instance
 *          prrlu_batch_kernel<RS, CS, false, 8>, or 20001..20008 for the
 *          learned-proposal kernels; kind 1: 10000*tile + 1000*complex +
 *          100*precision + op + 1 with op the fused epilogue (-1 none, else
 *          aci_op) and tile as in aci_tune_contract: instance
 *          contract_kernel<op, complex, Tile<TM, TN> > (FP64) or
 *          contract_lp_kernel<op, precision, complex, Tile<TM, TN> >;
 *          kind 2: 0.
 * part: kind 1 only: 1 environment product, 2 two-site tensor (with f).
 * update: local update within its sweep, 0..2(L-1)-1 (left-to-right first).
 * flops: algorithmic flops of this launch, counted as in aci_sweep_stats. */
typedef struct {
  int32_t kind;
  int32_t variant;
  int32_t part;
  int32_t sweep;                     /* sweep index within the session, from 0 */
  int32_t update;
  float us;                          /* device time from HIP events on the stream */
  double flops;
} aci_launch;

/* A sweep session keeps the state of Alg. 1 between calls (frames, index
 * sets, cached environments) so that sweeps can be run one at a time, e.g.
 * for timing or to stop on a custom criterion.  It owns its device
 * workspace; the input cores must stay valid until aci_session_destroy. */
typedef struct aci_session aci_session;

/* Validates the problem exactly like aci_elementwise, allocates the
 * workspace and runs the initialisation of Alg. 1 (CI-canonical Y_init and
 * the initial right frames). */
int aci_session_create(aci_ctx* ctx, const aci_tt* inputs, int32_t n_inputs, int32_t dtype,
                       int32_t op, double tol, int32_t maxrank, const aci_options* opt,
                       aci_session** session);
/* Runs nsweeps sweeps (left-to-right then right-to-left) and the
 * convergence test after each; stops early once converged unless
 * options.fixed_sweeps.  stats may be NULL.  Returns ACI_OK when converged,
 * ACI_W_NOT_CONVERGED otherwise, or an error. */
int aci_session_sweep(aci_session* session, int32_t nsweeps, aci_sweep_stats* stats);
/* Writes the current output cores (those of the last right-to-left half
 * sweep) like aci_elementwise does. */
int aci_session_result(aci_session* session, void* out, int64_t out_capacity, aci_result* result);
/* Copies the launch log of the most recent aci_session_sweep call (empty
 * unless options.profile) into out[0 .. min(capacity, count)); *count gets
 * the number of launches.  out may be NULL to query the count. */
int aci_session_launches(aci_session* session, aci_launch* out, int32_t capacity, int32_t* count);
void aci_session_destroy(aci_session* session);

/* Context: owns the device workspace, bound to the current device and to
 * `stream` (a hipStream_t; NULL = the null stream). */
int aci_ctx_create(aci_ctx** ctx, void* stream);
/* The same, with the library's device memory (session and batch workspaces,
 * step and tuning buffers) taken from the caller's allocator instead of
 * hipMalloc, for callers whose memory pool should own it (for instance a
 * framework's caching allocator).  alloc(bytes, user) returns device memory
 * of the current device, aligned to at least 256 bytes, or NULL (the call
 * then fails with ACI_E_NOMEM); release(ptr, user) gives it back.  The
 * library synchronises every stream that used a buffer before releasing
 * it.  Batches created on this context use the same allocator.  Pinned host
 * buffers still come from hipHostMalloc.  ACI_E_INVALID if alloc or release
 * is NULL. */
int aci_ctx_create_with_allocator(aci_ctx** ctx, void* stream, void* (*alloc)(size_t bytes, void* user),
                                  void (*release)(void* ptr, void* user), void* user);
void aci_ctx_destroy(aci_ctx* ctx);
const char* aci_last_error(const aci_ctx* ctx);

/* Waits of the LDU pivot exchange (Alg. 2's global argmax and pivot-row
 * broadcast between cooperating workgroups), for failure-handling tests and
 * long-running contexts.  Applies to LDU launches enqueued after the call
 * (graphs captured earlier keep their settings).
 *   spin_limit      polls before one wait gives up and the launch ends with
 *                   ACI_E_TIMEOUT; 0 restores the default 2^22.
 *   stall_step      -1: off.  s >= 0: from pivot step s on, readers wait for
 *                   a step flag that no workgroup publishes, so every LDU
 *                   launch that needs more than one workgroup gives up after
 *                   at most spin_limit polls per wait and its call returns
 *                   ACI_E_TIMEOUT.  All kernels still exit; the context stays
 *                   usable once the hook is switched off.
 *   epoch_launches  LDU launches after which a session clears its exchange
 *                   words and restarts its step flags (0: the default,
 *                   2^21 - 1, just before the 32-bit flags would wrap).
 * ACI_E_INVALID for stall_step < -1 or epoch_launches outside [0, 2^21 - 1]. */
int aci_ctx_set_exchange_hooks(aci_ctx* ctx, uint32_t spin_limit, int32_t stall_step, int64_t epoch_launches);

/* Row publication of LDU launches whose workgroups span several XCDs (the
 * pivot exchange of Alg. 2 for 1024-column rows: complex ones, and real ones
 * past one XCD's CUs).  Each workgroup publishes its pivot candidate; its
 * candidate's row goes out with it ("eagerly") only if the candidate's key
 * (|entry|, or |entry|^2 for complex) is at least eager_frac times the next
 * pivot key predicted from the last two (last key times the last ratio, at
 * most 1), and from the third step on; otherwise the winner publishes its
 * row once every group knows the winner.  A tuning and test hook: results do
 * not depend on it, only the time per pivot.  Launches whose workgroups share
 * one XCD always publish eagerly.  Applies to LDU launches enqueued after the
 * call.
 *   eager_frac  0: every row eagerly; +INFINITY: only the first two steps
 *               eagerly, every later winner late; default 0.6.
 * ACI_E_INVALID for a negative or NaN eager_frac. */
int aci_ctx_set_row_publication(aci_ctx* ctx, double eager_frac);

/* Alg. 1: approximate f(x^1..x^N) as a TT with error estimate <= tol and bond
 * dimensions <= maxrank.
 *   inputs     host array of n_inputs TTs (device cores, dtype as given)
 *   dtype      aci_dtype of the input cores and of the output
 *   out        device buffer receiving the output cores; out_capacity is its
 *              size in elements (double or double-complex).  A capacity of
 *              L * d_max * maxrank^2 always suffices.
 *   result     host struct filled on return; release with aci_result_free.
 * Returns ACI_OK, ACI_W_NOT_CONVERGED, or an error. */
int aci_elementwise(aci_ctx* ctx, const aci_tt* inputs, int32_t n_inputs, int32_t dtype,
                    int32_t op, double tol, int32_t maxrank, const aci_options* opt,
                    void* out, int64_t out_capacity, aci_result* result);
void aci_result_free(aci_result* result);

/* ---- single steps of the local update (section 2.4-2.6, Algs. 2-5) ------- *
 * These run exactly the kernels aci_elementwise uses, on caller data, for
 * step-by-step checks.  All matrices are device, row-major, dtype as given. */

/* Environment contractions (Eq. pifromframes, Alg. 5):
 *   side 0 (left):  A = Lf (c x r0) * X (r0 x d r1)        -> A (c x d r1)
 *   side 1 (right): B = X (r0 d x r1) * Rf (r1 x c)        -> B (r0 d x c)
 * Each of the `count` contractions uses its own pointers; dims are shared.
 * precision: aci_precision of the products (operands and result FP64). */
int aci_env_contract(aci_ctx* ctx, int32_t dtype, int32_t side, int32_t count,
                     const void* const* frames, const void* const* cores,
                     void* const* out, int32_t c, int32_t r0, int32_t d, int32_t r1,
                     int32_t precision);

/* Two-site tensor with f applied (Eq. pifromframes, Eq. localupdate):
 *   M = f(A^1 B^1, ..., A^N B^N),  A^n: m x k[n] (ld k[n]), B^n: k[n] x n (ld n),
 *   M: m x n with leading dimension ldm >= n.
 * precision: aci_precision of the products; f is applied in FP64.
 * tile: output tile per workgroup as in aci_tune_contract (0, 1, 2), or -1
 *   for the default of the shape; the tile never changes the result. */
int aci_pi_eval(aci_ctx* ctx, int32_t dtype, int32_t op, int32_t n_inputs,
                const void* const* A, const void* const* B, const int32_t* k,
                int32_t m, int32_t n, void* M, int32_t ldm, int32_t precision, int32_t tile);

/* LDU with full pivoting (Alg. 2) of the m x n matrix M (ld ldm).  The input
 * is not modified.  Outputs (device): rows[r], cols[r] = pivot row/column ids
 * in pivot order, *rank (int32), *eps (double).  If Y is not NULL it receives
 * the r x n matrix U_JJ^{-1} U (Alg. 3, right-interpolative factor), leading
 * dimension ldy. */
int aci_prrlu(aci_ctx* ctx, int32_t dtype, const void* M, int32_t m, int32_t n, int32_t ldm,
              double tol, int32_t maxrank, int32_t stop_rule,
              int32_t* rows, int32_t* cols, int32_t* rank, double* eps,
              void* Y, int32_t ldy);

/* The LDU of aci_prrlu for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, outputs, results and errors, but the exchange
 * and error words live in a fixed static device array of the library
 * (2.1 MB per GPU, held until the process ends) instead of memory the
 * context allocates; no hipMalloc, hipFree or other allocating call is made.
 * Limit: the factorisation's exchange must fit that array, which holds every
 * real matrix up to ACI_MAX_MATRIX x ACI_MAX_MATRIX and complex matrices of up
 * to 512 columns; larger ones return ACI_E_LIMIT.  The array is cleared at
 * the start of every call on the context's stream.  All calls on one GPU
 * share it: calls that overlap in time on one GPU (several streams, several
 * threads or contexts) race and must be serialised by the caller. */
int aci_prrlu_noalloc(aci_ctx* ctx, int32_t dtype, const void* M, int32_t m, int32_t n, int32_t ldm,
                      double tol, int32_t maxrank, int32_t stop_rule,
                      int32_t* rows, int32_t* cols, int32_t* rank, double* eps,
                      void* Y, int32_t ldy);

/* ---------------------------------------------------------------- batches
 * Several independent elementwise operations (for instance the convective
 * terms u_j d_j u_k of a Navier-Stokes right-hand side), each run as Alg. 1
 * with the same op, tol, maxrank and options, advanced sweep by sweep
 * together.  Product b has n_inputs[b] input TTs, taken in order from
 * `inputs` (products may differ in L, d and ranks).  Each product's
 * contractions and gathers run on a stream of its own, created by the batch
 * and ordered after the work enqueued on ctx's stream before
 * aci_batch_create.  options.batch_mode picks how the LDUs (Alg. 2) of the
 * products share the GPU:
 *   joint (default when possible): the products advance update by update
 *     together; after every product's two-site tensor of update u is ready,
 *     one launch factorises all of them, each product's cooperating
 *     workgroups on a single XCD (products dealt largest first to the least
 *     loaded XCD), then every product continues with its gathers.  Needs at
 *     most 12 products of one length L, no learned proposal, and LDUs that
 *     fit one XCD's CUs each.  With options.use_graph the whole joint sweep
 *     (all streams) is captured once into one hipGraph.
 *   overlapped: every product sweeps on its own stream; its LDU launches
 *     use exactly their P workgroups dealt over all XCDs, P capped at
 *     8 * floor(CUs per XCD / products) (or the autotuned value with
 *     options.tune) so that all of them fit at once.
 *   serial: one product after another with cooperative LDU launches (also
 *     the fallback of overlapped when some LDU cannot fit its share).
 * The batch owns all device memory it uses; input cores must stay valid
 * until aci_batch_destroy.  options.init must be NULL (every product starts
 * from the seeded default guess).  Errors name the product. */
typedef struct aci_batch aci_batch;
int aci_batch_create(aci_ctx* ctx, const aci_tt* inputs, const int32_t* n_inputs,
                     int32_t n_products, int32_t dtype, int32_t op, double tol,
                     int32_t maxrank, const aci_options* opt, aci_batch** batch);
/* Runs up to nsweeps sweeps of every product not yet converged (all of
 * them with options.fixed_sweeps); stats sums kernel times, launches, flops
 * and pivots over the products, max_eps is the largest over them, ranks are
 * product 0's.  Returns ACI_OK once every product has converged. */
int aci_batch_sweep(aci_batch* batch, int32_t nsweeps, aci_sweep_stats* stats);
/* Output of product `product`, as aci_session_result. */
int aci_batch_result(aci_batch* batch, int32_t product, void* out, int64_t out_capacity,
                     aci_result* result);
/* Placement of a product's LDUs: xcd = -2 in joint mode (XCD chosen per
 * launch by the placement, max_groups = 0), -1 in overlapped mode (groups
 * dealt over all XCDs, max_groups = the cap), 0 in serial mode. */
int aci_batch_info(aci_batch* batch, int32_t product, int32_t* xcd, int32_t* max_groups);
void aci_batch_destroy(aci_batch* batch);
/* create + sweeps (the last allowed sweep in FP64, as aci_elementwise) +
 * results + destroy.  outs[b] / out_capacity[b] / results[b] as in
 * aci_elementwise.  Returns the worst status over the products. */
int aci_elementwise_batched(aci_ctx* ctx, const aci_tt* inputs, const int32_t* n_inputs,
                            int32_t n_products, int32_t dtype, int32_t op, double tol,
                            int32_t maxrank, const aci_options* opt, void* const* outs,
                            const int64_t* out_capacity, aci_result* results);

/* ------------------------------------------------------------- 2-site TCI
 * Point evaluator of aci_tci: fills val_buf[p] = f(idx_buf[p L .. p L + L)) for
 * p < count (the buffers passed to aci_tci; digits int32, values of the
 * dtype), with work ordered on `stream` (the context's hipStream_t).  Called
 * from the host between the library's launches; returns 0 on success. */
typedef int32_t (*aci_eval_fn)(int64_t count, int32_t L, void* user, void* stream);

/* 2-site tensor cross interpolation of a function given point by point —
 * the construction of the input TTs (Sec. 3), whose index-set optimisation
 * ACI follows (Sec. 2.6): the sweeps of Alg. 1 with the two-site tensor
 * evaluated directly, Pi[(a, s), (s', b)] = f(I_{l-1}[a], s, s', J_{l+2}[b])
 * (row a d_l + s, column s' |J_{l+2}| + b), each factorised by the LDU of
 * Alg. 2 (right-interpolative), the index sets taking its pivot rows and
 * columns after every update.
 *   L, d        sites and local dimensions (host, L values)
 *   dtype       ACI_F64 or ACI_C128 values
 *   f, user     the evaluator (above)
 *   idx_buf     device, buf_points x L int32: the library writes the points
 *   val_buf     device, buf_points values of the dtype: f writes the values;
 *               buf_points >= (max_l d_l * maxrank)^2
 *   pivots      host, n_pivots x L digits seeding the index sets (distinct
 *               prefixes and suffixes); n_pivots = 0: the all-zero index
 *   options     maxiter, stop_rule, fixed_sweeps (others ignored; FP64 / C128
 *               throughout)
 *   out, result as aci_elementwise (ranks, eps, cores of the last
 *               right-to-left half, index sets; no trace).
 * The evaluator is called once per local update, with the device synchronised
 * once per update to size the next one.  ACI_E_INVALID if the evaluator
 * fails or a pivot digit is out of range; ACI_E_NUMERIC if it produced NaN. */
int aci_tci(aci_ctx* ctx, int32_t L, const int32_t* d, int32_t dtype, aci_eval_fn f, void* user,
            int32_t* idx_buf, void* val_buf, int64_t buf_points, const int32_t* pivots,
            int32_t n_pivots, double tol, int32_t maxrank, const aci_options* opt, void* out,
            int64_t out_capacity, aci_result* result);

/* ---- TT operators and an explicit time step --------------------------------
 * In TT solvers of nonlinear differential equations the contractions are with
 * TT operators (MPOs) of small, constant bond dimension, such as finite-
 * difference derivatives, and the elementwise nonlinearity is what ACI
 * evaluates (Sec. 4).  These calls provide both parts of an explicit step on
 * a periodic quantics grid. */

/* A TT operator with real cores in caller device memory: core l has shape
 * ranks[l] x d[l] x d[l] x ranks[l+1] (C order: left bond, output digit s,
 * input digit t, right bond); the operator maps x to
 * y[s_1..s_L] = sum_t W_1[s_1, t_1] ... W_L[s_L, t_L] x[t_1..t_L]. */
typedef struct {
  int32_t L;
  const int32_t* d;            /* host, L local dimensions */
  const int32_t* ranks;        /* host, L+1 bond ranks, ranks[0] = ranks[L] = 1 */
  const double* const* cores;  /* host array of L device pointers */
} aci_mpo;

/* The periodic three-point stencil sum_{delta = -1, 0, 1} w_delta S^delta
 * along `axis` of a box with 2^R points per axis in `ndim` dimensions, where
 * (S^delta psi)(x) = psi(x + delta h), as an MPO of L = R ndim sites, d = 2,
 * bond dimension 3 (1 at both ends).  Quantics order: site ndim b + a
 * (0-based) holds bit R-1-b of axis a, most significant bit first.  The
 * bonds carry the carry of adding delta, from the least significant bit to
 * the most significant one, where it is dropped (periodicity).
 *   weights  host, {w_-1, w_0, w_+1}
 *   cores    host, 36 L doubles: core l at cores + 36 l, ranks[l] x 2 x 2 x
 *            ranks[l+1] doubles in C order
 *   ranks    host, L+1 values
 * Host computation only; no context needed.  ACI_E_INVALID for R < 1,
 * ndim < 1, axis outside [0, ndim) or a NULL pointer; ACI_E_LIMIT if
 * R ndim > ACI_MAX_SITES. */
int aci_mpo_stencil(int32_t R, int32_t ndim, int32_t axis, const double* weights, double* cores,
                    int32_t* ranks);

/* Exact MPO-TT contraction y = W x.  Core l of y has shape
 * (w_{l-1} r_{l-1}) x d_l x (w_l r_l) with bond index a r + c (MPO bond a,
 * TT bond c) and entries sum_t W_l[a, s, t, b] x_l[c, t, e]; for complex x
 * the real operator acts on real and imaginary parts alike.
 *   x        TT of the dtype (ACI_F64 or ACI_C128), device cores
 *   out      host array of L device pointers, core l with room for its
 *            (w_{l-1} r_{l-1}) d_l (w_l r_l) elements of the dtype; must not
 *            overlap x or the operator
 *   kernel_ms optional (NULL): device time of the launches, from HIP events
 *            on the context stream
 * ACI_E_INVALID on a length or local-dimension mismatch or a NULL pointer;
 * ACI_E_LIMIT if an output core exceeds 2^31 - 1 doubles. */
int aci_mpo_apply(aci_ctx* ctx, const aci_mpo* W, const aci_tt* x, int32_t dtype, void* const* out,
                  float* kernel_ms);

/* One explicit step of a cubic nonlinear equation,
 *   y = c0 psi + c_lap sum_a D_a psi + c3 |psi|^2 psi,
 * with D_a the periodic second difference (psi(x+h) - 2 psi(x) + psi(x-h)) /
 * h^2 along axis a of the box [0,1)^ndim with 2^R points per axis (R = L /
 * ndim, h = 2^-R, every d_l = 2, quantics order of aci_mpo_stencil).  The
 * time step is folded into coef = {c0, c_lap, c3}: 3 doubles for ACI_F64, 3
 * (re, im) pairs for ACI_C128 (Gross-Pitaevskii i psi_t = -1/2 Lap psi +
 * g |psi|^2 psi: c0 = 1, c_lap = i dt / 2, c3 = -i g dt).  The D_a psi are
 * formed exactly by aci_mpo_apply (bond ranks 3 r); then ACI evaluates
 * LINEAR_CUBIC of (psi, D_1 psi, ..., D_ndim psi) with coefficients
 * {c0, c_lap, ..., c_lap, c3}, started from Y_init = psi (the warm start)
 * unless options.init is set; options.coef is ignored.  ndim <=
 * ACI_MAX_INPUTS - 1; the ranks 3 r of D_a psi must stay <=
 * ACI_MAX_INPUT_RANK.
 * The operators and the D_a psi take temporary device memory from the
 * context's allocator, released before the return.  out, out_capacity,
 * result and the return value as aci_elementwise. */
int aci_cubic_step(aci_ctx* ctx, const aci_tt* psi, int32_t dtype, int32_t ndim, const double* coef,
                   double tol, int32_t maxrank, const aci_options* opt, void* out, int64_t out_capacity,
                   aci_result* result);

/* ---- patched ACI --------------------------------------------------------
 * f(x^1..x^N) as tensor trains on patches of the index space (the patched
 * elementwise scheme named in Sec. 4).  A patch is a prefix of k fixed
 * leading indices (sigma_1..sigma_k); its tensor, f restricted to them, is a
 * TT over sites k+1..L.  The inputs are restricted exactly on the device:
 * the prefix vector X_1[:, sigma_1, :] ... X_k[:, sigma_k, :] is absorbed
 * into the first free core.  Breadth first from the empty prefix, every
 * patch of a level runs ACI (Alg. 1; one batch per level, as
 * aci_elementwise_batched, with the same tol, maxrank and options, hence the
 * same seeded default Y_init); a patch whose sweeps converged is kept, the
 * others split into their d children, down to max_depth fixed indices, where
 * patches are kept whatever their state.  Patches are listed level by level,
 * prefixes in lexicographic order within a level. */
typedef struct {
  int32_t n_patches;
  int32_t L;
  int32_t levels;         /* levels run (1 + deepest prefix length) */
  int32_t* prefix_len;    /* host, n_patches: k */
  uint8_t* prefix;        /* host, n_patches x L digits; the first k used */
  int32_t* ranks;         /* host, n_patches x (L+1): bond ranks of the patch
                             TT over its L-k sites (first L-k+1 used) */
  int64_t* core_offset;   /* host, n_patches x L: element offsets of its
                             cores in `cores` (first L-k used); core j has
                             shape ranks[j] x d_{k+j} x ranks[j+1] */
  int32_t* converged;     /* host, n_patches */
  int32_t* sweeps;        /* host, n_patches */
  double* max_eps;        /* host, n_patches: largest error estimate */
  void* cores;            /* device, from the context's allocator: all cores */
  int64_t cores_elems;    /* elements of the dtype in `cores` */
} aci_patched_result;

/* Patched ACI of the inputs (as aci_elementwise) down to max_depth fixed
 * indices, 0 <= max_depth <= L - 2 (max_depth 0: one patch, the unpatched
 * ACI).  result is filled on return; release it with aci_patched_free on the
 * same context.  Returns ACI_OK if every kept patch converged, else
 * ACI_W_NOT_CONVERGED (patches at max_depth that did not converge), or an
 * error; ACI_E_INVALID if options.init is set (every patch starts from the
 * seeded default Y_init). */
int aci_patched(aci_ctx* ctx, const aci_tt* inputs, int32_t n_inputs, int32_t dtype, int32_t op,
                double tol, int32_t maxrank, int32_t max_depth, const aci_options* opt,
                aci_patched_result* result);
void aci_patched_free(aci_ctx* ctx, aci_patched_result* result);

/* Autotuner of the contraction tile shape (environment and two-site
 * products of Eq. pifromframes): times ngroup (1..ACI_MAX_INPUTS) side-by-side
 * copies of an m x k by k x n product (dtype, precision; operands seeded
 * uniform on [-1, 1), one term, elements of the dtype) with each output tile
 * per workgroup — 0: 64 x 64, 1: 32 x 64, 2: 32 x 32 (real-view elements) —
 * one untimed and three timed launches each, and returns the fastest in
 * *best_tile; us (optional, 3 floats) gets the mean microseconds per launch
 * of each tile.  The choice is cached in the context per shape.  Sessions
 * and batches created with options.tune pick the tile of every contraction
 * launch of their sweeps this way; otherwise the largest tile that still
 * gives every CU a workgroup is used.  Every output element is accumulated
 * in the same order whatever the tile, so the choice never changes a
 * result. */
int aci_tune_contract(aci_ctx* ctx, int32_t dtype, int32_t precision, int32_t ngroup, int32_t m,
                      int32_t k, int32_t n, int32_t* best_tile, float* us);

/* Autotuner of the LDU launch shape (Alg. 2 kernel): times the LDU of a
 * seeded random m x n matrix (entries uniform on [-1, 1)) to rank
 * min(maxrank, m, n) for group-count caps cap, cap/2, cap/4, ... (each
 * distinct launch shape once; cap <= 0 selects one XCD's CUs), three runs
 * each with the first discarded, and returns the fastest cap in
 * *best_groups.  The choice is cached in the context per (m, n, maxrank,
 * cap).  If candidates / us are given, up to `capacity` tried caps and
 * their mean times (microseconds) are written and *count gets the number
 * tried. */
int aci_tune_prrlu(aci_ctx* ctx, int32_t m, int32_t n, int32_t maxrank, int32_t cap,
                   int32_t* best_groups, int32_t* candidates, float* us, int32_t capacity,
                   int32_t* count);

/* ------------------------------------------------------- learned proposal
 * An extension of the method (not in the paper): a small network scores the
 * rows of the two-site matrix, a rook search seeded by the scores proposes
 * pivots, and the proposal is accepted only if the dense residual
 * max |M - L Up| is within tol; otherwise the full search of Alg. 2 decides.
 * All pointers are device pointers; every call returns after its work is
 * done.  Definitions (features, rounding, search order) are those of the
 * CPU reference in the test suite and are repeated at each call.
 *
 * Row features, X (m x 7 float32, row-major): f0, f1 = row 2-norm of the
 * left environment env[t] (m x env_w[t], leading dim env_ld[t]) over the
 * largest row norm (0 if absent or all zero); f2 = 1 for the n_prev rows in
 * prev_rows (pivot rows of the previous update of the same bond); f3..f6 =
 * |M[i, c_t]| / max over the four columns c_t = floor((2t + 1) n / 8). */
int aci_proposal_features(aci_ctx* ctx, const void* M, int32_t m, int32_t n, int32_t ldm,
                          const void* const* env, const int32_t* env_w, const int32_t* env_ld,
                          int32_t n_env, const int32_t* prev_rows, int32_t n_prev, float* X);
/* Training set of the scoring network from the library's own plain FP64
 * sweeps: runs Alg. 1 on real inputs (options as for aci_elementwise, at most
 * options.maxiter sweeps, stopping at convergence unless fixed_sweeps;
 * options.proposal must be NULL and precision FP64) and, after the LDU of
 * Alg. 2 of every local update of every sweep (left to right, then right to
 * left), appends that update's m rows of the two-site matrix M: their
 * features (as aci_proposal_features, with env = the update's left
 * environments A^n for the first two inputs and prev_rows = the pivot rows
 * of the previous update of the same bond and direction, none in the first
 * sweep) to X (capacity x 7 float32, device) and their labels to y (capacity
 * float32, device): 1 for the first max(1, r / 2) pivot rows of the update's
 * rank-r factorisation, else 0.  *count (host) receives the rows written,
 * *sweeps (host, optional) the sweeps run.  An update whose rows would pass
 * `capacity` is not recorded, nor is any later one; the call then returns
 * ACI_E_NOMEM with *count the rows of the updates that fit.  Otherwise
 * returns ACI_OK or ACI_W_NOT_CONVERGED as aci_elementwise would. */
int aci_proposal_dataset(aci_ctx* ctx, const aci_tt* inputs, int32_t n_inputs, int32_t op, double tol,
                         int32_t maxrank, const aci_options* options, float* X, float* y,
                         int64_t capacity, int64_t* count, int32_t* sweeps);
/* Initial parameters of the scoring network (device, ACI_MLP_PARAMS float32,
 * layout as below): W1, W2 and w3 in this order, each in C order, from one
 * SplitMix64 stream seeded with `seed` (S. Vigna's generator, as for the
 * default Y_init): entry = u sqrt(6 / fan_in) rounded to float32, with
 * u = (z >> 11) 2^-53 2 - 1 uniform on [-1, 1) and fan_in 7, 64, 64; all
 * biases zero. */
int aci_mlp_init(aci_ctx* ctx, uint64_t seed, float* params);
/* Network 7 -> 64 -> 64 -> 1 (ReLU), parameters: ACI_MLP_PARAMS float32 in
 * the order W1 (7 x 64, row-major), b1, W2 (64 x 64), b2, w3, b3.  Each
 * layer rounds inputs and weights to float16, accumulates the exact products
 * in float32 in index order and adds the float32 bias.  scores: count
 * logits for X (count x 7). */
int aci_mlp_forward(aci_ctx* ctx, const float* params, const float* X, int32_t count, float* scores);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias corrections for
 * step >= 1) on the mean binary cross entropy of logits vs labels y (0/1),
 * count <= ACI_MAX_MLP_BATCH samples, in one workgroup with gradients summed
 * in sample order.  params, adam_m, adam_v (ACI_MLP_PARAMS each) are
 * updated in place; grads (optional, device) receives the gradient; *loss
 * (optional, host) the mean loss before the step. */
int aci_mlp_train_step(aci_ctx* ctx, float* params, float* adam_m, float* adam_v, int32_t step,
                       const float* X, const float* y, int32_t count, float lr, float* grads,
                       float* loss);
/* Rook search with lazy residuals on M (m x n, ldm), at most maxrank pivots,
 * each step started at the best-scored free row (scores may be NULL: the
 * smallest free row) and at most max_iter row/column scan pairs long; stop
 * rule as the exclusive rule of Alg. 2.  Out (device): rows, cols (maxrank
 * each), *rank, *eps (|pivot| that stopped the search, 0 if exhausted), L
 * (m x maxrank, ldl >= maxrank: residual columns over the pivot), Up
 * (maxrank x n, ldu >= n: residual rows), *scans (optional). */
int aci_rook_lu(aci_ctx* ctx, const void* M, int32_t m, int32_t n, int32_t ldm, double tol,
                int32_t maxrank, const float* scores, int32_t max_iter, int32_t* rows,
                int32_t* cols, int32_t* rank, double* eps, void* L, int32_t ldl, void* Up,
                int32_t ldu, int32_t* scans);
/* Acceptance test: *eps = max |M - L Up| (FP64 matrix-core product), and
 * *accepted = (*eps <= tol); rank read from the device. */
int aci_rook_check(aci_ctx* ctx, const void* M, int32_t m, int32_t n, int32_t ldm, const void* L,
                   int32_t ldl, const void* Up, int32_t ldu, const int32_t* rank, double tol,
                   double* eps, int32_t* accepted);
/* Right factor of an accepted search (Alg. 3, right-interpolative form):
 * Y = T^{-1} Up with T = Up[:, cols] upper triangular, by back substitution
 * (Y[:, cols] = identity).  Y: rank x n, leading dim ldy. */
int aci_rook_right_factor(aci_ctx* ctx, const void* Up, int32_t ldu, const int32_t* cols,
                          const int32_t* rank, int32_t n, void* Y, int32_t ldy);

/* Frame update by gathering (Alg. 5, truncation step).  src is h x w with
 * leading dimension ld_src; idx (device) holds r indices, r read from the
 * device int *rank:
 *   side 0: out[k][c] = src[idx[k]][c]   (r x w result, leading dim ld_out)
 *   side 1: out[i][k] = src[i][idx[k]]   (h x r result, leading dim ld_out) */
int aci_gather(aci_ctx* ctx, int32_t dtype, int32_t side, const void* src, int32_t h,
               int32_t w, int32_t ld_src, const int32_t* idx, const int32_t* rank, void* out,
               int32_t ld_out);

#ifdef __cplusplus
}
#endif

#endif /* ACI_H */
