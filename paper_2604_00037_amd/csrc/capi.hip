// C ABI and sweep driver of the ACI library (Alg. 1 of the paper).
//
// The host enqueues a whole sweep without waiting: every kernel reads the
// ranks it depends on (|I_l|, |J_l|) from a small device array that the prrLU
// kernels write, and every grid is sized for the largest shape the bond can
// take.  The host synchronises once per sweep, to read the right-to-left
// ranks and error estimates for the convergence test.
//
// Environment caching: left frames change only in left-to-right half sweeps
// and right frames only in right-to-left ones, so A^n_l = L^n_{l-1} X^n_l
// computed going right is reused going left, and B^n_l = X^n_{l+1} R^n_{l+2}
// computed going left (or during initialisation) is reused going right.  Each
// local update therefore runs one fresh environment contraction.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "kernels.h"

using namespace aci;

struct aci_ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  std::string err;
  uint32_t flag_next = 1;
  bool step_flags_wrapped = false;   // flag_next wrapped since step_xbuf was cleared
  // exchange waits of the LDU launches enqueued from now on (see
  // aci_ctx_set_exchange_hooks): spin limit, and the test stall
  uint32_t spin_limit = 1u << 22;
  uint32_t poll_xor = 0;
  int stall_from = 0;
  uint64_t epoch_launches = 0;   // session epoch reset period (0: the default)
  // LDUs across XCDs: eager row publication above this fraction of the
  // predicted pivot key (aci_ctx_set_row_publication; 0.6 measured best on
  // the complex 1024 x 1024 two-site matrices)
  double eager_frac = 0.6;
  // small persistent workspace of the single-step entry points
  int* step_err = nullptr;     // [0] error flags, [1] abort word
  uint64_t* step_xbuf = nullptr;
  size_t step_xwords = 0;
  std::map<uint64_t, int> tuned;   // autotuned LDU group caps by shape
  std::map<uint64_t, int> tuned_tiles;   // autotuned contraction tiles by shape
  float* mlp_scratch = nullptr;    // training scratch of the scoring network
  size_t mlp_scratch_n = 0;
  double* check_c = nullptr;       // L Up of the residual check
  size_t check_c_n = 0;
  // optional caller allocator for the library's device memory
  void* (*alloc_fn)(size_t, void*) = nullptr;
  void (*free_fn)(void*, void*) = nullptr;
  void* alloc_user = nullptr;
};

static int ensure_step_ws(aci_ctx* ctx);

// Device memory for the library's own buffers: the caller's allocator when
// the context has one, else hipMalloc.  Memory given back to a caller
// allocator may be reused at once, so every stream that used it has been
// synchronised before dev_free is called.
static bool dev_alloc(aci_ctx* ctx, void** p, size_t bytes) {
  *p = nullptr;
  if (ctx->alloc_fn) {
    *p = ctx->alloc_fn(bytes, ctx->alloc_user);
    return *p != nullptr;
  }
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return false;
  }
  return true;
}
static void dev_free(aci_ctx* ctx, void* p) {
  if (!p) return;
  if (ctx->free_fn)
    ctx->free_fn(p, ctx->alloc_user);
  else
    (void)hipFree(p);
}

namespace {

constexpr uint32_t kSpinLimit = 1u << 22;   // polls before an exchange gives up (default)
// Noise floors of the precision ladder's low-precision sweeps, relative to
// the largest entry of the two-site matrix: 32 units of FP32 rounding, and
// 4 x 2^-15 for BF16x3 (operands split to about 16 significant bits).
constexpr double kNoiseFP32 = 32.0 * 0x1.0p-24;
constexpr double kNoiseBF16X3 = 4.0 * 0x1.0p-15;

// The exchange-wait settings of the context on an LDU launch.
void exchange_waits(const aci_ctx* c, PrrluArgs& a) {
  a.spin_limit = c->spin_limit;
  a.poll_xor = c->poll_xor;
  a.stall_from = c->stall_from;
  a.eager_frac = c->eager_frac;
}

int set_err(aci_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return set_err(ctx, ACI_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

uint32_t next_flag(aci_ctx* c) {
  // each prrLU launch uses flags base .. base + min(m, n) <= base + 1024
  uint32_t f = c->flag_next;
  c->flag_next += 2048u;
  if (c->flag_next < 2048u) {
    // wrapped: words of the step exchange buffer may carry flags that the
    // next launches reuse, so the buffer is cleared before the next launch
    c->flag_next = 1;
    c->step_flags_wrapped = true;
  }
  return f;
}

// Flag base of an LDU launch on the step exchange buffer; after a wrap of
// the flags the buffer is cleared first, on the context's stream.
hipError_t step_flag(aci_ctx* c, uint32_t* f) {
  *f = next_flag(c);
  if (c->step_flags_wrapped) {
    const hipError_t e = launch_fill_int((int*)c->step_xbuf, (int)(2 * c->step_xwords), 0, c->stream);
    if (e != hipSuccess) return e;
    c->step_flags_wrapped = false;
  }
  return hipSuccess;
}

// ---- bump allocator: pass 0 sizes the workspace, pass 1 hands out pointers
struct Arena {
  char* base = nullptr;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

int sat_mul(int a, int b, int cap) {
  long long v = (long long)a * b;
  return v > cap ? cap : (int)v;
}

// SplitMix64 (S. Vigna): default Y_init entries, uniform on [-1, 1).
struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * 0x1.0p-53 * 2.0 - 1.0; }
};

struct Plan {
  int L = 0, N = 0, op = 0, maxrank = 0, maxiter = 20, rule = 0;
  aci_pointwise_fn pointwise = nullptr;   // f of ACI_OP_CUSTOM
  void* pointwise_user = nullptr;
  double coef[2 * (ACI_MAX_INPUTS + 1)] = {};   // ACI_OP_LINEAR_CUBIC: b, a_1..a_N (re, im)
  double* Pibuf[ACI_MAX_INPUTS] = {};      // the N two-site tensors it reads
  int cplx = 0, ew = 1;       // complex entries; doubles per entry
  int prec_req = PREC_FP64;   // requested contraction precision
  int prec = PREC_FP64;       // precision of the sweep being enqueued
  int low_max = 4;            // ladder: most low-precision sweeps (< 0: no limit)
  int sketch = 0;             // size of the random index sketch that starts the sweeps (0: off)
  bool trace = false, fixed = false;
  // placement of the LDU launches (batches): XCD, group cap, launch kind
  int xcd = 0, max_groups = 0, cooperative = 1;
  uint32_t* epoch = nullptr;  // device word: flag base of the next LDU launch
  uint64_t ldu_launches = 0;  // LDU launches enqueued since epoch and xbuf were reset
  // learned proposal (options.proposal): network, scan limit and buffers
  const float* mlp = nullptr;
  int rook_iter = 8;
  float *feat = nullptr, *scores = nullptr;
  double *rkL = nullptr, *rkUp = nullptr, *rkC = nullptr, *rkeps = nullptr, *chkeps = nullptr;
  int *rkrows = nullptr, *rkcols = nullptr, *rkrank = nullptr, *acc = nullptr, *rkscans = nullptr;
  int* acc_count = nullptr;   // per sweep: [0] accepted proposals, [1] rook scans, [2] rook pivots
  int *prevr = nullptr, *prevk = nullptr;   // previous pivot rows per (direction, bond)
  // training set of the scoring network recorded from the sweeps
  // (aci_proposal_dataset): features and pivot labels of every local update
  bool rec_on = false;
  float *recX = nullptr, *recY = nullptr;
  int64_t rec_cap = 0;
  long long* rec_count = nullptr;   // [0] rows, [1] overflow
  double tol = 0.0;
  int d[ACI_MAX_SITES + 1];                         // d[l], l = 1..L
  int r[ACI_MAX_INPUTS][ACI_MAX_SITES + 1];         // r[n][l], l = 0..L
  const double* X[ACI_MAX_INPUTS][ACI_MAX_SITES + 1];  // X[n][l], l = 1..L
  int rho[ACI_MAX_SITES + 1];                       // Y_init ranks
  const double* Yin[ACI_MAX_SITES + 1];             // Y_init cores (device)
  int capI[ACI_MAX_SITES + 2], capJ[ACI_MAX_SITES + 2];
  // contraction tile per bond: [0] left environment, [1] right environment,
  // [2] two-site tensor (-1: the default for the shape; set by the tuner)
  int tiles[3][ACI_MAX_SITES + 2];
  int D = 1;          // max local dimension
  int ldm = 0;        // leading dimension of the two-site matrix
  int ldR = 0;        // leading dimension of right frames
  int n_rec = 0;
  // device buffers
  double* Lf[ACI_MAX_INPUTS][ACI_MAX_SITES + 1];
  double* Rf[ACI_MAX_INPUTS][ACI_MAX_SITES + 2];
  double* Ac[ACI_MAX_INPUTS][ACI_MAX_SITES + 1];
  double* Bc[ACI_MAX_INPUTS][ACI_MAX_SITES + 1];
  double* Mbuf = nullptr;
  double* G[ACI_MAX_SITES + 1];
  double* Gin[ACI_MAX_SITES + 1];
  double* Atmp = nullptr;
  double* Ycore[ACI_MAX_SITES + 1];
  int* nI = nullptr;   // |I_l|, l = 0..L
  int* nJ = nullptr;   // |J_l|, l = 1..L+1
  int* prow = nullptr;
  int* pcol = nullptr;
  // pivots of the last sweep per bond (the nested index sets): rows of the
  // left-to-right update, rows and columns of the right-to-left update
  int* pivLR = nullptr;
  int* pivRLr = nullptr;
  int* pivRLc = nullptr;
  int* cprank = nullptr;   // rank slot written by the copies of traced pivots
  int* prank = nullptr;
  double* peps = nullptr;
  double* eps_bond = nullptr;
  int* flags = nullptr;  // [0] error flags, [1] abort word
  uint64_t* xbuf = nullptr;
  size_t xbuf_words = 0;
  int* tr_meta = nullptr;
  double* tr_eps = nullptr;
  int* tr_rows = nullptr;
  int* tr_cols = nullptr;
  int* meta = nullptr;   // {rank, m, n} of the init calls, then of the current sweep
};

void layout(Plan& p, Arena& A, bool gen_init) {
  const int L = p.L;
  for (int n = 0; n < p.N; ++n) {
    for (int l = 0; l < L; ++l) p.Lf[n][l] = A.take<double>((size_t)p.ew * p.capI[l] * p.r[n][l]);
    for (int l = 2; l <= L + 1; ++l) p.Rf[n][l] = A.take<double>((size_t)p.ew * p.r[n][l - 1] * p.ldR);
    for (int l = 1; l < L; ++l) {
      p.Ac[n][l] = A.take<double>((size_t)p.ew * p.capI[l - 1] * p.d[l] * p.r[n][l]);
      p.Bc[n][l] = A.take<double>((size_t)p.ew * p.r[n][l] * p.d[l + 1] * p.capJ[l + 2]);
    }
  }
  p.Mbuf = A.take<double>((size_t)p.ew * p.ldm * p.ldm);
  if (p.op == ACI_OP_CUSTOM)
    for (int n = 0; n < p.N; ++n) p.Pibuf[n] = A.take<double>((size_t)p.ew * p.ldm * p.ldm);
  int rho_max = 1;
  for (int l = 0; l <= L; ++l) rho_max = std::max(rho_max, p.rho[l]);
  for (int l = 1; l <= L; ++l) {
    p.G[l] = A.take<double>((size_t)p.ew * p.rho[l - 1] * p.d[l] * p.rho[l]);
    p.Gin[l] = gen_init ? A.take<double>((size_t)p.ew * p.rho[l - 1] * p.d[l] * p.rho[l]) : nullptr;
    p.Ycore[l] = A.take<double>((size_t)p.ew * p.maxrank * p.d[l] * p.maxrank);
  }
  p.Atmp = A.take<double>((size_t)p.ew * rho_max * p.ldR);
  p.nI = A.take<int>(L + 2);
  p.nJ = A.take<int>(L + 3);
  p.prow = A.take<int>(p.maxrank + 1);
  p.pcol = A.take<int>(p.maxrank + 1);
  p.pivLR = A.take<int>((size_t)(L + 1) * p.maxrank);
  p.pivRLr = A.take<int>((size_t)(L + 1) * p.maxrank);
  p.pivRLc = A.take<int>((size_t)(L + 1) * p.maxrank);
  p.cprank = A.take<int>(4);
  p.prank = A.take<int>(4);
  p.peps = A.take<double>(4);
  p.eps_bond = A.take<double>(L + 1);
  p.flags = A.take<int>(4);
  p.epoch = A.take<uint32_t>(1);
  p.xbuf_words = prrlu_xbuf_words(p.ldm, p.ldm, p.cplx);
  p.xbuf = A.take<uint64_t>(p.xbuf_words);
  p.meta = A.take<int>((size_t)3 * 3 * (L - 1));
  if (p.mlp || p.rec_on) {
    p.feat = A.take<float>((size_t)p.D * p.maxrank * MLP_FEATURES);
    p.prevr = A.take<int>((size_t)2 * (L + 1) * p.maxrank);
    p.prevk = A.take<int>((size_t)2 * (L + 1));
  }
  if (p.rec_on) p.rec_count = A.take<long long>(2);
  if (p.mlp) {
    const size_t rows = (size_t)p.D * p.maxrank;
    p.scores = A.take<float>(rows);
    p.rkL = A.take<double>(rows * p.maxrank);
    p.rkUp = A.take<double>((size_t)p.maxrank * p.ldm);
    p.rkC = A.take<double>(rows * p.ldm);
    p.rkeps = A.take<double>(1);
    p.chkeps = A.take<double>(1);
    p.rkrows = A.take<int>(p.maxrank);
    p.rkcols = A.take<int>(p.maxrank);
    p.rkrank = A.take<int>(1);
    p.acc = A.take<int>(2);
    p.acc_count = A.take<int>(3);
    p.rkscans = A.take<int>(1);
  }
  if (p.trace) {
    p.tr_meta = A.take<int>((size_t)3 * p.n_rec);
    p.tr_eps = A.take<double>(p.n_rec);
    p.tr_rows = A.take<int>((size_t)p.n_rec * p.maxrank);
    p.tr_cols = A.take<int>((size_t)p.n_rec * p.maxrank);
  }
}

// Session LDUs take their step flags from a device epoch that every launch
// advances by kFlagStride; after 2^32 / kFlagStride launches the flags would
// wrap and reuse values that words written long before may still carry.
// Before that, the exchange words are cleared and the epoch restarts at 1.
constexpr uint64_t kEpochLaunches = (1ull << 32) / kFlagStride - 1;
int epoch_guard(aci_ctx* ctx, Plan& p, int launches, hipStream_t s) {
  const uint64_t limit = ctx->epoch_launches ? ctx->epoch_launches : kEpochLaunches;
  if (p.ldu_launches + (uint64_t)launches > limit) {
    HIPCHK(launch_fill_int((int*)p.xbuf, (int)(2 * p.xbuf_words), 0, s));
    HIPCHK(launch_fill_int((int*)p.epoch, 1, 1, s));
    p.ldu_launches = 0;
  }
  p.ldu_launches += (uint64_t)launches;
  return ACI_OK;
}

// Launch-log instance code of a contraction (see aci_launch).
int contract_variant(int op, int prec, int cplx, int tile) { return 10000 * tile + 1000 * cplx + 100 * prec + op + 1; }

// Kernel classes of the profile (see aci_sweep_stats).
enum { CLS_PRRLU = 0, CLS_CONTRACT = 1, CLS_GATHER = 2, NCLS = 3 };

struct Prof {
  bool on = false;
  std::vector<hipEvent_t> pool;
  // per event pair i (events 2i, 2i+1): class, instance, part, meta slot
  std::vector<int> cls, variant, part, slot;
  size_t used = 0;
  void clear() {
    used = 0;
    cls.clear();
    variant.clear();
    part.clear();
    slot.clear();
  }
};

struct Enq {
  aci_ctx* ctx;
  Plan& p;
  hipStream_t s;
  int rec = 0;          // prrLU calls so far (trace record index)
  int slot = 0;         // meta slot: init calls 0..L-2, sweep calls L-1 ..
  Prof* prof = nullptr;
  bool sweeping = false;  // enqueuing the local updates of a sweep (not the initialisation)
  // deferred LDU: prrlu() only records its arguments (a batch launches the
  // LDUs of all its products together)
  bool defer = false;
  bool has_pend = false;
  // where the LDU of the current sweep update puts its pivots (untraced):
  // the per-bond index-set arrays; null: the scratch rows / columns
  int* rows_to = nullptr;
  int* cols_to = nullptr;
  PrrluArgs pend{};
  int pend_mmax = 0, pend_nmax = 0;

  int begin(int c, int variant = 0, int part = 0) {
    if (!prof || !prof->on) return ACI_OK;
    if (prof->used + 2 > prof->pool.size()) {
      for (int i = 0; i < 64; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return set_err(ctx, ACI_E_HIP, "hipEventCreate");
        prof->pool.push_back(e);
      }
    }
    prof->cls.push_back(c);
    prof->variant.push_back(variant);
    prof->part.push_back(part);
    prof->slot.push_back(slot);
    if (hipEventRecord(prof->pool[prof->used], s) != hipSuccess) return set_err(ctx, ACI_E_HIP, "hipEventRecord");
    return ACI_OK;
  }
  int end() {
    if (!prof || !prof->on) return ACI_OK;
    if (hipEventRecord(prof->pool[prof->used + 1], s) != hipSuccess) return set_err(ctx, ACI_E_HIP, "hipEventRecord");
    prof->used += 2;
    return ACI_OK;
  }
  bool tracing() const { return p.trace && rec < p.n_rec; }

  int prrlu(const double* M, Dim m, Dim n, Dim ldm, int mmax, int nmax, int* rank2, double* eps2,
            double* Y, Dim ldy, const int* skip = nullptr) {
    PrrluArgs a{};
    a.skip = skip;
    a.cplx = p.cplx;
    a.M = M;
    a.m = m;
    a.n = n;
    a.ldm = ldm;
    a.tol = p.tol;
    // low-precision sweeps of the ladder stop at the contraction's noise
    // floor instead of factorising its rounding errors
    a.tol_rel = !sweeping ? 0.0 : (p.prec == PREC_FP32 ? kNoiseFP32 : (p.prec == PREC_BF16X3 ? kNoiseBF16X3 : 0.0));
    a.maxrank = p.maxrank;
    a.rule = p.rule;
    a.flag_base = 0;
    a.epoch = p.epoch;
    a.xcd = p.xcd;
    a.max_groups = p.max_groups;
    a.cooperative = p.cooperative;
    exchange_waits(ctx, a);
    a.xbuf = p.xbuf;
    a.xbuf_words = p.xbuf_words;
    if (tracing()) {
      a.rows = p.tr_rows + (size_t)rec * p.maxrank;
      a.cols = p.tr_cols + (size_t)rec * p.maxrank;
      a.eps = p.tr_eps + rec;
    } else {
      a.rows = rows_to ? rows_to : p.prow;
      a.cols = cols_to ? cols_to : p.pcol;
      a.eps = p.peps;
    }
    a.meta = p.meta + (size_t)3 * slot;
    a.meta2 = tracing() ? p.tr_meta + (size_t)3 * rec : nullptr;
    a.rank = p.prank;
    a.rank2 = rank2;
    a.eps2 = eps2;
    a.Y = Y;
    a.ldy = ldy;
    a.err = p.flags;
    a.abort_word = p.flags + 1;
    if (defer) {
      pend = a;
      pend_mmax = mmax;
      pend_nmax = nmax;
      has_pend = true;
      return ACI_OK;
    }
    int rc = begin(CLS_PRRLU, prrlu_variant(mmax, nmax, p.max_groups, p.cplx));
    if (rc) return rc;
    hipError_t e = launch_prrlu(a, mmax, nmax, s);
    if (e != hipSuccess) return set_err(ctx, ACI_E_HIP, std::string("prrlu launch: ") + hipGetErrorString(e));
    return end();
  }
  // Learned proposal for the two-site matrix in p.Mbuf at bond l (dir 0
  // left to right, 1 right to left): features, scores, seeded rook search,
  // dense residual check, and on acceptance the pivots, rank and error in
  // the places the LDU would write them.  p.acc[0] then tells the LDU to
  // skip, p.acc[1] the right-factor solve.
  int propose(int l, int dir, Dim m, Dim n, int mrows, int ncols_max, int* rank2, double* eps2) {
    if (int rc = features(l, dir, m, n)) return rc;
    if (int rc = stepf(20002, [&] { return launch_mlp_forward(p.mlp, p.feat, mrows, p.scores, s); })) return rc;
    return rook(m, n, mrows, ncols_max, rank2, eps2);
  }
  // row features of the two-site matrix in p.Mbuf at bond l into p.feat
  int features(int l, int dir, Dim m, Dim n) {
    FeatureArgs fa{};
    fa.M = p.Mbuf;
    fa.m = m;
    fa.n = n;
    fa.ldm = dconst(p.ldm);
    fa.n_env = p.N < 2 ? p.N : 2;
    for (int t = 0; t < fa.n_env; ++t) {
      fa.env[t] = p.Ac[t][l];
      fa.env_w[t] = dconst(p.r[t][l]);
      fa.env_ld[t] = dconst(p.r[t][l]);
    }
    fa.prev_rows = p.prevr + (size_t)(dir * (p.L + 1) + l) * p.maxrank;
    fa.prev_rank = p.prevk + dir * (p.L + 1) + l;
    fa.X = p.feat;
    return stepf(20001, [&] { return launch_features(fa, s); });
  }
  // seeded rook search, residual check and commit of an accepted proposal
  int rook(Dim m, Dim n, int mrows, int ncols_max, int* rank2, double* eps2) {
    RookArgs ra{};
    ra.M = p.Mbuf;
    ra.m = m;
    ra.n = n;
    ra.ldm = dconst(p.ldm);
    ra.tol = p.tol;
    ra.maxrank = p.maxrank;
    ra.max_iter = p.rook_iter;
    ra.scores = p.scores;
    ra.L = p.rkL;
    ra.ldl = p.maxrank;
    ra.Up = p.rkUp;
    ra.ldu = p.ldm;
    ra.rows = p.rkrows;
    ra.cols = p.rkcols;
    ra.rank = p.rkrank;
    ra.eps = p.rkeps;
    ra.scans = p.rkscans;
    if (int rc = stepf(20003, [&] { return launch_rook(ra, s); })) return rc;
    ContractArgs c{};
    c.ngroup = 1;
    Group& g = c.g[0];
    g.nterm = 1;
    g.t[0] = Term{p.rkL, p.rkUp, Dim{p.rkrank, 1, 0}, dconst(p.maxrank), dconst(p.ldm)};
    g.C = p.rkC;
    g.M = m;
    g.N = n;
    g.ldc = dconst(p.ldm);
    if (int rc = stepf(20004, [&] { return launch_contract(OP_NONE, PREC_FP64, c, mrows, ncols_max, s); })) return rc;
    CheckArgs ca{};
    ca.M = p.Mbuf;
    ca.m = m;
    ca.n = n;
    ca.ldm = dconst(p.ldm);
    ca.C = p.rkC;
    ca.ldc = p.ldm;
    ca.tol = p.tol;
    ca.eps = p.chkeps;
    ca.accepted = p.acc;
    ca.count = p.acc_count;
    if (int rc = stepf(20005, [&] { return launch_check(ca, s); })) return rc;
    CommitArgs cm{};
    cm.accepted = p.acc;
    cm.src_rows = p.rkrows;
    cm.src_cols = p.rkcols;
    cm.src_rank = p.rkrank;
    cm.src_eps = p.chkeps;
    cm.rows = const_cast<int*>(rows());
    cm.cols = const_cast<int*>(cols());
    cm.rank = p.prank;
    cm.rank2 = rank2;
    cm.eps = tracing() ? p.tr_eps + rec : p.peps;
    cm.eps2 = eps2;
    cm.meta = p.meta + (size_t)3 * slot;
    cm.meta2 = tracing() ? p.tr_meta + (size_t)3 * rec : nullptr;
    cm.m = m;
    cm.n = n;
    cm.maxrank = p.maxrank;
    cm.src_scans = p.rkscans;
    cm.scan_total = p.acc_count + 1;
    return stepf(20006, [&] { return launch_commit(cm, s); });
  }
  // the update's training rows (features of M, labels from the LDU's
  // pivots), appended to the recorded dataset
  int record(int l, int dir, Dim m, Dim n) {
    if (int rc = features(l, dir, m, n)) return rc;
    RecordArgs a{};
    a.feat = p.feat;
    a.m = m;
    a.rows = rows();
    a.rank = p.prank;
    a.X = p.recX;
    a.y = p.recY;
    a.capacity = p.rec_cap;
    a.count = p.rec_count;
    return stepf(20009, [&] { return launch_record(a, s); });
  }
  // keep this update's pivot rows for the next update of the same bond
  int keep_rows(int l, int dir) {
    CopyRowsArgs a{};
    a.src = rows();
    a.rank = p.prank;
    a.dst = p.prevr + (size_t)(dir * (p.L + 1) + l) * p.maxrank;
    a.dst_rank = p.prevk + dir * (p.L + 1) + l;
    a.maxrank = p.maxrank;
    return stepf(20007, [&] { return launch_copy_rows(a, s); });
  }
  // a profiled launch of the proposal pipeline (class prrLU, instance code)
  template <typename F>
  int stepf(int variant, F&& launch) {
    int rc = begin(CLS_PRRLU, variant);
    if (rc) return rc;
    const hipError_t e = launch();
    if (e != hipSuccess) return set_err(ctx, ACI_E_HIP, std::string("proposal launch: ") + hipGetErrorString(e));
    return end();
  }
  // pointers the prrLU of the current record wrote its pivots to
  const int* rows() const {
    return tracing() ? p.tr_rows + (size_t)rec * p.maxrank : (rows_to ? rows_to : p.prow);
  }
  const int* cols() const {
    return tracing() ? p.tr_cols + (size_t)rec * p.maxrank : (cols_to ? cols_to : p.pcol);
  }
  // traced pivots also go to the per-bond index-set arrays
  int copy_traced(const int* src, int* dst) {
    if (!tracing() || !dst) return ACI_OK;
    CopyRowsArgs a{};
    a.src = src;
    a.rank = p.prank;
    a.dst = dst;
    a.dst_rank = p.cprank;
    a.maxrank = p.maxrank;
    const hipError_t e = launch_copy_rows(a, s);
    if (e != hipSuccess) return set_err(ctx, ACI_E_HIP, std::string("pivot copy: ") + hipGetErrorString(e));
    return ACI_OK;
  }
  void next_record() {
    ++rec;
    ++slot;
    rows_to = cols_to = nullptr;
  }
};

#define ENQ(call)                                                                   \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      return set_err(ctx, ACI_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// a profiled launch of class `cls` (instance `var`, part `part` of the update)
#define ENQPV(q, cls, var, part, call)       \
  do {                                       \
    int rc_ = (q).begin(cls, var, part);     \
    if (rc_) return rc_;                     \
    ENQ(call);                               \
    rc_ = (q).end();                         \
    if (rc_) return rc_;                     \
  } while (0)
#define ENQP(q, cls, call) ENQPV(q, cls, 0, 0, call)
// a profiled contraction launch with tile `tile` (-1: the default for the shape)
#define ENQC(q, part, op, prec, c, mmax, nmax, tile)                                                   \
  do {                                                                                                 \
    const int t_ = (tile) >= 0 ? (tile) : contract_default_tile((mmax), (nmax), (c).ngroup, (q).p.cplx); \
    ENQPV(q, CLS_CONTRACT, contract_variant(op, prec, (q).p.cplx, t_), part,                          \
          launch_contract(op, prec, c, mmax, nmax, (q).s, t_));                                       \
  } while (0)

// Initialisation (Alg. 1, first two loops): CI-canonical form of Y_init from
// right to left, initial right frames R^n_l and the cached B^n_{l-1}.
int enqueue_init(Enq& q) {
  aci_ctx* ctx = q.ctx;
  Plan& p = q.p;
  hipStream_t s = q.s;
  const int L = p.L;
  for (int n = 0; n < p.N; ++n) {
    // the boundary frames are [1] (complex: 1 + 0i)
    ENQ(launch_fill(p.Lf[n][0], p.ew, 0.0, s));
    ENQ(launch_fill(p.Rf[n][L + 1], p.ew, 0.0, s));
    ENQ(launch_fill(p.Lf[n][0], 1, 1.0, s));
    ENQ(launch_fill(p.Rf[n][L + 1], 1, 1.0, s));
  }
  ENQ(launch_fill_int(p.nI, 1, 1, s));
  ENQ(launch_fill_int(p.nJ + L + 1, 1, 1, s));
  ENQ(launch_fill_int(p.flags, 4, 0, s));
  ENQ(launch_fill_int((int*)p.epoch, 1, 1, s));
  if (p.mlp || p.rec_on) ENQ(launch_fill_int(p.prevk, 2 * (L + 1), 0, s));
  if (p.rec_on) ENQ(launch_fill_int((int*)p.rec_count, 4, 0, s));
  // the LDU exchange words: flag 0 is never used, and the session's flags
  // restart at 1, so memory left by an earlier session must not look valid
  ENQ(launch_fill_int((int*)p.xbuf, 2 * p.xbuf_words, 0, s));
  p.ldu_launches = L - 1;
  for (int l = L; l >= 2; --l) {
    const int dl = p.d[l];
    const double* Msrc = (l == L) ? p.Yin[L] : p.G[l];
    const Dim ncols = ddev(p.nJ + l + 1, dl);
    // cross interpolation of the core matricised as rho_{l-1} x (d |J_{l+1}|)
    int rc = q.prrlu(Msrc, dconst(p.rho[l - 1]), ncols, ncols, p.rho[l - 1], dl * p.capJ[l + 1],
                     p.nJ + l, nullptr, nullptr, dconst(0));
    if (rc) return rc;
    const int* cols = q.cols();
    if (l > 2) {
      // G_{l-1} = Y_init_{l-1} * M[:, J_l]
      GatherArgs g{};
    g.esz = p.ew;
      g.count = 1;
      g.side = 1;
      g.idx = cols;
      g.rank = p.nJ + l;
      g.err = p.flags;
      g.it[0] = GatherItem{Msrc, p.Atmp, ncols, dconst(p.ldR), dconst(p.rho[l - 1]), ncols};
      ENQP(q, CLS_GATHER, launch_gather(g, p.maxrank, p.rho[l - 1], s));
      ContractArgs c{};
    c.cplx = p.cplx;
      c.ngroup = 1;
      c.err = nullptr;
      Group& gr = c.g[0];
      gr.nterm = 1;
      gr.t[0] = Term{p.Yin[l - 1], p.Atmp, dconst(p.rho[l - 1]), dconst(p.rho[l - 1]), dconst(p.ldR)};
      gr.C = p.G[l - 1];
      gr.M = dconst(p.rho[l - 2] * p.d[l - 1]);
      gr.N = ddev(p.nJ + l);
      gr.ldc = ddev(p.nJ + l);
      ENQC(q, 1, OP_NONE, PREC_FP64, c, p.rho[l - 2] * p.d[l - 1], p.maxrank, -1);
    }
    // B^n_{l-1} = X^n_l R^n_{l+1};  R^n_l = B^n_{l-1}[:, J_l]  (Alg. 5, Rightframe)
    ContractArgs c{};
    c.cplx = p.cplx;
    c.ngroup = p.N;
    int mmax = 0;
    for (int n = 0; n < p.N; ++n) {
      Group& gr = c.g[n];
      gr.nterm = 1;
      gr.t[0] = Term{p.X[n][l], p.Rf[n][l + 1], dconst(p.r[n][l]), dconst(p.r[n][l]), dconst(p.ldR)};
      gr.C = p.Bc[n][l - 1];
      gr.M = dconst(p.r[n][l - 1] * dl);
      gr.N = ddev(p.nJ + l + 1);
      gr.ldc = ddev(p.nJ + l + 1);
      mmax = std::max(mmax, p.r[n][l - 1] * dl);
    }
    ENQC(q, 1, OP_NONE, PREC_FP64, c, mmax, p.capJ[l + 1], -1);
    GatherArgs g{};
    g.esz = p.ew;
    g.count = p.N;
    g.side = 1;
    g.idx = cols;
    g.rank = p.nJ + l;
    g.err = p.flags;
    int emax = 0;
    for (int n = 0; n < p.N; ++n) {
      g.it[n] = GatherItem{p.Bc[n][l - 1], p.Rf[n][l], ncols, dconst(p.ldR), dconst(p.r[n][l - 1]), ncols};
      emax = std::max(emax, p.r[n][l - 1]);
    }
    ENQP(q, CLS_GATHER, launch_gather(g, p.capJ[l], emax, s));
    q.next_record();
  }
  return ACI_OK;
}

// Two-site tensor of bond l with f applied (Eq. pifromframes, localupdate).
int enqueue_pi(Enq& q, int l) {
  aci_ctx* ctx = q.ctx;
  Plan& p = q.p;
  ContractArgs c{};
  c.cplx = p.cplx;
  c.err = p.flags;
  const int mmax = p.d[l] * p.capI[l - 1], nmax = p.d[l + 1] * p.capJ[l + 2];
  if (p.op == ACI_OP_CUSTOM) {
    // the N two-site tensors side by side, then the caller's f into M
    c.ngroup = p.N;
    for (int n = 0; n < p.N; ++n) {
      Group& gr = c.g[n];
      gr.nterm = 1;
      gr.t[0] = Term{p.Ac[n][l], p.Bc[n][l], dconst(p.r[n][l]), dconst(p.r[n][l]), ddev(p.nJ + l + 2, p.d[l + 1])};
      gr.C = p.Pibuf[n];
      gr.M = ddev(p.nI + l - 1, p.d[l]);
      gr.N = ddev(p.nJ + l + 2, p.d[l + 1]);
      gr.ldc = dconst(p.ldm);
    }
    ENQC(q, 2, OP_NONE, p.prec, c, mmax, nmax, p.tiles[2][l]);
    void* pis[ACI_MAX_INPUTS];
    for (int n = 0; n < p.N; ++n) pis[n] = p.Pibuf[n];
    if (p.pointwise(pis, p.N, p.Mbuf, mmax, nmax, p.ldm, p.pointwise_user, (void*)q.s) != 0)
      return set_err(ctx, ACI_E_INVALID, "the pointwise f failed");
    return ACI_OK;
  }
  c.ngroup = 1;
  std::memcpy(c.coef, p.coef, sizeof c.coef);
  Group& gr = c.g[0];
  gr.nterm = p.N;
  for (int n = 0; n < p.N; ++n)
    gr.t[n] = Term{p.Ac[n][l], p.Bc[n][l], dconst(p.r[n][l]), dconst(p.r[n][l]),
                   ddev(p.nJ + l + 2, p.d[l + 1])};
  gr.C = p.Mbuf;
  gr.M = ddev(p.nI + l - 1, p.d[l]);
  gr.N = ddev(p.nJ + l + 2, p.d[l + 1]);
  gr.ldc = dconst(p.ldm);
  ENQC(q, 2, p.op, p.prec, c, mmax, nmax, p.tiles[2][l]);
  return ACI_OK;
}

// Local update u of a sweep (u < L-1: left to right at bond u+1, otherwise
// right to left at bond 2(L-1)-u).  Stage 0 enqueues the environment and
// two-site contractions, the proposal and the LDU (only recorded when q.defer);
// stage 1 what depends on the LDU's pivots.
int enqueue_update(Enq& q, int u, int stage) {
  aci_ctx* ctx = q.ctx;
  Plan& p = q.p;
  hipStream_t s = q.s;
  const int L = p.L;
  if (u < L - 1) {
    // ---- left to right
    const int l = u + 1;
    q.rows_to = p.pivLR + (size_t)l * p.maxrank;
    q.cols_to = nullptr;
    if (stage == 0) {
      ContractArgs c{};
      c.cplx = p.cplx;
      c.ngroup = p.N;
      int nmax = 0;
      for (int n = 0; n < p.N; ++n) {
        Group& gr = c.g[n];
        gr.nterm = 1;
        const int w = p.d[l] * p.r[n][l];
        gr.t[0] = Term{p.Lf[n][l - 1], p.X[n][l], dconst(p.r[n][l - 1]), dconst(p.r[n][l - 1]), dconst(w)};
        gr.C = p.Ac[n][l];
        gr.M = ddev(p.nI + l - 1);
        gr.N = dconst(w);
        gr.ldc = dconst(w);
        nmax = std::max(nmax, w);
      }
      ENQC(q, 1, OP_NONE, p.prec, c, p.capI[l - 1], nmax, p.tiles[0][l]);
      int rc = enqueue_pi(q, l);
      if (rc) return rc;
      const int mmax = p.d[l] * p.capI[l - 1], nmax2 = p.d[l + 1] * p.capJ[l + 2];
      const int* skip = nullptr;
      if (p.mlp) {
        rc = q.propose(l, 0, ddev(p.nI + l - 1, p.d[l]), ddev(p.nJ + l + 2, p.d[l + 1]), mmax, nmax2, p.nI + l,
                       nullptr);
        if (rc) return rc;
        skip = p.acc;
      }
      return q.prrlu(p.Mbuf, ddev(p.nI + l - 1, p.d[l]), ddev(p.nJ + l + 2, p.d[l + 1]), dconst(p.ldm),
                     mmax, nmax2, p.nI + l, nullptr, nullptr, dconst(0), skip);
    }
    int rc = q.copy_traced(q.rows(), p.pivLR + (size_t)l * p.maxrank);
    if (rc) return rc;
    if (p.rec_on && (rc = q.record(l, 0, ddev(p.nI + l - 1, p.d[l]), ddev(p.nJ + l + 2, p.d[l + 1])))) return rc;
    if ((p.mlp || p.rec_on) && (rc = q.keep_rows(l, 0))) return rc;
    // L^n_l = A^n_l[I_l, :]  (Alg. 5, Leftframe)
    GatherArgs g{};
    g.esz = p.ew;
    g.count = p.N;
    g.side = 0;
    g.idx = q.rows();
    g.rank = p.nI + l;
    g.err = p.flags;
    int emax = 0;
    for (int n = 0; n < p.N; ++n) {
      g.it[n] = GatherItem{p.Ac[n][l], p.Lf[n][l], dconst(p.r[n][l]), dconst(p.r[n][l]), dconst(p.r[n][l]),
                           ddev(p.nI + l - 1, p.d[l])};
      emax = std::max(emax, p.r[n][l]);
    }
    ENQP(q, CLS_GATHER, launch_gather(g, p.capI[l], emax, s));
    q.next_record();
    return ACI_OK;
  }
  // ---- right to left
  const int l = 2 * (L - 1) - u;
  const Dim ncols = ddev(p.nJ + l + 2, p.d[l + 1]);
  q.rows_to = p.pivRLr + (size_t)l * p.maxrank;
  q.cols_to = p.pivRLc + (size_t)l * p.maxrank;
  if (stage == 0) {
    ContractArgs c{};
    c.cplx = p.cplx;
    c.ngroup = p.N;
    int mmax = 0;
    for (int n = 0; n < p.N; ++n) {
      Group& gr = c.g[n];
      gr.nterm = 1;
      gr.t[0] = Term{p.X[n][l + 1], p.Rf[n][l + 2], dconst(p.r[n][l + 1]), dconst(p.r[n][l + 1]), dconst(p.ldR)};
      gr.C = p.Bc[n][l];
      gr.M = dconst(p.r[n][l] * p.d[l + 1]);
      gr.N = ddev(p.nJ + l + 2);
      gr.ldc = ddev(p.nJ + l + 2);
      mmax = std::max(mmax, p.r[n][l] * p.d[l + 1]);
    }
    ENQC(q, 1, OP_NONE, p.prec, c, mmax, p.capJ[l + 2], p.tiles[1][l]);
    int rc = enqueue_pi(q, l);
    if (rc) return rc;
    const int* skip = nullptr;
    if (p.mlp) {
      rc = q.propose(l, 1, ddev(p.nI + l - 1, p.d[l]), ncols, p.d[l] * p.capI[l - 1], p.d[l + 1] * p.capJ[l + 2],
                     p.nJ + l + 1, p.eps_bond + (l - 1));
      if (rc) return rc;
      skip = p.acc;
    }
    return q.prrlu(p.Mbuf, ddev(p.nI + l - 1, p.d[l]), ncols, dconst(p.ldm), p.d[l] * p.capI[l - 1],
                   p.d[l + 1] * p.capJ[l + 2], p.nJ + l + 1, p.eps_bond + (l - 1), p.Ycore[l + 1], ncols, skip);
  }
  int rc = q.copy_traced(q.rows(), p.pivRLr + (size_t)l * p.maxrank);
  if (rc) return rc;
  if ((rc = q.copy_traced(q.cols(), p.pivRLc + (size_t)l * p.maxrank))) return rc;
  if (p.mlp) {
    // an accepted proposal's right factor (the LDU forms it otherwise)
    SolveArgs sa{};
    sa.Up = p.rkUp;
    sa.ldu = p.ldm;
    sa.cols = p.rkcols;
    sa.rank = p.rkrank;
    sa.n = ncols;
    sa.Y = p.Ycore[l + 1];
    sa.ldy = ncols;
    sa.skip = p.acc + 1;
    rc = q.stepf(20008, [&] { return launch_rook_solve(sa, s); });
    if (rc) return rc;
  }
  if (p.rec_on && (rc = q.record(l, 1, ddev(p.nI + l - 1, p.d[l]), ncols))) return rc;
  if ((p.mlp || p.rec_on) && (rc = q.keep_rows(l, 1))) return rc;
  // R^n_{l+1} = B^n_l[:, J_{l+1}]  (Alg. 5, Rightframe)
  GatherArgs g{};
  g.esz = p.ew;
  g.count = p.N;
  g.side = 1;
  g.idx = q.cols();
  g.rank = p.nJ + l + 1;
  g.err = p.flags;
  int emax = 0;
  for (int n = 0; n < p.N; ++n) {
    g.it[n] = GatherItem{p.Bc[n][l], p.Rf[n][l + 1], ncols, dconst(p.ldR), dconst(p.r[n][l]), ncols};
    emax = std::max(emax, p.r[n][l]);
  }
  if (l == 1) {
    // Y_1 = M[:, J_2] (the left factor of the last update, Alg. 3)
    g.it[p.N] = GatherItem{p.Mbuf, p.Ycore[1], dconst(p.ldm), ddev(p.nJ + 2), dconst(p.d[1]), ncols};
    g.count = p.N + 1;
    emax = std::max(emax, p.d[1]);
  }
  ENQP(q, CLS_GATHER, launch_gather(g, p.capJ[l + 1], emax, s));
  q.next_record();
  return ACI_OK;
}

// One sweep of Alg. 1: 2(L-1) local updates, left to right then right to left.
int enqueue_sweep(Enq& q) {
  aci_ctx* ctx = q.ctx;
  Plan& p = q.p;
  q.slot = p.L - 1;
  q.sweeping = true;
  if (p.mlp) ENQ(launch_fill_int(p.acc_count, 3, 0, q.s));
  for (int u = 0; u < 2 * (p.L - 1); ++u)
    for (int stage = 0; stage < 2; ++stage)
      if (int rc = enqueue_update(q, u, stage)) return rc;
  return ACI_OK;
}

int validate_tt(aci_ctx* ctx, const aci_tt& t, int L) {
  if (t.L != L || !t.d || !t.ranks || !t.cores) return set_err(ctx, ACI_E_INVALID, "TT description incomplete or L mismatch");
  if (t.ranks[0] != 1 || t.ranks[L] != 1) return set_err(ctx, ACI_E_INVALID, "boundary ranks must be 1");
  for (int l = 0; l < L; ++l) {
    if (t.d[l] < 1 || t.d[l] > ACI_MAX_DIM) return set_err(ctx, ACI_E_LIMIT, "local dimension out of range");
    if (t.ranks[l + 1] < 1) return set_err(ctx, ACI_E_INVALID, "ranks must be >= 1");
    if (!t.cores[l]) return set_err(ctx, ACI_E_INVALID, "null core pointer");
  }
  return ACI_OK;
}

}  // namespace

// =============================================================== sessions
struct aci_session {
  aci_ctx* ctx = nullptr;
  std::unique_ptr<Plan> plan;
  void* ws = nullptr;
  int rec = 0;
  int sweeps = 0;
  bool converged = false;
  bool fixed = false;
  int low_done = 0;              // low-precision sweeps run so far
  bool use_graph = false;        // replay each sweep from a captured hipGraph
  hipStream_t cap_stream = nullptr;   // private stream the sweep is captured on
  hipGraphExec_t gexec = nullptr;
  int gprec = -1;                // precision the graph was captured with
  int swept_prec = 0;            // precision of the sweep in flight
  // pinned read-back of one sweep: ranks, eps, meta, flags
  void* hbuf = nullptr;
  int* h_cur = nullptr;
  double* h_eps = nullptr;
  int* h_meta = nullptr;
  int* h_flags = nullptr;
  std::vector<int> prev;
  int init_ranks[ACI_MAX_SITES + 1];
  Prof prof;
  std::vector<aci_launch> log;   // launches of the last aci_session_sweep call
  double sweep_ms = 0.0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
};

namespace {

// Entries of per-bond host arrays (with room for 2(L-1) updates' meta).
int L_pad(int L) { return 2 * L + 2; }

// Validation and static sizes shared by aci_elementwise and the sessions.
int plan_problem(aci_ctx* ctx, const aci_tt* inputs, int32_t n_inputs, int32_t dtype, int32_t op, double tol,
                 int32_t maxrank, const aci_options& o, Plan& p) {
  if (!inputs) return set_err(ctx, ACI_E_INVALID, "null inputs");
  if (n_inputs < 1 || n_inputs > ACI_MAX_INPUTS) return set_err(ctx, ACI_E_LIMIT, "n_inputs out of range");
  if (dtype != ACI_F64 && dtype != ACI_C128) return set_err(ctx, ACI_E_DTYPE, "unknown dtype");
  if (op != ACI_OP_PRODUCT && op != ACI_OP_SUM && op != ACI_OP_ABS2_MUL && op != ACI_OP_CUSTOM &&
      op != ACI_OP_LINEAR_CUBIC)
    return set_err(ctx, ACI_E_INVALID, "unknown op");
  if ((op == ACI_OP_CUSTOM) != (o.pointwise != nullptr))
    return set_err(ctx, ACI_E_INVALID, "ACI_OP_CUSTOM goes with options.pointwise (and only it)");
  if (op == ACI_OP_LINEAR_CUBIC) {
    if (!o.coef) return set_err(ctx, ACI_E_INVALID, "ACI_OP_LINEAR_CUBIC needs options.coef");
    const bool cx = dtype == ACI_C128;
    for (int t = 0; t <= n_inputs; ++t) {
      // API order a_1..a_N, b; kernel order b, a_1..a_N
      const int k = t < n_inputs ? t + 1 : 0;
      p.coef[2 * k] = o.coef[cx ? 2 * t : t];
      p.coef[2 * k + 1] = cx ? o.coef[2 * t + 1] : 0.0;
      if (!std::isfinite(p.coef[2 * k]) || !std::isfinite(p.coef[2 * k + 1]))
        return set_err(ctx, ACI_E_INVALID, "non-finite coefficient");
    }
  }
  if (op == ACI_OP_ABS2_MUL && n_inputs != 1) return set_err(ctx, ACI_E_INVALID, "ABS2_MUL takes one input");
  if (!(tol >= 0.0)) return set_err(ctx, ACI_E_INVALID, "tol must be >= 0");
  if (maxrank < 1) return set_err(ctx, ACI_E_INVALID, "maxrank must be >= 1");
  if (maxrank > ACI_MAX_RANK) return set_err(ctx, ACI_E_LIMIT, "maxrank above ACI_MAX_RANK");
  if (o.precision != ACI_PREC_FP64 && o.precision != ACI_PREC_FP32 && o.precision != ACI_PREC_BF16X3)
    return set_err(ctx, ACI_E_DTYPE, "unknown precision");
  if (o.stop_rule != 0 && o.stop_rule != 1) return set_err(ctx, ACI_E_INVALID, "stop_rule must be 0 or 1");
  if (o.sketch_rank < 0) return set_err(ctx, ACI_E_INVALID, "sketch_rank must be >= 0");
  const int L = inputs[0].L;
  if (L < 2 || L > ACI_MAX_SITES) return set_err(ctx, ACI_E_LIMIT, "L out of range");
  p.L = L;
  p.N = n_inputs;
  p.op = op;
  p.pointwise = o.pointwise;
  p.pointwise_user = o.pointwise_user;
  p.tol = tol;
  p.maxrank = maxrank;
  p.maxiter = o.maxiter;
  p.rule = o.stop_rule;
  p.trace = o.trace != 0;
  p.fixed = o.fixed_sweeps != 0;
  p.prec_req = o.precision;
  p.cplx = dtype == ACI_C128 ? 1 : 0;
  p.ew = p.cplx ? 2 : 1;
  p.mlp = o.proposal;
  if (p.mlp && p.cplx) return set_err(ctx, ACI_E_DTYPE, "the learned proposal takes real matrices only");
  p.rook_iter = o.proposal_scans > 0 ? o.proposal_scans : 8;
  p.prec = o.precision;
  p.low_max = o.low_precision_sweeps == 0 ? 4 : o.low_precision_sweeps;
  for (int n = 0; n < n_inputs; ++n) {
    int rc = validate_tt(ctx, inputs[n], L);
    if (rc) return rc;
    for (int l = 0; l < L; ++l)
      if (inputs[n].d[l] != inputs[0].d[l]) return set_err(ctx, ACI_E_INVALID, "inputs differ in local dimensions");
    for (int l = 0; l <= L; ++l) {
      p.r[n][l] = inputs[n].ranks[l];
      if (p.r[n][l] > ACI_MAX_INPUT_RANK) return set_err(ctx, ACI_E_LIMIT, "input rank above ACI_MAX_INPUT_RANK");
    }
    for (int l = 1; l <= L; ++l) p.X[n][l] = (const double*)inputs[n].cores[l - 1];
  }
  p.D = 1;
  for (int l = 1; l <= L; ++l) {
    p.d[l] = inputs[0].d[l - 1];
    p.D = std::max(p.D, p.d[l]);
  }
  p.d[0] = 1;
  if ((long long)p.D * maxrank > ACI_MAX_MATRIX) return set_err(ctx, ACI_E_LIMIT, "d * maxrank above ACI_MAX_MATRIX");
  p.capI[0] = 1;
  for (int l = 1; l <= L; ++l) p.capI[l] = sat_mul(p.capI[l - 1], p.d[l], maxrank);
  p.capJ[L + 1] = 1;
  for (int l = L; l >= 1; --l) p.capJ[l] = sat_mul(p.capJ[l + 1], p.d[l], maxrank);
  p.ldm = p.D * maxrank;
  p.ldR = maxrank;
  if (o.init) {
    int rc = validate_tt(ctx, *o.init, L);
    if (rc) return rc;
    for (int l = 0; l < L; ++l)
      if (o.init->d[l] != p.d[l + 1]) return set_err(ctx, ACI_E_INVALID, "init local dimensions differ");
    for (int l = 0; l <= L; ++l) {
      p.rho[l] = o.init->ranks[l];
      if (p.rho[l] > ACI_MAX_MATRIX) return set_err(ctx, ACI_E_LIMIT, "init rank above limit");
    }
  } else if (o.sketch_rank > 0) {
    // random index sketch: rho_l = min(k, maxrank, index points left and right of bond l)
    p.sketch = o.sketch_rank;
    p.rho[0] = p.rho[L] = 1;
    for (int l = 1; l < L; ++l) p.rho[l] = std::min(std::min(o.sketch_rank, maxrank), std::min(p.capI[l], p.capJ[l + 1]));
  } else {
    p.rho[0] = p.rho[L] = 1;
    for (int l = 1; l < L; ++l) {
      int mn = maxrank;
      for (int n = 0; n < n_inputs; ++n) mn = std::min(mn, p.r[n][l]);
      p.rho[l] = mn;
    }
  }
  p.n_rec = (L - 1) * (1 + 2 * p.maxiter);
  return ACI_OK;
}

// Algorithmic flops of one prrLU record and of the contractions of its update.
// Algorithmic flops of one part of a local update (kind 1 left-to-right, 2
// right-to-left, at bond `bond`, with prrLU rank r on an m x n matrix):
// part 0 the LDU (plus the pivot-matrix solve right to left), 1 the fresh
// environment product, 2 the two-site tensors.
double update_flops(const Plan& p, int kind, int bond, int r, int m, int n, int part) {
  // complex entries: a complex multiply-add is 8 real flops, 4x the real count
  const double cx = p.cplx ? 4.0 : 1.0;
  double f = 0.0;
  if (part == 0) {
    for (int k = 0; k < r; ++k) f += 2.0 * (double)(m - k - 1) * (double)(n - k - 1);
    if (kind == 2 && n > r) f += (double)r * (r - 1) * (double)(n - r);
    return cx * f;
  }
  const int l = bond;
  const double cL = (double)m / p.d[l], cR = (double)n / p.d[l + 1];
  for (int q = 0; q < p.N; ++q) {
    if (part == 1)
      f += kind == 1 ? 2.0 * cL * p.r[q][l - 1] * p.d[l] * p.r[q][l]
                     : 2.0 * p.r[q][l] * p.d[l + 1] * p.r[q][l + 1] * cR;
    else
      f += 2.0 * (double)m * p.r[q][l] * (double)n;
  }
  return cx * f;
}

void account(const Plan& p, int kind, int bond, int r, int m, int n, aci_sweep_stats& st) {
  st.flops[CLS_PRRLU] += update_flops(p, kind, bond, r, m, n, 0);
  st.pivots += r;
  st.flops[CLS_CONTRACT] += update_flops(p, kind, bond, r, m, n, 1) + update_flops(p, kind, bond, r, m, n, 2);
}

// kind and bond of local update u of a sweep
void update_of(int L, int u, int& kind, int& bond) {
  kind = u < L - 1 ? 1 : 2;
  bond = u < L - 1 ? u + 1 : 2 * (L - 1) - u;
}

}  // namespace

// =============================================================== C ABI
extern "C" {

int aci_ctx_create(aci_ctx** out, void* stream) {
  if (!out) return ACI_E_INVALID;
  *out = nullptr;
  aci_ctx* ctx = new (std::nothrow) aci_ctx();
  if (!ctx) return ACI_E_NOMEM;
  ctx->stream = (hipStream_t)stream;
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    delete ctx;
    return ACI_E_HIP;
  }
  *out = ctx;
  return ACI_OK;
}

int aci_ctx_create_with_allocator(aci_ctx** out, void* stream, void* (*alloc)(size_t bytes, void* user),
                                  void (*release)(void* ptr, void* user), void* user) {
  if (!out || !alloc || !release) return ACI_E_INVALID;
  const int rc = aci_ctx_create(out, stream);
  if (rc) return rc;
  (*out)->alloc_fn = alloc;
  (*out)->free_fn = release;
  (*out)->alloc_user = user;
  return ACI_OK;
}

void aci_ctx_destroy(aci_ctx* ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  dev_free(ctx, ctx->mlp_scratch);
  dev_free(ctx, ctx->check_c);
  dev_free(ctx, ctx->step_err);
  dev_free(ctx, ctx->step_xbuf);
  delete ctx;
}

const char* aci_last_error(const aci_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int aci_ctx_set_exchange_hooks(aci_ctx* ctx, uint32_t spin_limit, int32_t stall_step, int64_t epoch_launches) {
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  if (stall_step < -1 || epoch_launches < 0 || (uint64_t)epoch_launches > kEpochLaunches)
    return set_err(ctx, ACI_E_INVALID, "stall_step < -1 or epoch_launches out of range");
  ctx->spin_limit = spin_limit ? spin_limit : kSpinLimit;
  ctx->poll_xor = stall_step >= 0 ? 0x80000000u : 0u;
  ctx->stall_from = stall_step >= 0 ? stall_step : 0;
  ctx->epoch_launches = (uint64_t)epoch_launches;
  return ACI_OK;
}

int aci_ctx_set_row_publication(aci_ctx* ctx, double eager_frac) {
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  if (!(eager_frac >= 0.0)) return set_err(ctx, ACI_E_INVALID, "eager_frac must be >= 0 (or +inf)");
  ctx->eager_frac = eager_frac;
  return ACI_OK;
}

void aci_result_free(aci_result* r) {
  if (!r) return;
  free(r->rec_meta);
  free(r->rec_eps);
  free(r->rec_rows);
  free(r->rec_cols);
  free(r->I_idx);
  free(r->J_idx);
  r->I_idx = nullptr;
  r->J_idx = nullptr;
  r->rec_meta = nullptr;
  r->rec_eps = nullptr;
  r->rec_rows = nullptr;
  r->rec_cols = nullptr;
  r->n_records = 0;
}

int aci_session_launches(aci_session* S, aci_launch* out, int32_t capacity, int32_t* count) {
  if (!S || !count || capacity < 0) return ACI_E_INVALID;
  *count = (int32_t)S->log.size();
  if (out)
    for (int32_t i = 0; i < capacity && i < *count; ++i) out[i] = S->log[i];
  return ACI_OK;
}

void aci_session_destroy(aci_session* S) {
  if (!S) return;
  if (S->ctx) (void)hipStreamSynchronize(S->ctx->stream);
  if (S->gexec) (void)hipGraphExecDestroy(S->gexec);
  if (S->cap_stream) (void)hipStreamDestroy(S->cap_stream);
  if (S->hbuf) (void)hipHostFree(S->hbuf);
  if (S->ws && S->ctx) dev_free(S->ctx, S->ws);
  for (hipEvent_t e : S->prof.pool) (void)hipEventDestroy(e);
  if (S->e0) (void)hipEventDestroy(S->e0);
  if (S->e1) (void)hipEventDestroy(S->e1);
  delete S;
}

namespace {
// Contraction tile autotuner: times ngroup copies of an m x k by k x n
// product (seeded uniform operands, complex when cplx, one term) with every
// output tile and keeps the fastest, cached per context.  us (optional):
// mean time per launch of each tile.
int tune_tile(aci_ctx* ctx, int cplx, int prec, int ngroup, int m, int k, int n, int* best, float* us) {
  if (m < 1 || k < 1 || n < 1 || m > ACI_MAX_MATRIX || n > ACI_MAX_MATRIX || k > ACI_MAX_MATRIX ||
      ngroup < 1 || ngroup > ACI_MAX_INPUTS)
    return set_err(ctx, ACI_E_LIMIT, "tuning shape out of range");
  const uint64_t key = ((uint64_t)m << 40) | ((uint64_t)k << 28) | ((uint64_t)n << 16) |
                       ((uint64_t)ngroup << 8) | ((uint64_t)prec << 4) | (uint64_t)(cplx ? 1 : 0);
  auto hit = ctx->tuned_tiles.find(key);
  if (hit != ctx->tuned_tiles.end() && !us) {
    *best = hit->second;
    return ACI_OK;
  }
  const int ew = cplx ? 2 : 1;
  const size_t na = (size_t)m * k * ew, nb = (size_t)k * n * ew, nc = (size_t)m * n * ew;
  void* ws = nullptr;
  if (!dev_alloc(ctx, &ws, (na + nb + nc * ngroup) * sizeof(double))) return set_err(ctx, ACI_E_NOMEM, "tuning workspace");
  double* A = (double*)ws;
  double* B = A + na;
  double* Cb = B + nb;
  std::vector<double> h(na + nb);
  SplitMix64 rng{0x7113ull + (uint64_t)m * 131u + (uint64_t)k * 7u + (uint64_t)n};
  for (double& x : h) x = rng.uniform();
  ContractArgs c{};
  c.cplx = cplx;
  c.ngroup = ngroup;
  for (int g = 0; g < ngroup; ++g) {
    c.g[g].nterm = 1;
    c.g[g].t[0] = Term{A, B, dconst(k), dconst(k), dconst(n)};
    c.g[g].C = Cb + (size_t)g * nc;
    c.g[g].M = dconst(m);
    c.g[g].N = dconst(n);
    c.g[g].ldc = dconst(n);
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = ACI_OK;
  float best_us = 1e30f;
  int bt = contract_default_tile(m, n, ngroup, cplx);
  if (hipMemcpy(A, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipGetLastError();
    rc = set_err(ctx, ACI_E_HIP, "tuning set-up");
  }
  for (int t = 0; t < NUM_TILES && rc == ACI_OK; ++t) {
    constexpr int reps = 3;
    hipError_t e = launch_contract(OP_NONE, prec, c, m, n, ctx->stream, t);
    if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_contract(OP_NONE, prec, c, m, n, ctx->stream, t);
    if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      rc = set_err(ctx, ACI_E_HIP, std::string("tuning launch: ") + hipGetErrorString(e));
      break;
    }
    const float t_us = 1e3f * ms / reps;
    if (us) us[t] = t_us;
    if (t_us < best_us) {
      best_us = t_us;
      bt = t;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(ctx->stream);
  dev_free(ctx, ws);
  if (rc) return rc;
  ctx->tuned_tiles[key] = bt;
  *best = bt;
  return ACI_OK;
}

struct Placement {
  int xcd = 0, max_groups = 0, cooperative = 1;
};
// the training set aci_proposal_dataset records into
struct RecordSpec {
  float* X = nullptr;
  float* y = nullptr;
  int64_t capacity = 0;
};
int session_create(aci_ctx* ctx, const aci_tt* inputs, int32_t n_inputs, int32_t dtype, int32_t op, double tol,
                   int32_t maxrank, const aci_options* opt, const Placement& pl, aci_session** out,
                   const RecordSpec* record = nullptr);
}  // namespace

int aci_session_create(aci_ctx* ctx, const aci_tt* inputs, int32_t n_inputs, int32_t dtype, int32_t op,
                       double tol, int32_t maxrank, const aci_options* opt, aci_session** out) {
  return session_create(ctx, inputs, n_inputs, dtype, op, tol, maxrank, opt, Placement{}, out);
}

namespace {
int session_create(aci_ctx* ctx, const aci_tt* inputs, int32_t n_inputs, int32_t dtype, int32_t op, double tol,
                   int32_t maxrank, const aci_options* opt, const Placement& pl, aci_session** out,
                   const RecordSpec* record) {
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  if (!out) return set_err(ctx, ACI_E_INVALID, "null session pointer");
  *out = nullptr;
  aci_options o{};
  o.maxiter = 20;
  if (opt) o = *opt;
  if (o.maxiter <= 0) o.maxiter = 20;
  std::unique_ptr<aci_session> S(new (std::nothrow) aci_session());
  if (!S) return set_err(ctx, ACI_E_NOMEM, "host allocation");
  S->ctx = ctx;
  S->plan.reset(new (std::nothrow) Plan());
  if (!S->plan) return set_err(ctx, ACI_E_NOMEM, "host allocation");
  Plan& p = *S->plan;
  int rc = plan_problem(ctx, inputs, n_inputs, dtype, op, tol, maxrank, o, p);
  if (rc) return rc;
  if (record) {
    p.rec_on = true;
    p.recX = record->X;
    p.recY = record->y;
    p.rec_cap = record->capacity;
  }
  S->fixed = p.fixed;
  S->prof.on = o.profile != 0;
  for (auto& row : p.tiles) std::fill(row, row + ACI_MAX_SITES + 2, -1);
  if (o.tune) {
    // contraction tile of every environment and two-site launch shape
    for (int l = 1; l < p.L; ++l) {
      int wl = 1, kl = 1, mr = 1, kr = 1, kp = 1;
      for (int n = 0; n < p.N; ++n) {
        wl = std::max(wl, p.d[l] * p.r[n][l]);
        kl = std::max(kl, p.r[n][l - 1]);
        mr = std::max(mr, p.r[n][l] * p.d[l + 1]);
        kr = std::max(kr, p.r[n][l + 1]);
        kp = std::max(kp, p.r[n][l]);
      }
      // shapes beyond the tuner's range (inputs of rank > ACI_MAX_MATRIX)
      // keep the default tile
      auto tunable = [](int m, int k, int n) {
        return m <= ACI_MAX_MATRIX && k <= ACI_MAX_MATRIX && n <= ACI_MAX_MATRIX;
      };
      if (tunable(p.capI[l - 1], kl, wl) &&
          (rc = tune_tile(ctx, p.cplx, p.prec, p.N, p.capI[l - 1], kl, wl, &p.tiles[0][l], nullptr)))
        return rc;
      if (tunable(mr, kr, p.capJ[l + 2]) &&
          (rc = tune_tile(ctx, p.cplx, p.prec, p.N, mr, kr, p.capJ[l + 2], &p.tiles[1][l], nullptr)))
        return rc;
      if (tunable(p.d[l] * p.capI[l - 1], kp, p.d[l + 1] * p.capJ[l + 2]) &&
          (rc = tune_tile(ctx, p.cplx, p.prec, 1, p.d[l] * p.capI[l - 1], kp, p.d[l + 1] * p.capJ[l + 2],
                          &p.tiles[2][l], nullptr)))
        return rc;
    }
  }
  // graphs need launches with static arguments: no events, no trace records
  S->use_graph = o.use_graph != 0 && !S->prof.on && !p.trace && p.op != ACI_OP_CUSTOM && !p.rec_on;
  p.xcd = pl.xcd;
  p.max_groups = pl.max_groups;
  if (S->use_graph) {
    // captured launches are plain launches: every LDU must fit one XCD
    const int mn = std::min(p.D * p.maxrank, (int)ACI_MAX_MATRIX);
    const int cap = pl.max_groups > 0 ? pl.max_groups : prrlu_xcd_cus();
    const int g = prrlu_groups(mn, mn, cap, p.cplx);
    if (g < 0 || g > cap) S->use_graph = false;
  }
  p.cooperative = S->use_graph ? 0 : pl.cooperative;
  {
    const size_t nb = sizeof(int) * (L_pad(p.L)) * 5 + sizeof(double) * L_pad(p.L) + 64;
    if (hipHostMalloc(&S->hbuf, nb, 0) != hipSuccess) {
      (void)hipGetLastError();
      return set_err(ctx, ACI_E_NOMEM, "pinned host allocation failed");
    }
    char* hb = (char*)S->hbuf;
    S->h_eps = (double*)hb;
    hb += sizeof(double) * L_pad(p.L);
    S->h_cur = (int*)hb;
    hb += sizeof(int) * L_pad(p.L);
    S->h_meta = (int*)hb;
    hb += sizeof(int) * 3 * L_pad(p.L);
    S->h_flags = (int*)hb;
  }
  const bool gen_init = (o.init == nullptr);
  Arena sz;
  layout(p, sz, gen_init);
  if (!dev_alloc(ctx, &S->ws, sz.off + 256)) return set_err(ctx, ACI_E_NOMEM, "workspace allocation failed");
  Arena ar;
  ar.base = (char*)S->ws;
  layout(p, ar, gen_init);
  HIPCHK(hipEventCreate(&S->e0));
  HIPCHK(hipEventCreate(&S->e1));
  hipStream_t s = ctx->stream;
  const int L = p.L;
  if (gen_init && p.sketch > 0) {
    // the random index sketch as a Y_init whose CI-canonical form selects
    // exactly the drawn points: sites L..1, rho_{l-1} distinct columns of
    // the d_l rho_l by partial Fisher-Yates, one non-zero per row
    SplitMix64 rng{o.seed};
    std::vector<double> h;
    std::vector<int> a;
    const double step = 0x1.0p-11;
    for (int l = L; l >= 1; --l) {
      const int r0 = p.rho[l - 1], r1 = p.rho[l], dl = p.d[l], n = dl * r1;
      h.assign((size_t)p.ew * r0 * dl * r1, 0.0);
      a.resize(n);
      for (int i = 0; i < n; ++i) a[i] = i;
      for (int s2 = 0; s2 < r0; ++s2) {
        const int j = s2 + (int)(rng.next() % (uint64_t)(n - s2));
        std::swap(a[s2], a[j]);
        const int q = a[s2], b = q % r1;
        h[(size_t)p.ew * ((size_t)s2 * n + q)] = (1.0 - s2 * step) / (1.0 - b * step);
      }
      HIPCHK(hipMemcpyAsync(p.Gin[l], h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, s));
      HIPCHK(hipStreamSynchronize(s));
      p.Yin[l] = p.Gin[l];
    }
  } else if (gen_init) {
    SplitMix64 rng{o.seed};
    std::vector<double> h;
    for (int l = 1; l <= L; ++l) {
      // complex entries take two consecutive draws (re, im)
      const size_t cnt = (size_t)p.ew * p.rho[l - 1] * p.d[l] * p.rho[l];
      h.resize(cnt);
      for (size_t i = 0; i < cnt; ++i) h[i] = rng.uniform();
      HIPCHK(hipMemcpyAsync(p.Gin[l], h.data(), cnt * sizeof(double), hipMemcpyHostToDevice, s));
      HIPCHK(hipStreamSynchronize(s));
      p.Yin[l] = p.Gin[l];
    }
  } else {
    for (int l = 1; l <= L; ++l) p.Yin[l] = (const double*)o.init->cores[l - 1];
  }
  Enq q{ctx, p, s, 0, 0, nullptr};
  rc = enqueue_init(q);
  if (rc) return rc;
  S->rec = q.rec;
  S->init_ranks[0] = S->init_ranks[L] = 1;
  HIPCHK(hipMemcpyAsync(S->init_ranks + 1, p.nJ + 2, sizeof(int) * (L - 1), hipMemcpyDeviceToHost, s));
  int flags[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(flags, p.flags, sizeof(flags), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (flags[0] & ERR_TIMEOUT) return set_err(ctx, ACI_E_TIMEOUT, "a pivot exchange exceeded its spin limit");
  if (flags[0] & ERR_LIMIT) return set_err(ctx, ACI_E_LIMIT, "a pivot index fell outside its matrix");
  S->prev.assign(S->init_ranks + 1, S->init_ranks + L);
  *out = S.release();
  return ACI_OK;
}
}  // namespace

namespace {

// Enqueues one sweep (or replays its graph) and the read-back of its ranks,
// error estimates, per-update meta and flags into pinned host memory.
// End of a sweep on stream s: the end event and the read-back of ranks, eps,
// meta and flags into pinned host memory.
int sweep_readback(aci_session* S, hipStream_t s) {
  aci_ctx* ctx = S->ctx;
  Plan& p = *S->plan;
  const int L = p.L;
  HIPCHK(hipEventRecord(S->e1, s));
  HIPCHK(hipMemcpyAsync(S->h_cur, p.nJ + 2, sizeof(int) * (L - 1), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(S->h_eps, p.eps_bond, sizeof(double) * (L - 1), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(S->h_meta, p.meta + 3 * (L - 1), sizeof(int) * 3 * 2 * (L - 1), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(S->h_flags, p.flags, sizeof(int) * 2, hipMemcpyDeviceToHost, s));
  if (p.mlp) HIPCHK(hipMemcpyAsync(S->h_flags + 2, p.acc_count, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
  return ACI_OK;
}

int sweep_enqueue(aci_session* S) {
  aci_ctx* ctx = S->ctx;
  Plan& p = *S->plan;
  const int L = p.L;
  hipStream_t s = ctx->stream;
  S->prof.clear();
  S->swept_prec = p.prec;
  if (int rc = epoch_guard(ctx, p, 2 * (L - 1), s)) return rc;
  HIPCHK(hipEventRecord(S->e0, s));
  if (S->use_graph) {
    if (!S->gexec || S->gprec != p.prec) {
      if (S->gexec) {
        HIPCHK(hipGraphExecDestroy(S->gexec));
        S->gexec = nullptr;
      }
      // captured on a private stream (the context's may be the null
      // stream, which cannot be captured), replayed on the context's
      hipGraph_t g = nullptr;
      if (!S->cap_stream) HIPCHK(hipStreamCreateWithFlags(&S->cap_stream, hipStreamNonBlocking));
      HIPCHK(hipStreamBeginCapture(S->cap_stream, hipStreamCaptureModeRelaxed));
      Enq q{ctx, p, S->cap_stream, S->rec, L - 1, &S->prof};
      const int rc = enqueue_sweep(q);
      const hipError_t ec = hipStreamEndCapture(S->cap_stream, &g);
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (ec != hipSuccess) return set_err(ctx, ACI_E_HIP, std::string("sweep capture: ") + hipGetErrorString(ec));
      const hipError_t ei = hipGraphInstantiate(&S->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ei != hipSuccess) return set_err(ctx, ACI_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(ei));
      S->gprec = p.prec;
    }
    HIPCHK(hipGraphLaunch(S->gexec, s));
  } else {
    Enq q{ctx, p, s, S->rec, L - 1, &S->prof};
    const int rc = enqueue_sweep(q);
    if (rc) return rc;
    S->rec = q.rec;
  }
  return sweep_readback(S, s);
}

// After the stream has drained: errors, statistics, launch log, the
// convergence test of Alg. 1 and the precision ladder.
int sweep_finish(aci_session* S, aci_sweep_stats& st) {
  aci_ctx* ctx = S->ctx;
  Plan& p = *S->plan;
  const int L = p.L;
  ++S->sweeps;
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, S->e0, S->e1));
  S->sweep_ms += ms;
  const int fl = S->h_flags[0];
  if (fl & ERR_TIMEOUT) return set_err(ctx, ACI_E_TIMEOUT, "a pivot exchange exceeded its spin limit");
  if (fl & ERR_NONFINITE) return set_err(ctx, ACI_E_NUMERIC, "NaN or Inf in a two-site tensor");
  if (fl & ERR_LIMIT) return set_err(ctx, ACI_E_LIMIT, "a pivot index fell outside its matrix");
  const int* meta = S->h_meta;
  for (size_t i = 0; i < S->prof.cls.size(); ++i) {
    float kms = 0.f;
    HIPCHK(hipEventElapsedTime(&kms, S->prof.pool[2 * i], S->prof.pool[2 * i + 1]));
    const int c = S->prof.cls[i];
    st.kernel_ms[c] += kms;
    st.launches[c] += 1;
    aci_launch rec{};
    rec.kind = c;
    rec.variant = S->prof.variant[i];
    rec.part = S->prof.part[i];
    rec.sweep = S->sweeps - 1;
    rec.update = S->prof.slot[i] - (L - 1);
    rec.us = 1e3f * kms;
    // flops of the LDU and contraction launches (not of the proposal kernels,
    // which are logged in the LDU class with codes 20001..20008)
    const bool proposal_kernel = c == CLS_PRRLU && rec.variant >= 20000 && rec.variant < 30000;
    if (rec.update >= 0 && rec.update < 2 * (L - 1) && c != CLS_GATHER && !proposal_kernel) {
      int kind, bond;
      update_of(L, rec.update, kind, bond);
      const int* mt = meta + 3 * rec.update;
      rec.flops = update_flops(p, kind, bond, mt[0], mt[1], mt[2], c == CLS_PRRLU ? 0 : rec.part);
    }
    S->log.push_back(rec);
  }
  for (int u = 0; u < 2 * (L - 1); ++u) {
    int kind, bond;
    update_of(L, u, kind, bond);
    account(p, kind, bond, meta[3 * u], meta[3 * u + 1], meta[3 * u + 2], st);
  }
  bool grew = false;
  double emax = 0.0;
  for (int b = 0; b < L - 1; ++b) {
    grew = grew || S->h_cur[b] > S->prev[b];
    emax = std::max(emax, S->h_eps[b]);
  }
  S->prev.assign(S->h_cur, S->h_cur + (L - 1));
  st.max_eps = emax;
  st.last_precision = S->swept_prec;
  if (p.mlp) {
    st.proposals_tried += 2 * (L - 1);
    st.proposals_accepted += S->h_flags[2];
    st.proposal_scans += S->h_flags[3];
    st.proposal_pivots += S->h_flags[4];
  }
  if (S->swept_prec == PREC_FP64) {
    S->converged = !grew && emax <= p.tol;
  } else {
    // precision ladder: a low-precision sweep never converges (its Pi
    // carries errors above the tolerance); the next sweeps run in FP64 once
    // a low-precision sweep kept the ranks or after low_max of them
    S->converged = false;
    ++S->low_done;
    if (p.low_max >= 0 && (!grew || S->low_done >= p.low_max)) p.prec = PREC_FP64;
  }
  return ACI_OK;
}

void stats_tail(aci_session* S, aci_sweep_stats& st) {
  const int L = S->plan->L;
  st.sweeps_done = S->sweeps;
  st.converged = S->converged ? 1 : 0;
  st.ranks[0] = st.ranks[L] = 1;
  for (int b = 1; b < L; ++b) st.ranks[b] = S->prev[b - 1];
}

}  // namespace

int aci_session_sweep(aci_session* S, int32_t nsweeps, aci_sweep_stats* stats) {
  if (!S || !S->ctx) return ACI_E_INVALID;
  aci_ctx* ctx = S->ctx;
  ctx->err.clear();
  if (nsweeps < 0) return set_err(ctx, ACI_E_INVALID, "nsweeps < 0");
  aci_sweep_stats st{};
  S->log.clear();
  for (int it = 0; it < nsweeps; ++it) {
    int rc = sweep_enqueue(S);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    rc = sweep_finish(S, st);
    if (rc) return rc;
    if (S->converged && !S->fixed) break;
  }
  stats_tail(S, st);
  if (stats) *stats = st;
  return S->converged ? ACI_OK : ACI_W_NOT_CONVERGED;
}

int aci_session_result(aci_session* S, void* out, int64_t out_capacity, aci_result* result) {
  if (!S || !S->ctx) return ACI_E_INVALID;
  aci_ctx* ctx = S->ctx;
  ctx->err.clear();
  if (!out || !result) return set_err(ctx, ACI_E_INVALID, "null argument");
  std::memset(result, 0, sizeof(*result));
  if (S->sweeps < 1) return set_err(ctx, ACI_E_INVALID, "no sweep has run");
  Plan& p = *S->plan;
  const int L = p.L;
  const int maxrank = p.maxrank;
  hipStream_t s = ctx->stream;
  std::vector<int> cur(L - 1);
  std::vector<double> epsb(L - 1);
  HIPCHK(hipMemcpyAsync(cur.data(), p.nJ + 2, sizeof(int) * (L - 1), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(epsb.data(), p.eps_bond, sizeof(double) * (L - 1), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  result->L = L;
  result->sweeps = S->sweeps;
  result->converged = S->converged ? 1 : 0;
  result->sweep_ms = S->sweep_ms;
  std::memcpy(result->init_ranks, S->init_ranks, sizeof(int) * (L + 1));
  result->ranks[0] = result->ranks[L] = 1;
  for (int b = 1; b < L; ++b) {
    result->ranks[b] = cur[b - 1];
    result->eps[b - 1] = epsb[b - 1];
  }
  int64_t off = 0;
  for (int l = 1; l <= L; ++l) off += (int64_t)result->ranks[l - 1] * p.d[l] * result->ranks[l];
  if (off > out_capacity) return set_err(ctx, ACI_E_NOMEM, "output buffer too small");
  off = 0;
  for (int l = 1; l <= L; ++l) {
    const int64_t cnt = (int64_t)result->ranks[l - 1] * p.d[l] * result->ranks[l];
    result->core_offset[l - 1] = off;
    HIPCHK(hipMemcpyAsync((double*)out + off * p.ew, p.Ycore[l], cnt * p.ew * sizeof(double), hipMemcpyDeviceToDevice,
                          s));
    off += cnt;
  }
  result->out_elems = off;
  {
    // nested index sets of the last sweep, as the oracle keeps them: I_l
    // from the rows of the right-to-left update at bond l (through the I_{l-1}
    // of the left-to-right half), J_{l+1} from its columns (through J_{l+2})
    const size_t per = (size_t)(L + 1) * maxrank;
    std::vector<int> lr(per), rr(per), rc(per), nI(L + 2), nJ(L + 3);
    HIPCHK(hipMemcpyAsync(lr.data(), p.pivLR, sizeof(int) * per, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(rr.data(), p.pivRLr, sizeof(int) * per, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(rc.data(), p.pivRLc, sizeof(int) * per, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(nI.data(), p.nI, sizeof(int) * (L + 2), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(nJ.data(), p.nJ, sizeof(int) * (L + 3), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    // I^LR_l, l = 0..L-2, as nI[l] strings of l digits
    std::vector<std::vector<uint8_t>> ilr(L);
    ilr[0].clear();
    bool ok = true;
    for (int l = 1; l <= L - 2 && ok; ++l) {
      const int cnt = nI[l], prev = l == 1 ? 1 : nI[l - 1], d = p.d[l];
      ilr[l].resize((size_t)cnt * l);
      for (int k = 0; k < cnt && ok; ++k) {
        const int row = lr[(size_t)l * maxrank + k], a = row / d;
        ok = row >= 0 && a < prev;
        if (!ok) break;
        for (int t = 0; t < l - 1; ++t) ilr[l][(size_t)k * l + t] = ilr[l - 1][(size_t)a * (l - 1) + t];
        ilr[l][(size_t)k * l + l - 1] = (uint8_t)(row % d);
      }
    }
    int64_t ni = 0, nj = 0;
    for (int l = 1; l < L; ++l) {
      ni += (int64_t)result->ranks[l] * l;
      nj += (int64_t)result->ranks[l] * (L - l);
    }
    result->I_idx = (uint8_t*)calloc(std::max<int64_t>(ni, 1), 1);
    result->J_idx = (uint8_t*)calloc(std::max<int64_t>(nj, 1), 1);
    if (!result->I_idx || !result->J_idx) {
      aci_result_free(result);
      return set_err(ctx, ACI_E_NOMEM, "host allocation of the index sets");
    }
    int64_t oi = 0;
    for (int l = 1; l < L && ok; ++l) {
      const int cnt = result->ranks[l], prev = l == 1 ? 1 : nI[l - 1], d = p.d[l];
      result->I_off[l - 1] = oi;
      for (int k = 0; k < cnt && ok; ++k) {
        const int row = rr[(size_t)l * maxrank + k], a = row / d;
        ok = row >= 0 && a < prev;
        if (!ok) break;
        uint8_t* dst = result->I_idx + oi + (int64_t)k * l;
        for (int t = 0; t < l - 1; ++t) dst[t] = ilr[l - 1][(size_t)a * (l - 1) + t];
        dst[l - 1] = (uint8_t)(row % d);
      }
      oi += (int64_t)cnt * l;
    }
    // J_{l+1}, l = L-1 .. 1: ranks[l] strings of L - l digits
    int64_t oj = nj;
    std::vector<int64_t> joff(L + 2, 0);
    for (int l = L - 1; l >= 1 && ok; --l) {
      const int cnt = result->ranks[l], w = L - l, cR = l == L - 1 ? 1 : result->ranks[l + 1];
      oj -= (int64_t)cnt * w;
      joff[l] = oj;
      result->J_off[l - 1] = oj;
      for (int k = 0; k < cnt && ok; ++k) {
        const int col = rc[(size_t)l * maxrank + k], b = col % cR;
        ok = col >= 0 && col / cR < p.d[l + 1];
        if (!ok) break;
        uint8_t* dst = result->J_idx + oj + (int64_t)k * w;
        dst[0] = (uint8_t)(col / cR);
        for (int t = 1; t < w; ++t) dst[t] = result->J_idx[joff[l + 1] + (int64_t)b * (w - 1) + t - 1];
      }
    }
    if (!ok) {
      aci_result_free(result);
      return set_err(ctx, ACI_E_LIMIT, "a pivot index fell outside its matrix");
    }
  }
  if (p.trace) {
    const int nr = std::min(S->rec, p.n_rec);
    result->n_records = nr;
    result->record_stride = maxrank;
    result->rec_meta = (int32_t*)calloc((size_t)nr * 6, sizeof(int32_t));
    result->rec_eps = (double*)calloc(nr, sizeof(double));
    result->rec_rows = (int32_t*)calloc((size_t)nr * maxrank, sizeof(int32_t));
    result->rec_cols = (int32_t*)calloc((size_t)nr * maxrank, sizeof(int32_t));
    if (!result->rec_meta || !result->rec_eps || !result->rec_rows || !result->rec_cols) {
      aci_result_free(result);
      return set_err(ctx, ACI_E_NOMEM, "host allocation of the trace");
    }
    HIPCHK(hipMemcpyAsync(result->rec_eps, p.tr_eps, sizeof(double) * nr, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(result->rec_rows, p.tr_rows, sizeof(int) * (size_t)nr * maxrank, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(result->rec_cols, p.tr_cols, sizeof(int) * (size_t)nr * maxrank, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::vector<int> meta3((size_t)3 * nr);
    HIPCHK(hipMemcpy(meta3.data(), p.tr_meta, sizeof(int) * 3 * nr, hipMemcpyDeviceToHost));
    int r = 0;
    auto put = [&](int kind, int sweep, int bond) {
      if (r >= nr) return;
      int* m6 = result->rec_meta + 6 * r;
      m6[0] = kind;
      m6[1] = sweep;
      m6[2] = bond;
      m6[3] = meta3[3 * r];
      m6[4] = meta3[3 * r + 1];
      m6[5] = meta3[3 * r + 2];
      ++r;
    };
    for (int l = L; l >= 2; --l) put(0, 0, l);
    for (int it = 1; it <= S->sweeps; ++it) {
      for (int l = 1; l <= L - 1; ++l) put(1, it, l);
      for (int l = L - 1; l >= 1; --l) put(2, it, l);
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  return S->converged ? ACI_OK : ACI_W_NOT_CONVERGED;
}

int aci_tci(aci_ctx* ctx, int32_t L, const int32_t* d, int32_t dtype, aci_eval_fn f, void* user,
            int32_t* idx_buf, void* val_buf, int64_t buf_points, const int32_t* pivots, int32_t n_pivots,
            double tol, int32_t maxrank, const aci_options* opt, void* out, int64_t out_capacity,
            aci_result* result) {
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  if (!d || !f || !idx_buf || !val_buf || !out || !result) return set_err(ctx, ACI_E_INVALID, "null argument");
  std::memset(result, 0, sizeof(*result));
  if (L < 2 || L > ACI_MAX_SITES) return set_err(ctx, ACI_E_LIMIT, "L out of range");
  if (dtype != ACI_F64 && dtype != ACI_C128) return set_err(ctx, ACI_E_DTYPE, "unknown dtype");
  if (!(tol >= 0.0)) return set_err(ctx, ACI_E_INVALID, "tol must be >= 0");
  if (maxrank < 1 || maxrank > ACI_MAX_RANK) return set_err(ctx, ACI_E_LIMIT, "maxrank out of range");
  if (n_pivots < 0 || (n_pivots > 0 && !pivots)) return set_err(ctx, ACI_E_INVALID, "bad pivots");
  aci_options o{};
  o.maxiter = 20;
  if (opt) o = *opt;
  if (o.maxiter < 1) return set_err(ctx, ACI_E_INVALID, "maxiter must be >= 1");
  const int cplx = dtype == ACI_C128 ? 1 : 0, ew = cplx ? 2 : 1;
  std::vector<int> dd(L + 2, 1);
  int D = 1;
  for (int l = 1; l <= L; ++l) {
    dd[l] = d[l - 1];
    if (dd[l] < 1 || dd[l] > ACI_MAX_DIM) return set_err(ctx, ACI_E_LIMIT, "local dimension out of range");
    D = std::max(D, dd[l]);
  }
  if ((long long)D * maxrank > ACI_MAX_MATRIX) return set_err(ctx, ACI_E_LIMIT, "d * maxrank above ACI_MAX_MATRIX");
  const int ldmax = D * maxrank;
  if (buf_points < (int64_t)ldmax * ldmax) return set_err(ctx, ACI_E_LIMIT, "point buffers below (d maxrank)^2");
  // ---- initial index sets: distinct prefixes / suffixes of the pivots
  std::vector<std::vector<int32_t>> piv;
  if (n_pivots == 0) piv.push_back(std::vector<int32_t>(L, 0));
  for (int i = 0; i < n_pivots; ++i) {
    std::vector<int32_t> v(pivots + (size_t)i * L, pivots + (size_t)(i + 1) * L);
    for (int t = 0; t < L; ++t)
      if (v[t] < 0 || v[t] >= dd[t + 1]) return set_err(ctx, ACI_E_INVALID, "pivot digit out of range");
    piv.push_back(v);
  }
  std::vector<int> nI(L + 2, 0), nJ(L + 3, 0);
  const size_t setw = (size_t)maxrank * L;   // one index set: maxrank digit rows of length L
  std::vector<int32_t> hI((size_t)(L + 1) * setw, 0), hJ((size_t)(L + 2) * setw, 0);
  nI[0] = 1;
  nJ[L + 1] = 1;
  for (int l = 1; l < L; ++l) {
    std::vector<std::vector<int32_t>> seen;
    for (auto& v : piv) {
      std::vector<int32_t> pre(v.begin(), v.begin() + l);
      if (std::find(seen.begin(), seen.end(), pre) == seen.end()) seen.push_back(pre);
    }
    if ((int)seen.size() > maxrank) return set_err(ctx, ACI_E_LIMIT, "more distinct pivot prefixes than maxrank");
    nI[l] = (int)seen.size();
    for (int k = 0; k < nI[l]; ++k) std::copy(seen[k].begin(), seen[k].end(), hI.begin() + l * setw + (size_t)k * L);
  }
  for (int l = 2; l <= L; ++l) {
    std::vector<std::vector<int32_t>> seen;
    for (auto& v : piv) {
      std::vector<int32_t> suf(v.begin() + (l - 1), v.end());
      if (std::find(seen.begin(), seen.end(), suf) == seen.end()) seen.push_back(suf);
    }
    if ((int)seen.size() > maxrank) return set_err(ctx, ACI_E_LIMIT, "more distinct pivot suffixes than maxrank");
    nJ[l] = (int)seen.size();
    for (int k = 0; k < nJ[l]; ++k) std::copy(seen[k].begin(), seen[k].end(), hJ.begin() + l * setw + (size_t)k * L);
  }
  // ---- device workspace
  const size_t xwords = prrlu_xbuf_words(ldmax, ldmax, cplx);
  size_t ycore = 0;
  for (int l = 1; l <= L; ++l) ycore += (size_t)maxrank * dd[l] * maxrank * ew;
  const size_t bytes = sizeof(int32_t) * ((size_t)(L + 1) * setw + (size_t)(L + 2) * setw) +
                       sizeof(double) * ycore + sizeof(uint64_t) * xwords +
                       sizeof(int) * (2 * (size_t)maxrank + 16) + sizeof(double) * 8 + 4096;
  void* ws = nullptr;
  if (!dev_alloc(ctx, &ws, bytes)) return set_err(ctx, ACI_E_NOMEM, "TCI workspace");
  char* base = (char*)ws;
  auto take = [&](size_t nbytes) {
    char* q = base;
    base += (nbytes + 255) & ~(size_t)255;
    return q;
  };
  int32_t* dI = (int32_t*)take(sizeof(int32_t) * (size_t)(L + 1) * setw);
  int32_t* dJ = (int32_t*)take(sizeof(int32_t) * (size_t)(L + 2) * setw);
  uint64_t* xbuf = (uint64_t*)take(sizeof(uint64_t) * xwords);
  int* rows = (int*)take(sizeof(int) * maxrank);
  int* cols = (int*)take(sizeof(int) * maxrank);
  int* misc = (int*)take(sizeof(int) * 16);   // [0] rank, [4] flags, [5] abort, [8] epoch
  double* peps = (double*)take(sizeof(double) * 8);
  std::vector<double*> Y(L + 1, nullptr);
  for (int l = 1; l <= L; ++l) Y[l] = (double*)take(sizeof(double) * (size_t)maxrank * dd[l] * maxrank * ew);
  hipStream_t s = ctx->stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = ACI_OK;
  auto fail = [&](int code, const std::string& msg) {
    rc = set_err(ctx, code, msg);
    return rc;
  };
#define TCICHK(call)                                                                      \
  do {                                                                                    \
    const hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) {                                                               \
      (void)hipGetLastError();                                                            \
      fail(ACI_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));                 \
      goto done;                                                                          \
    }                                                                                     \
  } while (0)
  {
    std::vector<int> rho(L + 1, 1), rho_prev(L + 1, 1);
    std::vector<double> eps_rl(L + 1, 0.0);
    for (int l = 1; l < L; ++l) rho_prev[l] = nJ[l + 1];
    int sweeps = 0;
    bool converged = false;
    float ms_total = 0.f;
    TCICHK(hipMemcpyAsync(dI, hI.data(), sizeof(int32_t) * hI.size(), hipMemcpyHostToDevice, s));
    TCICHK(hipMemcpyAsync(dJ, hJ.data(), sizeof(int32_t) * hJ.size(), hipMemcpyHostToDevice, s));
    TCICHK(launch_fill_int((int*)xbuf, 2 * xwords, 0, s));
    TCICHK(launch_fill_int(misc, 16, 0, s));
    TCICHK(launch_fill_int(misc + 8, 1, 1, s));
    TCICHK(hipEventCreate(&e0));
    TCICHK(hipEventCreate(&e1));
    for (int it = 1; it <= o.maxiter; ++it) {
      sweeps = it;
      TCICHK(hipEventRecord(e0, s));
      for (int u = 0; u < 2 * (L - 1); ++u) {
        const bool lr = u < L - 1;
        const int l = lr ? u + 1 : 2 * (L - 1) - u;
        const int cR = nJ[l + 2], m = nI[l - 1] * dd[l], n = dd[l + 1] * cR;
        TciPointsArgs pa{};
        pa.I_prev = dI + (size_t)(l - 1) * setw;
        pa.J_next = dJ + (size_t)(l + 2) * setw;
        pa.pts = idx_buf;
        pa.m = m;
        pa.n = n;
        pa.d = dd[l];
        pa.cR = cR;
        pa.l = l;
        pa.L = L;
        TCICHK(launch_tci_points(pa, s));
        if (f((int64_t)m * n, L, user, (void*)s) != 0) {
          fail(ACI_E_INVALID, "the point evaluator failed");
          goto done;
        }
        PrrluArgs a{};
        a.cplx = cplx;
        a.M = (const double*)val_buf;
        a.m = dconst(m);
        a.n = dconst(n);
        a.ldm = dconst(n);
        a.tol = tol;
        a.maxrank = maxrank;
        a.rule = o.stop_rule == 1 ? RULE_LITERAL : RULE_EXCLUSIVE;
        a.xbuf = xbuf;
        a.xbuf_words = xwords;
        exchange_waits(ctx, a);
        a.rows = rows;
        a.cols = cols;
        a.rank = misc;
        a.eps = peps;
        a.Y = lr ? nullptr : Y[l + 1];
        a.ldy = dconst(n);
        a.err = misc + 4;
        a.abort_word = misc + 5;
        a.epoch = (uint32_t*)(misc + 8);
        a.xcd = 0;
        a.max_groups = 0;
        a.cooperative = 1;
        TCICHK(launch_prrlu(a, m, n, s));
        TciSetsArgs sa{};
        sa.rows = rows;
        sa.cols = cols;
        sa.rank = misc;
        sa.I_prev = pa.I_prev;
        sa.J_next = pa.J_next;
        sa.I_out = dI + (size_t)l * setw;
        sa.J_out = dJ + (size_t)(l + 1) * setw;
        sa.d = dd[l];
        sa.cR = cR;
        sa.l = l;
        sa.L = L;
        TCICHK(launch_tci_sets(sa, std::min(maxrank, std::min(m, n)), s));
        if (!lr && l == 1) {
          // Y_1 = M[:, J_2] (the left factor of the last update, Alg. 3)
          GatherArgs g{};
          g.esz = ew;
          g.count = 1;
          g.side = 1;
          g.idx = cols;
          g.rank = misc;
          g.err = misc + 4;
          g.it[0] = GatherItem{(const double*)val_buf, Y[1], dconst(n), ddev(misc), dconst(m), dconst(n)};
          TCICHK(launch_gather(g, std::min(maxrank, n), m, s));
        }
        int hr[8];
        double he = 0.0;
        TCICHK(hipMemcpyAsync(hr, misc, sizeof(int) * 8, hipMemcpyDeviceToHost, s));
        TCICHK(hipMemcpyAsync(&he, peps, sizeof(double), hipMemcpyDeviceToHost, s));
        TCICHK(hipStreamSynchronize(s));
        if (hr[4] & ERR_TIMEOUT) {
          fail(ACI_E_TIMEOUT, "a pivot exchange exceeded its spin limit");
          goto done;
        }
        if (hr[4] & ERR_LIMIT) {
          fail(ACI_E_LIMIT, "a pivot index fell outside its matrix");
          goto done;
        }
        if (!(he == he)) {
          fail(ACI_E_NUMERIC, "NaN in the evaluated two-site tensor");
          goto done;
        }
        nI[l] = hr[0];
        nJ[l + 1] = hr[0];
        if (!lr) {
          rho[l] = hr[0];
          eps_rl[l] = he;
        }
      }
      TCICHK(hipEventRecord(e1, s));
      TCICHK(hipEventSynchronize(e1));
      float ms = 0.f;
      TCICHK(hipEventElapsedTime(&ms, e0, e1));
      ms_total += ms;
      bool grew = false;
      double emax = 0.0;
      for (int l = 1; l < L; ++l) {
        grew = grew || rho[l] > rho_prev[l];
        emax = std::max(emax, eps_rl[l]);
      }
      rho_prev = rho;
      converged = !grew && emax <= tol;
      if (converged && !o.fixed_sweeps) break;
    }
    // ---- result
    result->L = L;
    result->sweeps = sweeps;
    result->converged = converged ? 1 : 0;
    result->sweep_ms = ms_total;
    result->ranks[0] = result->ranks[L] = 1;
    result->init_ranks[0] = result->init_ranks[L] = 1;
    for (int l = 1; l < L; ++l) {
      result->ranks[l] = rho[l];
      result->eps[l - 1] = eps_rl[l];
      result->init_ranks[l] = (int)std::min<size_t>(piv.size(), (size_t)maxrank);
    }
    int64_t off = 0;
    for (int l = 1; l <= L; ++l) off += (int64_t)result->ranks[l - 1] * dd[l] * result->ranks[l];
    if (off > out_capacity) {
      fail(ACI_E_NOMEM, "output buffer too small");
      goto done;
    }
    off = 0;
    for (int l = 1; l <= L; ++l) {
      const int64_t cnt = (int64_t)result->ranks[l - 1] * dd[l] * result->ranks[l];
      result->core_offset[l - 1] = off;
      TCICHK(hipMemcpyAsync((double*)out + off * ew, Y[l], cnt * ew * sizeof(double), hipMemcpyDeviceToDevice, s));
      off += cnt;
    }
    result->out_elems = off;
    // index sets I_l, J_{l+1} of the last updates (right to left)
    TCICHK(hipMemcpyAsync(hI.data(), dI, sizeof(int32_t) * hI.size(), hipMemcpyDeviceToHost, s));
    TCICHK(hipMemcpyAsync(hJ.data(), dJ, sizeof(int32_t) * hJ.size(), hipMemcpyDeviceToHost, s));
    TCICHK(hipStreamSynchronize(s));
    int64_t ni = 0, nj = 0;
    for (int l = 1; l < L; ++l) {
      ni += (int64_t)rho[l] * l;
      nj += (int64_t)rho[l] * (L - l);
    }
    result->I_idx = (uint8_t*)calloc(std::max<int64_t>(ni, 1), 1);
    result->J_idx = (uint8_t*)calloc(std::max<int64_t>(nj, 1), 1);
    if (!result->I_idx || !result->J_idx) {
      aci_result_free(result);
      fail(ACI_E_NOMEM, "host allocation of the index sets");
      goto done;
    }
    int64_t oi = 0, oj = 0;
    for (int l = 1; l < L; ++l) {
      result->I_off[l - 1] = oi;
      result->J_off[l - 1] = oj;
      for (int k = 0; k < rho[l]; ++k) {
        for (int t = 0; t < l; ++t) result->I_idx[oi + (int64_t)k * l + t] = (uint8_t)hI[l * setw + (size_t)k * L + t];
        for (int t = 0; t < L - l; ++t)
          result->J_idx[oj + (int64_t)k * (L - l) + t] = (uint8_t)hJ[(l + 1) * setw + (size_t)k * L + t];
      }
      oi += (int64_t)rho[l] * l;
      oj += (int64_t)rho[l] * (L - l);
    }
    rc = converged ? ACI_OK : ACI_W_NOT_CONVERGED;
  }
done:
#undef TCICHK
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  dev_free(ctx, ws);
  return rc;
}

int aci_elementwise(aci_ctx* ctx, const aci_tt* inputs, int32_t n_inputs, int32_t dtype, int32_t op,
                    double tol, int32_t maxrank, const aci_options* opt, void* out, int64_t out_capacity,
                    aci_result* result) {
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  if (!result || !out) return set_err(ctx, ACI_E_INVALID, "null argument");
  std::memset(result, 0, sizeof(*result));
  aci_options o{};
  o.maxiter = 20;
  if (opt) o = *opt;
  if (o.maxiter <= 0) o.maxiter = 20;
  aci_session* S = nullptr;
  int rc = aci_session_create(ctx, inputs, n_inputs, dtype, op, tol, maxrank, &o, &S);
  if (rc < 0) return rc;
  if (S->plan->prec != PREC_FP64 && o.maxiter > 1) {
    // precision ladder: the last allowed sweep is always FP64, so the
    // returned cores, ranks and error estimates are FP64 results
    rc = aci_session_sweep(S, o.maxiter - 1, nullptr);
    if (rc >= 0 && !S->converged) {
      S->plan->prec = PREC_FP64;
      rc = aci_session_sweep(S, 1, nullptr);
    }
  } else {
    if (S->plan->prec != PREC_FP64) S->plan->prec = PREC_FP64;
    rc = aci_session_sweep(S, o.maxiter, nullptr);
  }
  if (rc < 0) {
    aci_session_destroy(S);
    return rc;
  }
  rc = aci_session_result(S, out, out_capacity, result);
  aci_session_destroy(S);
  return rc;
}

// ------------------------------------------------------------ batches
struct aci_batch {
  aci_ctx* parent = nullptr;
  bool serial = false;   // products swept one after another (cooperative LDUs)
  // joint: the products advance update by update together, and the LDUs of
  // one local update run as one launch with every product on its own XCD
  bool joint = false;
  bool jgraph = false;   // joint sweeps captured once into a hipGraph
  std::vector<hipStream_t> streams;
  std::vector<aci_ctx*> ctxs;
  std::vector<aci_session*> sess;
  std::vector<int> groups;
  hipEvent_t ready = nullptr;
  hipStream_t jstream = nullptr;     // the joint LDU launches
  hipEvent_t jdone = nullptr, jfork = nullptr;
  std::vector<hipEvent_t> pre;       // per product: update stage 0 enqueued
  hipGraphExec_t jexec = nullptr;
  std::vector<int> jkey;             // products and precisions jexec was captured for
};

void aci_batch_destroy(aci_batch* B) {
  if (!B) return;
  if (B->jstream) (void)hipStreamSynchronize(B->jstream);
  for (hipStream_t st : B->streams) (void)hipStreamSynchronize(st);
  for (aci_session* S : B->sess) aci_session_destroy(S);
  for (aci_ctx* c : B->ctxs) aci_ctx_destroy(c);
  for (hipStream_t st : B->streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  if (B->ready) (void)hipEventDestroy(B->ready);
  if (B->jexec) (void)hipGraphExecDestroy(B->jexec);
  if (B->jstream) {
    (void)hipStreamSynchronize(B->jstream);
    (void)hipStreamDestroy(B->jstream);
  }
  if (B->jdone) (void)hipEventDestroy(B->jdone);
  if (B->jfork) (void)hipEventDestroy(B->jfork);
  for (hipEvent_t e : B->pre) (void)hipEventDestroy(e);
  delete B;
}

extern "C++" {
namespace {

// The 2(L-1) local updates of one sweep of the active products `ids`, in
// lockstep: per update, every product's contractions on its own stream, then
// one batched LDU launch on the joint stream, then every product's gathers.
// With `timed`, each product's start event is recorded first (not inside a
// graph capture).
int joint_enqueue(aci_batch* B, const std::vector<int>& ids, bool timed) {
  aci_ctx* ctx = B->parent;
  const int L = B->sess[ids[0]]->plan->L;
  std::vector<Enq> qs;
  qs.reserve(ids.size());
  for (int b : ids) {
    aci_session* S = B->sess[b];
    S->prof.clear();
    S->swept_prec = S->plan->prec;
    if (timed) HIPCHK(hipEventRecord(S->e0, B->streams[b]));
    qs.push_back(Enq{B->ctxs[b], *S->plan, B->streams[b], S->rec, L - 1, &S->prof});
    qs.back().defer = true;
    qs.back().sweeping = true;
  }
  const int cnt = (int)ids.size();
  std::vector<PrrluArgs> args(cnt);
  std::vector<int> mm(cnt);
  auto fail = [&](int i, int rc) {
    return set_err(ctx, rc, std::string("product ") + std::to_string(ids[i]) + ": " + B->ctxs[ids[i]]->err);
  };
  for (int u = 0; u < 2 * (L - 1); ++u) {
    int nmax = 1;
    for (int i = 0; i < cnt; ++i) {
      Enq& q = qs[i];
      q.has_pend = false;
      if (int rc = enqueue_update(q, u, 0)) return fail(i, rc);
      if (!q.has_pend) return set_err(ctx, ACI_E_INVALID, "joint batch: update without an LDU");
      args[i] = q.pend;
      mm[i] = q.pend_mmax;
      nmax = std::max(nmax, q.pend_nmax);
      HIPCHK(hipEventRecord(B->pre[ids[i]], B->streams[ids[i]]));
      HIPCHK(hipStreamWaitEvent(B->jstream, B->pre[ids[i]], 0));
    }
    // the batched LDU, logged as a launch of the first active product
    Enq& q0 = qs[0];
    const hipStream_t own = q0.s;
    q0.s = B->jstream;
    if (int rc = q0.begin(CLS_PRRLU, prrlu_batch_variant(mm.data(), cnt, nmax, q0.p.cplx))) return fail(0, rc);
    const hipError_t e = launch_prrlu_batch(args.data(), mm.data(), cnt, nmax, B->jstream);
    if (e != hipSuccess) return set_err(ctx, ACI_E_HIP, std::string("batched prrlu launch: ") + hipGetErrorString(e));
    if (int rc = q0.end()) return fail(0, rc);
    q0.s = own;
    HIPCHK(hipEventRecord(B->jdone, B->jstream));
    for (int i = 0; i < cnt; ++i) {
      HIPCHK(hipStreamWaitEvent(B->streams[ids[i]], B->jdone, 0));
      if (int rc = enqueue_update(qs[i], u, 1)) return fail(i, rc);
    }
  }
  for (int i = 0; i < cnt; ++i) B->sess[ids[i]]->rec = qs[i].rec;
  return ACI_OK;
}

// One joint sweep of the active products, replayed from a captured graph
// when the batch uses graphs, followed by every product's read-back.
int joint_sweep(aci_batch* B, const std::vector<int>& ids) {
  aci_ctx* ctx = B->parent;
  // the joint LDU launches run on the joint stream
  for (int b : ids) {
    Plan& p = *B->sess[b]->plan;
    if (int rc = epoch_guard(ctx, p, 2 * (p.L - 1), B->jstream)) return rc;
  }
  if (!B->jgraph) {
    if (int rc = joint_enqueue(B, ids, true)) return rc;
  } else {
    std::vector<int> key(B->sess.size(), -1);
    for (int b : ids) key[b] = B->sess[b]->plan->prec;
    if (!B->jexec || key != B->jkey) {
      if (B->jexec) {
        HIPCHK(hipGraphExecDestroy(B->jexec));
        B->jexec = nullptr;
      }
      // every product stream joins the capture through the fork event and
      // is joined back before it ends
      HIPCHK(hipStreamBeginCapture(B->jstream, hipStreamCaptureModeRelaxed));
      int rc = ACI_OK;
      hipError_t ec = hipEventRecord(B->jfork, B->jstream);
      for (int b : ids)
        if (ec == hipSuccess) ec = hipStreamWaitEvent(B->streams[b], B->jfork, 0);
      if (ec == hipSuccess) rc = joint_enqueue(B, ids, false);
      for (int b : ids)
        if (ec == hipSuccess && rc == ACI_OK) {
          ec = hipEventRecord(B->pre[b], B->streams[b]);
          if (ec == hipSuccess) ec = hipStreamWaitEvent(B->jstream, B->pre[b], 0);
        }
      hipGraph_t g = nullptr;
      const hipError_t ee = hipStreamEndCapture(B->jstream, &g);
      if (rc || ec != hipSuccess || ee != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        if (rc) return rc;
        return set_err(ctx, ACI_E_HIP, std::string("joint sweep capture: ") +
                                           hipGetErrorString(ec != hipSuccess ? ec : ee));
      }
      const hipError_t ei = hipGraphInstantiate(&B->jexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ei != hipSuccess) return set_err(ctx, ACI_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(ei));
      B->jkey = key;
    }
    for (int b : ids) {
      aci_session* S = B->sess[b];
      S->prof.clear();
      S->swept_prec = S->plan->prec;
      HIPCHK(hipEventRecord(S->e0, B->jstream));
    }
    HIPCHK(hipGraphLaunch(B->jexec, B->jstream));
    HIPCHK(hipEventRecord(B->jdone, B->jstream));
    for (int b : ids) HIPCHK(hipStreamWaitEvent(B->streams[b], B->jdone, 0));
  }
  for (int b : ids) {
    if (int rc = sweep_readback(B->sess[b], B->streams[b]))
      return set_err(ctx, rc, std::string("product ") + std::to_string(b) + ": " + B->ctxs[b]->err);
  }
  return ACI_OK;
}

}  // namespace
}  // extern "C++"

int aci_batch_create(aci_ctx* ctx, const aci_tt* inputs, const int32_t* n_inputs, int32_t n_products,
                     int32_t dtype, int32_t op, double tol, int32_t maxrank, const aci_options* opt,
                     aci_batch** out) {
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  if (!out || !inputs || !n_inputs) return set_err(ctx, ACI_E_INVALID, "null argument");
  *out = nullptr;
  if (n_products < 1 || n_products > ACI_MAX_BATCH) return set_err(ctx, ACI_E_LIMIT, "n_products out of range");
  aci_options o{};
  o.maxiter = 20;
  if (opt) o = *opt;
  if (o.init) return set_err(ctx, ACI_E_INVALID, "a batch takes the default initial guess (options.init must be NULL)");
  if (o.batch_mode < 0 || o.batch_mode > 3) return set_err(ctx, ACI_E_INVALID, "batch_mode must be 0..3");
  std::unique_ptr<aci_batch, void (*)(aci_batch*)> B(new (std::nothrow) aci_batch(), aci_batch_destroy);
  if (!B) return set_err(ctx, ACI_E_NOMEM, "host allocation");
  B->parent = ctx;
  HIPCHK(hipEventCreateWithFlags(&B->ready, hipEventDisableTiming));
  HIPCHK(hipEventRecord(B->ready, ctx->stream));
  // Placement: the products' sweeps overlap on their own streams, so their
  // LDU launches spin side by side.  Each launches exactly its P groups,
  // dealt round robin over the 8 XCDs (ceil(P/8) per XCD); with P capped at
  // 8 * floor(CUs per XCD / products) every XCD can hold all the groups of
  // all products at once, one per CU, so no launch waits for CUs held by a
  // spinning one.  If some LDU needs more groups than that, the products are
  // swept one after another with cooperative launches instead.
  //
  // Joint mode (the default when it fits): the products advance update by
  // update together and the LDUs of one update form one launch in which
  // every product's groups sit on a single XCD, so every exchange stays in
  // an L2 and no two spinning launches ever wait for each other's CUs.  It
  // needs products of one length, no learned proposal, at most
  // kBatchMaxProducts products, and LDUs that fit one XCD share each at their
  // largest sizes.
  const int cus = prrlu_xcd_cus();
  const int share = 8 * (cus / n_products);
  {
    int off0 = 0;
    bool same_len = true;
    std::vector<int> mm;
    int nmx = 1;
    for (int b = 0; b < n_products; ++b) {
      if (n_inputs[b] < 1 || n_inputs[b] > ACI_MAX_INPUTS) return set_err(ctx, ACI_E_LIMIT, "n_inputs out of range");
      int dmax = 1;
      for (int n = 0; n < n_inputs[b]; ++n)
        for (int l = 0; l < inputs[off0 + n].L && inputs[off0 + n].d; ++l) dmax = std::max(dmax, (int)inputs[off0 + n].d[l]);
      same_len = same_len && inputs[off0].L == inputs[0].L;
      const int mn = std::min(dmax * std::max(1, maxrank), (int)ACI_MAX_MATRIX);
      mm.push_back(mn);
      nmx = std::max(nmx, mn);
      const int g = prrlu_groups(mn, mn, share, dtype == ACI_C128);
      if (share < 1 || g < 0 || g > share) B->serial = true;
      off0 += n_inputs[b];
    }
    const bool joint_ok = n_products <= kBatchMaxProducts && !o.proposal && same_len &&
                          prrlu_batch_variant(mm.data(), n_products, nmx, dtype == ACI_C128) >= 0;
    if (o.batch_mode == 1 && !joint_ok)
      return set_err(ctx, ACI_E_LIMIT, "joint batch needs at most 12 products of one length, no proposal, and LDUs "
                                       "that fit one XCD share each");
    B->joint = joint_ok && o.batch_mode <= 1;
    if (o.batch_mode == 3) B->serial = true;
    if (B->joint) {
      B->serial = false;
      B->jgraph = o.use_graph && !o.profile && !o.trace && op != ACI_OP_CUSTOM;
    }
  }
  aci_options os = o;
  if (B->joint) os.use_graph = 0;   // the batch captures the joint sweep itself
  int off = 0;
  for (int b = 0; b < n_products; ++b) {
    if (n_inputs[b] < 1 || n_inputs[b] > ACI_MAX_INPUTS) return set_err(ctx, ACI_E_LIMIT, "n_inputs out of range");
    int cap = (B->serial || B->joint) ? 0 : share;
    if (o.tune && !B->serial && !B->joint) {
      int dmax = 1;
      for (int n = 0; n < n_inputs[b]; ++n)
        for (int l = 0; l < inputs[off + n].L && inputs[off + n].d; ++l) dmax = std::max(dmax, (int)inputs[off + n].d[l]);
      const int mn = std::min(dmax * std::max(1, maxrank), (int)ACI_MAX_MATRIX);
      int best = cap;
      const int rc = aci_tune_prrlu(ctx, mn, mn, std::min(maxrank, mn), cap, &best, nullptr, nullptr, 0, nullptr);
      if (rc < 0) return rc;
      cap = best;
    }
    hipStream_t st = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    B->streams.push_back(st);
    HIPCHK(hipStreamWaitEvent(st, B->ready, 0));
    aci_ctx* c = nullptr;
    int rc = aci_ctx_create(&c, st);
    if (rc) return set_err(ctx, rc, "context creation");
    c->alloc_fn = ctx->alloc_fn;   // the products' memory comes from the caller's allocator too
    c->free_fn = ctx->free_fn;
    c->alloc_user = ctx->alloc_user;
    // and the exchange waits of the parent (aci_ctx_set_exchange_hooks)
    c->spin_limit = ctx->spin_limit;
    c->poll_xor = ctx->poll_xor;
    c->stall_from = ctx->stall_from;
    c->epoch_launches = ctx->epoch_launches;
    B->ctxs.push_back(c);
    Placement pl;
    pl.xcd = (B->serial || B->joint) ? 0 : -1;
    pl.max_groups = cap;
    pl.cooperative = (B->serial || B->joint) ? 1 : 0;   // plain launches: LDUs of different products overlap
    aci_session* S = nullptr;
    rc = session_create(c, inputs + off, n_inputs[b], dtype, op, tol, maxrank, &os, pl, &S);
    if (rc < 0) return set_err(ctx, rc, std::string("product ") + std::to_string(b) + ": " + c->err);
    // cooperative initialisation LDUs of different products never overlap
    if (pl.cooperative) HIPCHK(hipStreamSynchronize(st));
    B->sess.push_back(S);
    B->groups.push_back(cap);
    off += n_inputs[b];
  }
  if (B->joint) {
    HIPCHK(hipStreamCreateWithFlags(&B->jstream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&B->jdone, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&B->jfork, hipEventDisableTiming));
    for (int b = 0; b < n_products; ++b) {
      hipEvent_t e = nullptr;
      HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      B->pre.push_back(e);
    }
  }
  *out = B.release();
  return ACI_OK;
}

int aci_batch_sweep(aci_batch* B, int32_t nsweeps, aci_sweep_stats* stats) {
  if (!B || !B->parent) return ACI_E_INVALID;
  aci_ctx* ctx = B->parent;
  ctx->err.clear();
  if (nsweeps < 0) return set_err(ctx, ACI_E_INVALID, "nsweeps < 0");
  aci_sweep_stats st{};
  double emax = 0.0;
  for (aci_session* S : B->sess) S->log.clear();
  const int n = (int)B->sess.size();
  std::vector<char> act(n);
  for (int it = 0; it < nsweeps; ++it) {
    bool any = false;
    for (int b = 0; b < n; ++b) {
      aci_session* S = B->sess[b];
      act[b] = !(S->converged && !S->fixed);
      any = any || act[b];
    }
    if (!any) break;
    // enqueue every product's sweep on its own stream, then drain them (in
    // serial mode each product is drained before the next starts)
    if (B->joint) {
      std::vector<int> ids;
      for (int b = 0; b < n; ++b)
        if (act[b]) ids.push_back(b);
      if (const int rc = joint_sweep(B, ids)) return rc;
    } else if (!B->serial) {
      for (int b = 0; b < n; ++b)
        if (act[b]) {
          const int rc = sweep_enqueue(B->sess[b]);
          if (rc) return set_err(ctx, rc, std::string("product ") + std::to_string(b) + ": " + B->ctxs[b]->err);
        }
    }
    emax = 0.0;
    for (int b = 0; b < n; ++b)
      if (act[b]) {
        if (B->serial) {
          const int rc = sweep_enqueue(B->sess[b]);
          if (rc) return set_err(ctx, rc, std::string("product ") + std::to_string(b) + ": " + B->ctxs[b]->err);
        }
        HIPCHK(hipStreamSynchronize(B->streams[b]));
        aci_sweep_stats one{};
        const int rc = sweep_finish(B->sess[b], one);
        if (rc) return set_err(ctx, rc, std::string("product ") + std::to_string(b) + ": " + B->ctxs[b]->err);
        for (int c = 0; c < 3; ++c) {
          st.kernel_ms[c] += one.kernel_ms[c];
          st.launches[c] += one.launches[c];
          st.flops[c] += one.flops[c];
        }
        st.pivots += one.pivots;
        st.last_precision = std::max(st.last_precision, one.last_precision);
      }
    for (int b = 0; b < n; ++b) {
      const aci_session* S = B->sess[b];
      double e = 0.0;
      for (int k = 0; k < S->plan->L - 1; ++k) e = std::max(e, S->h_eps[k]);
      emax = std::max(emax, e);
    }
  }
  bool all = true;
  int sweeps = 0;
  for (aci_session* S : B->sess) {
    all = all && S->converged;
    sweeps = std::max(sweeps, S->sweeps);
  }
  stats_tail(B->sess[0], st);
  st.sweeps_done = sweeps;
  st.converged = all ? 1 : 0;
  st.max_eps = emax;
  if (stats) *stats = st;
  return all ? ACI_OK : ACI_W_NOT_CONVERGED;
}

int aci_batch_result(aci_batch* B, int32_t product, void* out, int64_t out_capacity, aci_result* result) {
  if (!B || !B->parent) return ACI_E_INVALID;
  if (product < 0 || product >= (int)B->sess.size()) return set_err(B->parent, ACI_E_INVALID, "product out of range");
  const int rc = aci_session_result(B->sess[product], out, out_capacity, result);
  if (rc < 0) return set_err(B->parent, rc, B->ctxs[product]->err);
  return rc;
}

int aci_batch_info(aci_batch* B, int32_t product, int32_t* xcd, int32_t* max_groups) {
  if (!B || product < 0 || product >= (int)B->sess.size()) return ACI_E_INVALID;
  // -2: joint launches; -1: groups spread over all XCDs (overlapping
  // products); 0: serial batch
  if (xcd) *xcd = B->joint ? -2 : B->sess[product]->plan->xcd;
  if (max_groups) *max_groups = B->groups[product];
  return ACI_OK;
}

int aci_elementwise_batched(aci_ctx* ctx, const aci_tt* inputs, const int32_t* n_inputs, int32_t n_products,
                            int32_t dtype, int32_t op, double tol, int32_t maxrank, const aci_options* opt,
                            void* const* outs, const int64_t* out_capacity, aci_result* results) {
  if (!ctx) return ACI_E_INVALID;
  if (!outs || !out_capacity || !results) return set_err(ctx, ACI_E_INVALID, "null argument");
  for (int b = 0; b < n_products; ++b) std::memset(&results[b], 0, sizeof(aci_result));
  aci_options o{};
  o.maxiter = 20;
  if (opt) o = *opt;
  if (o.maxiter <= 0) o.maxiter = 20;
  aci_batch* B = nullptr;
  int rc = aci_batch_create(ctx, inputs, n_inputs, n_products, dtype, op, tol, maxrank, &o, &B);
  if (rc < 0) return rc;
  if (o.precision != ACI_PREC_FP64 && o.maxiter > 1) {
    rc = aci_batch_sweep(B, o.maxiter - 1, nullptr);
    if (rc >= 0) {
      // the last allowed sweep is FP64 for every product not yet converged
      for (aci_session* S : B->sess) S->plan->prec = PREC_FP64;
      rc = aci_batch_sweep(B, 1, nullptr);
    }
  } else {
    for (aci_session* S : B->sess) S->plan->prec = PREC_FP64;
    rc = aci_batch_sweep(B, o.maxiter, nullptr);
  }
  int worst = rc;
  for (int b = 0; b < n_products && rc >= 0; ++b) {
    const int r = aci_batch_result(B, b, outs[b], out_capacity[b], &results[b]);
    if (r < 0) {
      rc = r;
      break;
    }
    worst = std::max(worst, r);
  }
  aci_batch_destroy(B);
  return rc < 0 ? rc : worst;
}

// ------------------------------------------------------------ learned proposal
extern "C++" {
namespace {
template <typename T>
int grow(aci_ctx* ctx, T*& buf, size_t& have, size_t need, const char* what) {
  if (have >= need) return ACI_OK;
  if (buf) {
    (void)hipStreamSynchronize(ctx->stream);
    dev_free(ctx, buf);
  }
  buf = nullptr;
  have = 0;
  void* p = nullptr;
  if (!dev_alloc(ctx, &p, need * sizeof(T))) return set_err(ctx, ACI_E_NOMEM, what);
  buf = (T*)p;
  have = need;
  return ACI_OK;
}
}  // namespace
}  // extern "C++"

int aci_proposal_features(aci_ctx* ctx, const void* M, int32_t m, int32_t n, int32_t ldm, const void* const* env,
                          const int32_t* env_w, const int32_t* env_ld, int32_t n_env, const int32_t* prev_rows,
                          int32_t n_prev, float* X) {
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  if (!M || !X || m < 1 || n < 1 || ldm < n || n_env < 0 || n_env > 2 || n_prev < 0 || (n_prev > 0 && !prev_rows))
    return set_err(ctx, ACI_E_INVALID, "bad arguments");
  if (m > ACI_MAX_MATRIX || n > ACI_MAX_MATRIX) return set_err(ctx, ACI_E_LIMIT, "matrix too large");
  int rc = ensure_step_ws(ctx);
  if (rc) return rc;
  FeatureArgs a{};
  a.M = (const double*)M;
  a.m = dconst(m);
  a.n = dconst(n);
  a.ldm = dconst(ldm);
  a.n_env = n_env;
  for (int t = 0; t < n_env; ++t) {
    if (!env || !env[t] || !env_w || !env_ld || env_w[t] < 1 || env_ld[t] < env_w[t])
      return set_err(ctx, ACI_E_INVALID, "bad environment");
    a.env[t] = (const double*)env[t];
    a.env_w[t] = dconst(env_w[t]);
    a.env_ld[t] = dconst(env_ld[t]);
  }
  a.prev_rows = prev_rows;
  HIPCHK(hipMemcpyAsync(ctx->step_err + 2, &n_prev, sizeof(int), hipMemcpyHostToDevice, ctx->stream));
  a.prev_rank = ctx->step_err + 2;
  a.X = X;
  HIPCHK(launch_features(a, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return ACI_OK;
}

int aci_mlp_init(aci_ctx* ctx, uint64_t seed, float* params) {
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  if (!params) return set_err(ctx, ACI_E_INVALID, "null params");
  // W1 (7 x 64), W2 (64 x 64), w3 (64) in this order from one stream, each
  // entry u sqrt(6 / fan_in) with u uniform on [-1, 1); biases zero
  std::vector<float> h(ACI_MLP_PARAMS, 0.f);
  SplitMix64 rng{seed};
  const int H = ACI_MLP_HIDDEN, F = ACI_MLP_FEATURES;
  const size_t oW1 = 0, oW2 = (size_t)F * H + H, ow3 = oW2 + (size_t)H * H + H;
  const double s1 = std::sqrt(6.0 / F), s2 = std::sqrt(6.0 / H);
  for (int i = 0; i < F * H; ++i) h[oW1 + i] = (float)(rng.uniform() * s1);
  for (int i = 0; i < H * H; ++i) h[oW2 + i] = (float)(rng.uniform() * s2);
  for (int i = 0; i < H; ++i) h[ow3 + i] = (float)(rng.uniform() * s2);
  HIPCHK(hipMemcpyAsync(params, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return ACI_OK;
}

int aci_proposal_dataset(aci_ctx* ctx, const aci_tt* inputs, int32_t n_inputs, int32_t op, double tol,
                         int32_t maxrank, const aci_options* opt, float* X, float* y, int64_t capacity,
                         int64_t* count, int32_t* sweeps) {
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  if (!X || !y || !count) return set_err(ctx, ACI_E_INVALID, "null argument");
  if (capacity < 0) return set_err(ctx, ACI_E_INVALID, "capacity < 0");
  *count = 0;
  if (sweeps) *sweeps = 0;
  aci_options o{};
  o.maxiter = 20;
  if (opt) o = *opt;
  if (o.maxiter <= 0) o.maxiter = 20;
  if (o.proposal) return set_err(ctx, ACI_E_INVALID, "the dataset records the full search: options.proposal must be NULL");
  if (o.precision != ACI_PREC_FP64) return set_err(ctx, ACI_E_INVALID, "the dataset records plain FP64 sweeps");
  o.use_graph = 0;
  RecordSpec rs;
  rs.X = X;
  rs.y = y;
  rs.capacity = capacity;
  aci_session* S = nullptr;
  int rc = session_create(ctx, inputs, n_inputs, ACI_F64, op, tol, maxrank, &o, Placement{}, &S, &rs);
  if (rc < 0) return rc;
  rc = aci_session_sweep(S, o.maxiter, nullptr);
  long long cnt[2] = {0, 0};
  if (rc >= 0) {
    const hipError_t e1 = hipMemcpyAsync(cnt, S->plan->rec_count, sizeof cnt, hipMemcpyDeviceToHost, ctx->stream);
    const hipError_t e2 = e1 == hipSuccess ? hipStreamSynchronize(ctx->stream) : e1;
    if (e2 != hipSuccess) rc = set_err(ctx, ACI_E_HIP, std::string("dataset count: ") + hipGetErrorString(e2));
  }
  if (sweeps) *sweeps = S->sweeps;
  aci_session_destroy(S);
  if (rc < 0) return rc;
  *count = cnt[0];
  if (cnt[1]) return set_err(ctx, ACI_E_NOMEM, "dataset capacity reached; count holds the rows of the updates that fit");
  return rc;
}

int aci_mlp_forward(aci_ctx* ctx, const float* params, const float* X, int32_t count, float* scores) {
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  if (!params || !X || !scores || count < 0) return set_err(ctx, ACI_E_INVALID, "bad arguments");
  HIPCHK(launch_mlp_forward(params, X, count, scores, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return ACI_OK;
}

int aci_mlp_train_step(aci_ctx* ctx, float* params, float* adam_m, float* adam_v, int32_t step, const float* X,
                       const float* y, int32_t count, float lr, float* grads, float* loss) {
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  if (!params || !adam_m || !adam_v || !X || !y || count < 1 || step < 1) return set_err(ctx, ACI_E_INVALID, "bad arguments");
  if (count > ACI_MAX_MLP_BATCH) return set_err(ctx, ACI_E_LIMIT, "minibatch too large");
  int rc = grow(ctx, ctx->mlp_scratch, ctx->mlp_scratch_n, (size_t)(6 * MLP_HIDDEN + 1) * count + 64, "network scratch");
  if (rc) return rc;
  rc = ensure_step_ws(ctx);
  if (rc) return rc;
  const double b1 = 0.9, b2 = 0.999;
  TrainArgs a{};
  a.params = params;
  a.adam_m = adam_m;
  a.adam_v = adam_v;
  a.X = X;
  a.y = y;
  a.count = count;
  a.lr = lr;
  a.beta1 = (float)b1;
  a.beta2 = (float)b2;
  a.one_minus_beta1 = (float)(1.0 - b1);
  a.one_minus_beta2 = (float)(1.0 - b2);
  a.c1 = (float)(1.0 - std::pow(b1, (double)step));
  a.c2 = (float)(1.0 - std::pow(b2, (double)step));
  a.eps = 1e-8f;
  a.scratch = ctx->mlp_scratch;
  a.grads = grads;
  float* dloss = (float*)(ctx->step_err + 3);
  a.loss = dloss;
  HIPCHK(launch_mlp_train(a, ctx->stream));
  float lh = 0.f;
  HIPCHK(hipMemcpyAsync(&lh, dloss, sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (loss) *loss = lh;
  return ACI_OK;
}

int aci_rook_lu(aci_ctx* ctx, const void* M, int32_t m, int32_t n, int32_t ldm, double tol, int32_t maxrank,
                const float* scores, int32_t max_iter, int32_t* rows, int32_t* cols, int32_t* rank, double* eps,
                void* L, int32_t ldl, void* Up, int32_t ldu, int32_t* scans) {
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  if (!M || !rows || !cols || !rank || !eps || !L || !Up || m < 1 || n < 1 || ldm < n || maxrank < 1 ||
      ldl < maxrank || ldu < n || max_iter < 1 || !(tol >= 0.0))
    return set_err(ctx, ACI_E_INVALID, "bad arguments");
  if (m > ACI_MAX_MATRIX || n > ACI_MAX_MATRIX) return set_err(ctx, ACI_E_LIMIT, "matrix too large");
  RookArgs a{};
  a.M = (const double*)M;
  a.m = dconst(m);
  a.n = dconst(n);
  a.ldm = dconst(ldm);
  a.tol = tol;
  a.maxrank = maxrank;
  a.max_iter = max_iter;
  a.scores = scores;
  a.L = (double*)L;
  a.ldl = ldl;
  a.Up = (double*)Up;
  a.ldu = ldu;
  a.rows = rows;
  a.cols = cols;
  a.rank = rank;
  a.eps = eps;
  a.scans = scans;
  HIPCHK(launch_rook(a, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return ACI_OK;
}

int aci_rook_check(aci_ctx* ctx, const void* M, int32_t m, int32_t n, int32_t ldm, const void* L, int32_t ldl,
                   const void* Up, int32_t ldu, const int32_t* rank, double tol, double* eps, int32_t* accepted) {
  // the kernel writes the flag and its negation: stage them in the step workspace
  int32_t* flags2 = nullptr;
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  if (!M || !L || !Up || !rank || !eps || !accepted || m < 1 || n < 1 || ldm < n || ldu < n || ldl < 1)
    return set_err(ctx, ACI_E_INVALID, "bad arguments");
  int rc = grow(ctx, ctx->check_c, ctx->check_c_n, (size_t)m * n, "check workspace");
  if (rc) return rc;
  ContractArgs c{};
  c.ngroup = 1;
  Group& g = c.g[0];
  g.nterm = 1;
  g.t[0] = Term{(const double*)L, (const double*)Up, Dim{rank, 1, 0}, dconst(ldl), dconst(ldu)};
  g.C = ctx->check_c;
  g.M = dconst(m);
  g.N = dconst(n);
  g.ldc = dconst(n);
  HIPCHK(launch_contract(OP_NONE, PREC_FP64, c, m, n, ctx->stream));
  CheckArgs a{};
  a.M = (const double*)M;
  a.m = dconst(m);
  a.n = dconst(n);
  a.ldm = dconst(ldm);
  a.C = ctx->check_c;
  a.ldc = n;
  a.tol = tol;
  a.eps = eps;
  rc = ensure_step_ws(ctx);
  if (rc) return rc;
  flags2 = ctx->step_err + 2;
  a.accepted = flags2;
  HIPCHK(launch_check(a, ctx->stream));
  HIPCHK(hipMemcpyAsync(accepted, flags2, sizeof(int32_t), hipMemcpyDeviceToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return ACI_OK;
}

int aci_rook_right_factor(aci_ctx* ctx, const void* Up, int32_t ldu, const int32_t* cols, const int32_t* rank,
                          int32_t n, void* Y, int32_t ldy) {
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  if (!Up || !cols || !rank || !Y || n < 1 || ldu < n || ldy < n) return set_err(ctx, ACI_E_INVALID, "bad arguments");
  SolveArgs a{};
  a.Up = (const double*)Up;
  a.ldu = ldu;
  a.cols = cols;
  a.rank = rank;
  a.n = dconst(n);
  a.Y = (double*)Y;
  a.ldy = dconst(ldy);
  HIPCHK(launch_rook_solve(a, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return ACI_OK;
}

// ------------------------------------------------------------ autotuner
int aci_tune_contract(aci_ctx* ctx, int32_t dtype, int32_t precision, int32_t ngroup, int32_t m, int32_t k,
                      int32_t n, int32_t* best_tile, float* us) {
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  if (!best_tile) return set_err(ctx, ACI_E_INVALID, "null argument");
  if (dtype != ACI_F64 && dtype != ACI_C128) return set_err(ctx, ACI_E_DTYPE, "unknown dtype");
  if (precision < ACI_PREC_FP64 || precision > ACI_PREC_BF16X3) return set_err(ctx, ACI_E_DTYPE, "unknown precision");
  return tune_tile(ctx, dtype == ACI_C128, precision, ngroup, m, k, n, best_tile, us);
}

int aci_tune_prrlu(aci_ctx* ctx, int32_t m, int32_t n, int32_t maxrank, int32_t cap, int32_t* best_groups,
                   int32_t* candidates, float* us, int32_t capacity, int32_t* count) {
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  if (!best_groups) return set_err(ctx, ACI_E_INVALID, "null argument");
  if (m < 1 || n < 1 || m > ACI_MAX_MATRIX || n > ACI_MAX_MATRIX || maxrank < 1) return set_err(ctx, ACI_E_LIMIT, "shape out of range");
  if (cap < 1) cap = prrlu_xcd_cus();
  const uint64_t key = ((uint64_t)m << 40) | ((uint64_t)n << 24) | ((uint64_t)maxrank << 8) | (uint64_t)std::min(cap, 255);
  auto hit = ctx->tuned.find(key);
  if (hit != ctx->tuned.end() && !candidates && !us) {
    *best_groups = hit->second;
    return ACI_OK;
  }
  // candidate caps: cap, then halving; each distinct P (group count) once
  std::vector<int> cand;
  for (int c = cap; c >= 1; c /= 2) {
    const int v = prrlu_variant(m, n, c);
    bool dup = false;
    for (int x : cand) dup = dup || prrlu_variant(m, n, x) == v;
    if (!dup) cand.push_back(c);
  }
  int rc = ensure_step_ws(ctx);
  if (rc) return rc;
  const size_t bytes = ((size_t)m * n + 8) * sizeof(double) + ((size_t)2 * ACI_MAX_MATRIX + 16) * sizeof(int);
  void* ws = nullptr;
  if (!dev_alloc(ctx, &ws, bytes)) return set_err(ctx, ACI_E_NOMEM, "tuning workspace");
  double* M = (double*)ws;
  double* ep = M + (size_t)m * n;
  int* rows = (int*)(ep + 8);
  int* cols = rows + ACI_MAX_MATRIX;
  int* rk = cols + ACI_MAX_MATRIX;
  std::vector<double> h((size_t)m * n);
  SplitMix64 rng{0x5eedull + (uint64_t)m * 7919u + (uint64_t)n};
  for (double& x : h) x = rng.uniform();
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int best = cand.empty() ? 1 : cand[0];
  float best_us = 1e30f;
  int k = 0;
  auto cleanup = [&]() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(ctx->stream);
    dev_free(ctx, ws);
  };
  if (hipMemcpy(M, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return set_err(ctx, ACI_E_HIP, "tuning setup");
  }
  for (int c : cand) {
    float tot = 0.f;
    for (int rep = 0; rep < 3; ++rep) {
      PrrluArgs a{};
      a.M = M;
      a.m = dconst(m);
      a.n = dconst(n);
      a.ldm = dconst(n);
      a.tol = 0.0;
      a.maxrank = std::min(maxrank, std::min(m, n));
      a.rule = RULE_EXCLUSIVE;
      exchange_waits(ctx, a);
      a.xbuf = ctx->step_xbuf;
      a.xbuf_words = ctx->step_xwords;
      a.rows = rows;
      a.cols = cols;
      a.rank = rk;
      a.eps = ep;
      a.err = ctx->step_err;
      a.abort_word = ctx->step_err + 1;
      a.max_groups = c;
      a.cooperative = 1;
      hipError_t e = step_flag(ctx, &a.flag_base);
      if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
      if (e == hipSuccess) e = launch_fill_int(ctx->step_err, 2, 0, ctx->stream);
      if (e == hipSuccess) e = launch_prrlu(a, m, n, ctx->stream);
      if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        cleanup();
        return set_err(ctx, ACI_E_HIP, std::string("tuning run: ") + hipGetErrorString(e));
      }
      if (rep > 0) tot += ms;   // the first run warms up
    }
    const float t = 1e3f * tot / 2.f;
    if (candidates && k < capacity) candidates[k] = c;
    if (us && k < capacity) us[k] = t;
    ++k;
    if (t < best_us) {
      best_us = t;
      best = c;
    }
  }
  int fl[2] = {0, 0};
  (void)hipMemcpy(fl, ctx->step_err, sizeof(fl), hipMemcpyDeviceToHost);
  cleanup();
  if (fl[0] & ERR_TIMEOUT) return set_err(ctx, ACI_E_TIMEOUT, "a pivot exchange exceeded its spin limit");
  if (count) *count = k;
  ctx->tuned[key] = best;
  *best_groups = best;
  return ACI_OK;
}

// ------------------------------------------------------------ single steps
static int ensure_step_ws(aci_ctx* ctx) {
  if (!ctx->step_err) {
    void* p = nullptr;
    if (!dev_alloc(ctx, &p, 4 * sizeof(int))) return set_err(ctx, ACI_E_NOMEM, "step workspace");
    ctx->step_err = (int*)p;
  }
  const size_t words = prrlu_xbuf_words(ACI_MAX_MATRIX, ACI_MAX_MATRIX, 1);
  if (ctx->step_xwords < words) {
    if (ctx->step_xbuf) {
      (void)hipStreamSynchronize(ctx->stream);
      dev_free(ctx, ctx->step_xbuf);
    }
    ctx->step_xbuf = nullptr;
    void* p = nullptr;
    if (!dev_alloc(ctx, &p, words * sizeof(uint64_t))) return set_err(ctx, ACI_E_NOMEM, "step exchange buffer");
    ctx->step_xbuf = (uint64_t*)p;
    ctx->step_xwords = words;
    // recycled memory may hold words whose flags a launch of this context
    // will use (flags restart at 1 in every context): clear it, as the
    // sessions clear theirs
    HIPCHK(launch_fill_int((int*)ctx->step_xbuf, (int)(2 * words), 0, ctx->stream));
    ctx->step_flags_wrapped = false;
  }
  return ACI_OK;
}

int aci_env_contract(aci_ctx* ctx, int32_t dtype, int32_t side, int32_t count, const void* const* frames,
                     const void* const* cores, void* const* outp, int32_t c, int32_t r0, int32_t d, int32_t r1,
                     int32_t precision) {
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  if (dtype != ACI_F64 && dtype != ACI_C128) return set_err(ctx, ACI_E_DTYPE, "unknown dtype");
  if (precision < ACI_PREC_FP64 || precision > ACI_PREC_BF16X3) return set_err(ctx, ACI_E_DTYPE, "unknown precision");
  if (count < 1 || count > ACI_MAX_INPUTS || !frames || !cores || !outp) return set_err(ctx, ACI_E_INVALID, "bad count or null");
  if (c < 1 || r0 < 1 || d < 1 || r1 < 1) return set_err(ctx, ACI_E_INVALID, "bad dims");
  ContractArgs a{};
  a.cplx = dtype == ACI_C128 ? 1 : 0;
  a.ngroup = count;
  int mmax, nmax;
  for (int i = 0; i < count; ++i) {
    if (!frames[i] || !cores[i] || !outp[i]) return set_err(ctx, ACI_E_INVALID, "null pointer");
    Group& g = a.g[i];
    g.nterm = 1;
    g.C = (double*)outp[i];
    if (side == 0) {
      g.t[0] = Term{(const double*)frames[i], (const double*)cores[i], dconst(r0), dconst(r0), dconst(d * r1)};
      g.M = dconst(c);
      g.N = dconst(d * r1);
      g.ldc = dconst(d * r1);
    } else {
      g.t[0] = Term{(const double*)cores[i], (const double*)frames[i], dconst(r1), dconst(r1), dconst(c)};
      g.M = dconst(r0 * d);
      g.N = dconst(c);
      g.ldc = dconst(c);
    }
  }
  if (side == 0) { mmax = c; nmax = d * r1; } else { mmax = r0 * d; nmax = c; }
  HIPCHK(launch_contract(OP_NONE, precision, a, mmax, nmax, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return ACI_OK;
}

int aci_pi_eval(aci_ctx* ctx, int32_t dtype, int32_t op, int32_t n_inputs, const void* const* A,
                const void* const* B, const int32_t* k, int32_t m, int32_t n, void* M, int32_t ldm,
                int32_t precision, int32_t tile) {
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  if (dtype != ACI_F64 && dtype != ACI_C128) return set_err(ctx, ACI_E_DTYPE, "unknown dtype");
  if (precision < ACI_PREC_FP64 || precision > ACI_PREC_BF16X3) return set_err(ctx, ACI_E_DTYPE, "unknown precision");
  if (n_inputs < 1 || n_inputs > ACI_MAX_INPUTS || !A || !B || !k || !M) return set_err(ctx, ACI_E_INVALID, "bad arguments");
  if (op == ACI_OP_ABS2_MUL && n_inputs != 1) return set_err(ctx, ACI_E_INVALID, "ABS2_MUL takes one input");
  if (op != ACI_OP_PRODUCT && op != ACI_OP_SUM && op != ACI_OP_ABS2_MUL) return set_err(ctx, ACI_E_INVALID, "op");
  if (m < 1 || n < 1 || ldm < n) return set_err(ctx, ACI_E_INVALID, "bad dims");
  ContractArgs a{};
  a.cplx = dtype == ACI_C128 ? 1 : 0;
  a.ngroup = 1;
  a.err = ctx->step_err;
  int rc = ensure_step_ws(ctx);
  if (rc) return rc;
  a.err = ctx->step_err;
  HIPCHK(launch_fill_int(ctx->step_err, 2, 0, ctx->stream));
  Group& g = a.g[0];
  g.nterm = n_inputs;
  for (int i = 0; i < n_inputs; ++i) {
    if (!A[i] || !B[i] || k[i] < 1) return set_err(ctx, ACI_E_INVALID, "bad term");
    g.t[i] = Term{(const double*)A[i], (const double*)B[i], dconst(k[i]), dconst(k[i]), dconst(n)};
  }
  g.C = (double*)M;
  g.M = dconst(m);
  g.N = dconst(n);
  g.ldc = dconst(ldm);
  if (tile < -1 || tile >= NUM_TILES) return set_err(ctx, ACI_E_INVALID, "tile must be -1, 0, 1 or 2");
  HIPCHK(launch_contract(op, precision, a, m, n, ctx->stream, tile));
  int flags = 0;
  HIPCHK(hipMemcpyAsync(&flags, ctx->step_err, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (flags & ERR_NONFINITE) return set_err(ctx, ACI_E_NUMERIC, "NaN or Inf in the two-site tensor");
  return ACI_OK;
}

int aci_prrlu(aci_ctx* ctx, int32_t dtype, const void* M, int32_t m, int32_t n, int32_t ldm, double tol,
              int32_t maxrank, int32_t stop_rule, int32_t* rows, int32_t* cols, int32_t* rank, double* eps,
              void* Y, int32_t ldy) {
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  if (dtype != ACI_F64 && dtype != ACI_C128) return set_err(ctx, ACI_E_DTYPE, "unknown dtype");
  if (!M || !rows || !cols || !rank || !eps) return set_err(ctx, ACI_E_INVALID, "null pointer");
  if (m < 1 || n < 1 || ldm < n || maxrank < 1 || !(tol >= 0.0)) return set_err(ctx, ACI_E_INVALID, "bad dims or tolerance");
  if (m > ACI_MAX_MATRIX || n > ACI_MAX_MATRIX) return set_err(ctx, ACI_E_LIMIT, "matrix above ACI_MAX_MATRIX");
  if (stop_rule != 0 && stop_rule != 1) return set_err(ctx, ACI_E_INVALID, "stop_rule");
  if (Y && ldy < n) return set_err(ctx, ACI_E_INVALID, "ldy < n");
  int rc = ensure_step_ws(ctx);
  if (rc) return rc;
  HIPCHK(launch_fill_int(ctx->step_err, 2, 0, ctx->stream));
  PrrluArgs a{};
  a.M = (const double*)M;
  a.cplx = dtype == ACI_C128 ? 1 : 0;
  a.m = dconst(m);
  a.n = dconst(n);
  a.ldm = dconst(ldm);
  a.tol = tol;
  a.maxrank = maxrank;
  a.rule = stop_rule;
  HIPCHK(step_flag(ctx, &a.flag_base));
  a.cooperative = 1;
  exchange_waits(ctx, a);
  a.xbuf = ctx->step_xbuf;
  a.xbuf_words = ctx->step_xwords;
  a.rows = rows;
  a.cols = cols;
  a.rank = rank;
  a.eps = eps;
  a.Y = (double*)Y;
  a.ldy = dconst(ldy);
  a.err = ctx->step_err;
  a.abort_word = ctx->step_err + 1;
  HIPCHK(launch_prrlu(a, m, n, ctx->stream));
  int flags = 0;
  HIPCHK(hipMemcpyAsync(&flags, ctx->step_err, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (flags & ERR_TIMEOUT) return set_err(ctx, ACI_E_TIMEOUT, "pivot exchange timed out");
  return ACI_OK;
}

}  // extern "C"

// ---- LDU without allocation
// Fixed device workspace of aci_prrlu_noalloc: kNoAllocFlagWords words for
// the error and abort words, then the exchange words of one factorisation.
// The exchange size covers every real matrix up to ACI_MAX_MATRIX x
// ACI_MAX_MATRIX (64 groups of 1024-column rows) and complex matrices up to
// 512 columns; larger exchanges are refused.  Every GPU holds its own copy
// until the process ends.
namespace {
constexpr size_t kNoAllocFlagWords = 32;   // keeps the exchange 256-byte aligned
constexpr size_t kNoAllocXWords = (size_t)2 * 64 * (4 + 2 * 64 * 16);
constexpr size_t kNoAllocWords = kNoAllocFlagWords + kNoAllocXWords;
}  // namespace
static __device__ __align__(256) uint64_t scratch[kNoAllocWords];

namespace {
constexpr int kNoAllocMaxDevices = 64;
std::mutex g_noalloc_mu;
uint64_t* g_noalloc_ptr[kNoAllocMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (in host code the symbol's name is not a device address).
int noalloc_scratch(aci_ctx* ctx, uint64_t** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocMaxDevices) return set_err(ctx, ACI_E_LIMIT, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return set_err(ctx, ACI_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_noalloc_ptr[dev] = (uint64_t*)p;
  }
  *out = g_noalloc_ptr[dev];
  return ACI_OK;
}
}  // namespace

extern "C" {

int aci_prrlu_noalloc(aci_ctx* ctx, int32_t dtype, const void* M, int32_t m, int32_t n, int32_t ldm, double tol,
                      int32_t maxrank, int32_t stop_rule, int32_t* rows, int32_t* cols, int32_t* rank, double* eps,
                      void* Y, int32_t ldy) {
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  if (dtype != ACI_F64 && dtype != ACI_C128) return set_err(ctx, ACI_E_DTYPE, "unknown dtype");
  if (!M || !rows || !cols || !rank || !eps) return set_err(ctx, ACI_E_INVALID, "null pointer");
  if (m < 1 || n < 1 || ldm < n || maxrank < 1 || !(tol >= 0.0)) return set_err(ctx, ACI_E_INVALID, "bad dims or tolerance");
  if (m > ACI_MAX_MATRIX || n > ACI_MAX_MATRIX) return set_err(ctx, ACI_E_LIMIT, "matrix above ACI_MAX_MATRIX");
  if (stop_rule != 0 && stop_rule != 1) return set_err(ctx, ACI_E_INVALID, "stop_rule");
  if (Y && ldy < n) return set_err(ctx, ACI_E_INVALID, "ldy < n");
  const int cplx = dtype == ACI_C128 ? 1 : 0;
  const size_t used = prrlu_xbuf_used(m, n, 0, cplx);
  if (used == 0) return set_err(ctx, ACI_E_LIMIT, "no LDU shape for these dimensions");
  if (used > kNoAllocXWords)
    return set_err(ctx, ACI_E_LIMIT, "exchange of " + std::to_string(used) + " words exceeds the static scratch of " +
                                         std::to_string(kNoAllocXWords) + " (complex matrices above 512 columns)");
  uint64_t* ws = nullptr;
  if (int rc = noalloc_scratch(ctx, &ws)) return rc;
  int* err = (int*)ws;
  // The scratch keeps the previous call's words: clear the flags and the
  // exchange words this launch uses, so that its step flags (from 1) match
  // nothing stale.
  HIPCHK(launch_fill_int((int*)ws, 2 * (kNoAllocFlagWords + used), 0, ctx->stream));
  PrrluArgs a{};
  a.M = (const double*)M;
  a.cplx = cplx;
  a.m = dconst(m);
  a.n = dconst(n);
  a.ldm = dconst(ldm);
  a.tol = tol;
  a.maxrank = maxrank;
  a.rule = stop_rule;
  a.flag_base = 1;
  a.cooperative = 1;
  exchange_waits(ctx, a);
  a.xbuf = ws + kNoAllocFlagWords;
  a.xbuf_words = used;
  a.rows = rows;
  a.cols = cols;
  a.rank = rank;
  a.eps = eps;
  a.Y = (double*)Y;
  a.ldy = dconst(ldy);
  a.err = err;
  a.abort_word = err + 1;
  HIPCHK(launch_prrlu(a, m, n, ctx->stream));
  int flags = 0;
  HIPCHK(hipMemcpyAsync(&flags, err, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (flags & ERR_TIMEOUT) return set_err(ctx, ACI_E_TIMEOUT, "pivot exchange timed out");
  return ACI_OK;
}

int aci_gather(aci_ctx* ctx, int32_t dtype, int32_t side, const void* src, int32_t h, int32_t w, int32_t ld_src,
               const int32_t* idx, const int32_t* rank, void* out, int32_t ld_out) {
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  if (dtype != ACI_F64 && dtype != ACI_C128) return set_err(ctx, ACI_E_DTYPE, "unknown dtype");
  if (!src || !idx || !rank || !out) return set_err(ctx, ACI_E_INVALID, "null pointer");
  if (h < 1 || w < 1 || ld_src < w || ld_out < 1 || (side != 0 && side != 1)) return set_err(ctx, ACI_E_INVALID, "bad dims");
  GatherArgs a{};
  a.esz = dtype == ACI_C128 ? 2 : 1;
  a.count = 1;
  a.side = side;
  a.idx = idx;
  a.rank = rank;
  a.it[0] = GatherItem{(const double*)src, (double*)out, dconst(ld_src), dconst(ld_out), dconst(side == 0 ? w : h),
                       dconst(side == 0 ? h : w)};
  int rc = ensure_step_ws(ctx);
  if (rc) return rc;
  HIPCHK(launch_fill_int(ctx->step_err, 2, 0, ctx->stream));
  a.err = ctx->step_err;
  HIPCHK(launch_gather(a, side == 0 ? h : w, side == 0 ? w : h, ctx->stream));
  int flags = 0;
  HIPCHK(hipMemcpyAsync(&flags, ctx->step_err, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (flags & ERR_LIMIT) return set_err(ctx, ACI_E_INVALID, "gather index out of range");
  return ACI_OK;
}

// ------------------------------------------------ TT operators, time step
int aci_mpo_stencil(int32_t R, int32_t ndim, int32_t axis, const double* weights, double* cores,
                    int32_t* ranks) {
  if (R < 1 || ndim < 1 || axis < 0 || axis >= ndim || !weights || !cores || !ranks) return ACI_E_INVALID;
  if ((long long)R * ndim > ACI_MAX_SITES) return ACI_E_LIMIT;
  const int L = R * ndim;
  for (int l = 0; l <= L; ++l) ranks[l] = (l == 0 || l == L) ? 1 : 3;
  // bond state k = carry + 1; the right bond of a site holds the carry coming
  // from the less significant bits, the left bond the carry going on
  for (int l = 0; l < L; ++l) {
    double* W = cores + 36 * l;
    std::fill(W, W + 36, 0.0);
    const int wb = ranks[l + 1];
    for (int kin = 0; kin < 3; ++kin)
      for (int sb = 0; sb < 2; ++sb) {
        int tb = sb, kout = kin;
        if (l % ndim == axis) {
          const int v = sb + kin - 1;               // output bit plus carry, in [-1, 2]
          tb = (v + 2) & 1;
          kout = (v < 0 ? -1 : v / 2) + 1;
        }
        // left end: the carry out of the top bit is dropped (all states
        // summed); right end: the carry into the lowest bit is delta,
        // weighted by w_delta
        const int ia = l == 0 ? 0 : kout;
        const int ib = l == L - 1 ? 0 : kin;
        const double wt = l == L - 1 ? weights[kin] : 1.0;
        W[((ia * 2 + sb) * 2 + tb) * wb + ib] += wt;
      }
  }
  return ACI_OK;
}

}  // extern "C"

namespace {

// Enqueues Z_l = W_l X_l for every site (real operator; ew doubles per TT
// element).  The caller has validated the shapes.
int enqueue_mpo_apply(aci_ctx* ctx, int L, const int32_t* d, const int32_t* w, const double* const* Wc,
                      const int32_t* r, const void* const* X, void* const* Z, int ew) {
  for (int l0 = 0; l0 < L; l0 += kMpoSitesPerLaunch) {
    MpoArgs a{};
    int blocks = 0;
    for (int l = l0; l < std::min(L, l0 + kMpoSitesPerLaunch); ++l) {
      MpoSite& m = a.site[a.nsite++];
      m.W = Wc[l];
      m.X = (const double*)X[l];
      m.Z = (double*)Z[l];
      m.wa = w[l];
      m.wb = w[l + 1];
      m.ra = r[l];
      m.xe = ew * r[l + 1];
      m.d = d[l];
      m.vec = (m.xe % 2 == 0 && (uintptr_t)m.X % 16 == 0 && (uintptr_t)m.Z % 16 == 0) ? 1 : 0;
      m.block0 = blocks;
      blocks += mpo_site_blocks(m);
    }
    HIPCHK(launch_mpo_apply(a, blocks, ctx->stream));
  }
  return ACI_OK;
}

int validate_mpo_apply(aci_ctx* ctx, const aci_mpo* W, const aci_tt* x, int32_t dtype) {
  if (!W || !x || !W->d || !W->ranks || !W->cores) return set_err(ctx, ACI_E_INVALID, "null pointer");
  if (dtype != ACI_F64 && dtype != ACI_C128) return set_err(ctx, ACI_E_DTYPE, "unknown dtype");
  const int L = W->L;
  if (L < 1 || L > ACI_MAX_SITES) return set_err(ctx, ACI_E_LIMIT, "L out of range");
  if (x->L != L || !x->d || !x->ranks || !x->cores) return set_err(ctx, ACI_E_INVALID, "TT and operator differ in length");
  if (W->ranks[0] != 1 || W->ranks[L] != 1 || x->ranks[0] != 1 || x->ranks[L] != 1)
    return set_err(ctx, ACI_E_INVALID, "boundary ranks must be 1");
  const int ew = dtype == ACI_C128 ? 2 : 1;
  for (int l = 0; l < L; ++l) {
    if (W->d[l] != x->d[l]) return set_err(ctx, ACI_E_INVALID, "local dimensions differ");
    if (x->d[l] < 1 || x->d[l] > ACI_MAX_DIM) return set_err(ctx, ACI_E_LIMIT, "local dimension out of range");
    if (W->ranks[l + 1] < 1 || x->ranks[l + 1] < 1) return set_err(ctx, ACI_E_INVALID, "ranks must be >= 1");
    if (!W->cores[l] || !x->cores[l]) return set_err(ctx, ACI_E_INVALID, "null core pointer");
    const long long elems =
        (long long)W->ranks[l] * x->ranks[l] * x->d[l] * W->ranks[l + 1] * x->ranks[l + 1] * ew;
    if (elems > 0x7fffffffLL) return set_err(ctx, ACI_E_LIMIT, "output core too large");
  }
  return ACI_OK;
}

}  // namespace

extern "C" {

int aci_mpo_apply(aci_ctx* ctx, const aci_mpo* W, const aci_tt* x, int32_t dtype, void* const* out,
                  float* kernel_ms) {
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  int rc = validate_mpo_apply(ctx, W, x, dtype);
  if (rc) return rc;
  if (!out) return set_err(ctx, ACI_E_INVALID, "null output");
  for (int l = 0; l < W->L; ++l)
    if (!out[l]) return set_err(ctx, ACI_E_INVALID, "null output core");
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (kernel_ms) {
    HIPCHK(hipEventCreate(&ev[0]));
    if (hipEventCreate(&ev[1]) != hipSuccess) {
      (void)hipEventDestroy(ev[0]);
      return set_err(ctx, ACI_E_HIP, "hipEventCreate");
    }
    (void)hipEventRecord(ev[0], ctx->stream);
  }
  rc = enqueue_mpo_apply(ctx, W->L, W->d, W->ranks, W->cores, x->ranks, x->cores, out, dtype == ACI_C128 ? 2 : 1);
  if (kernel_ms && rc == ACI_OK) (void)hipEventRecord(ev[1], ctx->stream);
  const hipError_t se = hipStreamSynchronize(ctx->stream);
  if (kernel_ms) {
    if (rc == ACI_OK && se == hipSuccess && hipEventElapsedTime(kernel_ms, ev[0], ev[1]) != hipSuccess) *kernel_ms = -1.f;
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
  }
  if (rc) return rc;
  if (se != hipSuccess) return set_err(ctx, ACI_E_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(se));
  return ACI_OK;
}

int aci_cubic_step(aci_ctx* ctx, const aci_tt* psi, int32_t dtype, int32_t ndim, const double* coef,
                   double tol, int32_t maxrank, const aci_options* opt, void* out, int64_t out_capacity,
                   aci_result* result) {
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  if (!psi || !coef) return set_err(ctx, ACI_E_INVALID, "null pointer");
  if (dtype != ACI_F64 && dtype != ACI_C128) return set_err(ctx, ACI_E_DTYPE, "unknown dtype");
  if (ndim < 1 || ndim > ACI_MAX_INPUTS - 1) return set_err(ctx, ACI_E_LIMIT, "ndim out of range");
  const int L = psi->L;
  if (L < 2 || L > ACI_MAX_SITES) return set_err(ctx, ACI_E_LIMIT, "L out of range");
  if (L % ndim != 0) return set_err(ctx, ACI_E_INVALID, "L must be a multiple of ndim");
  int rc = validate_tt(ctx, *psi, L);
  if (rc) return rc;
  for (int l = 0; l < L; ++l)
    if (psi->d[l] != 2) return set_err(ctx, ACI_E_INVALID, "quantics grids have d = 2 at every site");
  const int R = L / ndim, ew = dtype == ACI_C128 ? 2 : 1;

  // the second-difference operators (1, -2, 1) / h^2 along each axis
  const double inv_h2 = std::ldexp(1.0, 2 * R);
  const double wts[3] = {inv_h2, -2.0 * inv_h2, inv_h2};
  std::vector<double> hcores((size_t)ndim * 36 * L);
  std::vector<int32_t> wr(L + 1);
  for (int a = 0; a < ndim; ++a) {
    rc = aci_mpo_stencil(R, ndim, a, wts, hcores.data() + (size_t)a * 36 * L, wr.data());
    if (rc) return set_err(ctx, rc, "stencil operator");
  }
  // device memory: the operators, then the D_a psi
  std::vector<int32_t> zr(L + 1);
  std::vector<size_t> zoff(L + 1, 0);
  for (int l = 0; l <= L; ++l) zr[l] = wr[l] * psi->ranks[l];
  for (int l = 0; l < L; ++l) {
    if (zr[l + 1] > ACI_MAX_INPUT_RANK) return set_err(ctx, ACI_E_LIMIT, "3 x rank of psi above ACI_MAX_INPUT_RANK");
    zoff[l + 1] = zoff[l] + (size_t)zr[l] * 2 * zr[l + 1] * ew;
  }
  const size_t wbytes = hcores.size() * sizeof(double);
  void* buf = nullptr;
  if (!dev_alloc(ctx, &buf, wbytes + (size_t)ndim * zoff[L] * sizeof(double)))
    return set_err(ctx, ACI_E_NOMEM, "step workspace");
  double* dW = (double*)buf;
  double* dZ = dW + hcores.size();
  std::vector<int32_t> d2(L, 2);
  std::vector<const double*> Wp((size_t)ndim * L);
  std::vector<void*> Zp((size_t)ndim * L);
  std::vector<aci_tt> in(ndim + 1);
  in[0] = *psi;
  for (int a = 0; a < ndim; ++a)
    for (int l = 0; l < L; ++l) {
      Wp[(size_t)a * L + l] = dW + ((size_t)a * L + l) * 36;
      Zp[(size_t)a * L + l] = dZ + (size_t)a * zoff[L] + zoff[l];
    }
  const hipError_t ce = hipMemcpyAsync(dW, hcores.data(), wbytes, hipMemcpyHostToDevice, ctx->stream);
  rc = ce == hipSuccess ? ACI_OK : set_err(ctx, ACI_E_HIP, std::string("operator upload: ") + hipGetErrorString(ce));
  for (int a = 0; a < ndim && rc == ACI_OK; ++a) {
    rc = enqueue_mpo_apply(ctx, L, d2.data(), wr.data(), Wp.data() + (size_t)a * L, psi->ranks, psi->cores,
                           Zp.data() + (size_t)a * L, ew);
    in[a + 1] = aci_tt{L, d2.data(), zr.data(), (const void* const*)(Zp.data() + (size_t)a * L)};
  }
  if (rc == ACI_OK) {
    // f = c0 psi + c_lap (D_1 psi + ... ) + c3 |psi|^2 psi, started from psi
    aci_options o{};
    if (opt) o = *opt;
    if (!o.init) o.init = psi;
    double cf[2 * (ACI_MAX_INPUTS + 1)];
    for (int t = 0; t <= ndim + 1; ++t) {
      const int src = t == 0 ? 0 : (t <= ndim ? 1 : 2);
      for (int k = 0; k < ew; ++k) cf[ew * t + k] = coef[ew * src + k];
    }
    o.coef = cf;
    o.pointwise = nullptr;
    rc = aci_elementwise(ctx, in.data(), ndim + 1, dtype, ACI_OP_LINEAR_CUBIC, tol, maxrank, &o, out,
                         out_capacity, result);
  }
  const std::string keep = ctx->err;
  (void)hipStreamSynchronize(ctx->stream);
  dev_free(ctx, buf);
  ctx->err = keep;
  return rc;
}

}  // extern "C"

// ------------------------------------------------------------ patched ACI
namespace {

struct PatchNode {
  std::vector<uint8_t> prefix;
  std::vector<const void*> first;   // per input: restricted first core (depth > 0)
  void* out = nullptr;              // output cores of the patch's ACI
  int64_t cap = 0;
  int32_t ranks[ACI_MAX_SITES + 1] = {};
  int64_t offs[ACI_MAX_SITES] = {};
  int64_t elems = 0;
  int converged = 0, sweeps = 0;
  double eps = 0.0;
};

// Elements that always hold the output cores of a TT over sites with local
// dimensions d[0..n) and bond ranks capped by maxrank.
int64_t patch_capacity(const int32_t* d, int n, int maxrank) {
  std::vector<int64_t> left(n + 1, 1), right(n + 1, 1);
  for (int l = 0; l < n; ++l) left[l + 1] = std::min<int64_t>(left[l] * d[l], maxrank);
  for (int l = n - 1; l >= 0; --l) right[l] = std::min<int64_t>(right[l + 1] * d[l], maxrank);
  int64_t cap = 0;
  for (int l = 0; l < n; ++l) {
    const int64_t r0 = std::min(left[l], right[l]), r1 = std::min(left[l + 1], right[l + 1]);
    cap += r0 * d[l] * r1;
  }
  return cap;
}

}  // namespace

extern "C" {

void aci_patched_free(aci_ctx* ctx, aci_patched_result* r) {
  if (!r) return;
  std::free(r->prefix_len);
  std::free(r->prefix);
  std::free(r->ranks);
  std::free(r->core_offset);
  std::free(r->converged);
  std::free(r->sweeps);
  std::free(r->max_eps);
  if (ctx && r->cores) {
    (void)hipStreamSynchronize(ctx->stream);
    dev_free(ctx, r->cores);
  }
  std::memset(r, 0, sizeof(*r));
}

int aci_patched(aci_ctx* ctx, const aci_tt* inputs, int32_t n_inputs, int32_t dtype, int32_t op,
                double tol, int32_t maxrank, int32_t max_depth, const aci_options* opt,
                aci_patched_result* result) {
  if (!ctx) return ACI_E_INVALID;
  ctx->err.clear();
  if (!inputs || !result) return set_err(ctx, ACI_E_INVALID, "null pointer");
  std::memset(result, 0, sizeof(*result));
  if (n_inputs < 1 || n_inputs > ACI_MAX_INPUTS) return set_err(ctx, ACI_E_LIMIT, "n_inputs out of range");
  if (dtype != ACI_F64 && dtype != ACI_C128) return set_err(ctx, ACI_E_DTYPE, "unknown dtype");
  if (maxrank < 1 || maxrank > ACI_MAX_RANK) return set_err(ctx, ACI_E_LIMIT, "maxrank out of range");
  const int L = inputs[0].L;
  if (L < 2 || L > ACI_MAX_SITES) return set_err(ctx, ACI_E_LIMIT, "L out of range");
  if (max_depth < 0 || max_depth > L - 2) return set_err(ctx, ACI_E_INVALID, "max_depth must lie in [0, L - 2]");
  if (opt && opt->init) return set_err(ctx, ACI_E_INVALID, "patches start from the seeded default Y_init (options.init must be NULL)");
  for (int n = 0; n < n_inputs; ++n) {
    const int rc = validate_tt(ctx, inputs[n], L);
    if (rc) return rc;
    for (int l = 0; l < L; ++l)
      if (inputs[n].d[l] != inputs[0].d[l]) return set_err(ctx, ACI_E_INVALID, "inputs differ in local dimensions");
  }
  const int ew = dtype == ACI_C128 ? 2 : 1;
  const int32_t* dims = inputs[0].d;
  std::vector<void*> bufs;   // every device buffer of the call, released at the end
  auto release = [&]() {
    (void)hipStreamSynchronize(ctx->stream);
    for (void* b : bufs) dev_free(ctx, b);
    bufs.clear();
  };
  auto alloc = [&](size_t bytes) -> void* {
    void* p = nullptr;
    if (!dev_alloc(ctx, &p, bytes)) return nullptr;
    bufs.push_back(p);
    return p;
  };

  std::vector<PatchNode> level(1), kept;
  int rc = ACI_OK, worst = ACI_OK, levels = 0;
  for (int depth = 0; depth <= max_depth && !level.empty() && rc >= 0; ++depth) {
    levels = depth + 1;
    const int Lp = L - depth;
    const int64_t cap = patch_capacity(dims + depth, Lp, maxrank);
    // restricted inputs of every patch of the level
    std::vector<std::vector<int32_t>> ranks(level.size() * n_inputs, std::vector<int32_t>(Lp + 1));
    std::vector<std::vector<const void*>> cores(level.size() * n_inputs, std::vector<const void*>(Lp));
    std::vector<aci_tt> tts(level.size() * n_inputs);
    for (size_t p = 0; p < level.size(); ++p)
      for (int n = 0; n < n_inputs; ++n) {
        const size_t i = p * n_inputs + n;
        ranks[i][0] = 1;
        for (int j = 1; j <= Lp; ++j) ranks[i][j] = inputs[n].ranks[depth + j];
        for (int j = 0; j < Lp; ++j) cores[i][j] = inputs[n].cores[depth + j];
        if (depth > 0) cores[i][0] = level[p].first[n];
        tts[i] = aci_tt{Lp, dims + depth, ranks[i].data(), cores[i].data()};
      }
    for (PatchNode& nd : level) {
      nd.cap = cap;
      nd.out = alloc((size_t)cap * ew * sizeof(double));
      if (!nd.out) {
        release();
        return set_err(ctx, ACI_E_NOMEM, "patch output");
      }
    }
    // ACI on the level, ACI_MAX_BATCH patches per batch
    for (size_t p0 = 0; p0 < level.size() && rc >= 0; p0 += ACI_MAX_BATCH) {
      const int cnt = (int)std::min<size_t>(ACI_MAX_BATCH, level.size() - p0);
      std::vector<int32_t> nin(cnt, n_inputs);
      std::vector<void*> outs(cnt);
      std::vector<int64_t> caps(cnt, cap);
      std::vector<aci_result> res(cnt);
      for (int b = 0; b < cnt; ++b) outs[b] = level[p0 + b].out;
      rc = aci_elementwise_batched(ctx, tts.data() + p0 * n_inputs, nin.data(), cnt, dtype, op, tol, maxrank, opt,
                                   outs.data(), caps.data(), res.data());
      for (int b = 0; b < cnt; ++b) {
        PatchNode& nd = level[p0 + b];
        if (rc >= 0) {
          nd.converged = res[b].converged;
          nd.sweeps = res[b].sweeps;
          nd.elems = res[b].out_elems;
          for (int j = 0; j <= Lp; ++j) nd.ranks[j] = res[b].ranks[j];
          for (int j = 0; j < Lp; ++j) nd.offs[j] = res[b].core_offset[j];
          nd.eps = 0.0;
          for (int j = 0; j < Lp - 1; ++j) nd.eps = std::max(nd.eps, res[b].eps[j]);
        }
        aci_result_free(&res[b]);
      }
    }
    if (rc < 0) break;
    // keep the converged patches (all of them at the last level), split the
    // rest; a split patch's own output is not needed any more (the batch
    // call has synchronised its streams)
    std::vector<PatchNode> next;
    for (PatchNode& nd : level) {
      if (nd.converged || depth == max_depth) {
        if (!nd.converged) worst = ACI_W_NOT_CONVERGED;
        kept.push_back(nd);
        continue;
      }
      auto it = std::find(bufs.begin(), bufs.end(), nd.out);
      if (it != bufs.end()) {
        bufs.erase(it);
        dev_free(ctx, nd.out);
        nd.out = nullptr;
      }
      // child sigma: first core v @ X_{depth+1}, v = row sigma of this
      // patch's first core (1 x r_{depth+1})
      for (int sg = 0; sg < dims[depth]; ++sg) {
        PatchNode ch;
        ch.prefix = nd.prefix;
        ch.prefix.push_back((uint8_t)sg);
        ch.first.resize(n_inputs);
        ContractArgs c{};
        c.cplx = ew == 2 ? 1 : 0;
        c.ngroup = n_inputs;
        int nmax = 1;
        for (int n = 0; n < n_inputs; ++n) {
          const int r1 = inputs[n].ranks[depth + 1];
          const int w = dims[depth + 1] * inputs[n].ranks[depth + 2];
          void* buf = alloc((size_t)w * ew * sizeof(double));
          if (!buf) {
            release();
            return set_err(ctx, ACI_E_NOMEM, "patch inputs");
          }
          const double* parent = (const double*)(depth == 0 ? inputs[n].cores[0] : nd.first[n]);
          Group& g = c.g[n];
          g.nterm = 1;
          g.t[0] = Term{parent + (size_t)sg * r1 * ew, (const double*)inputs[n].cores[depth + 1], dconst(r1),
                        dconst(r1), dconst(w)};
          g.C = (double*)buf;
          g.M = dconst(1);
          g.N = dconst(w);
          g.ldc = dconst(w);
          ch.first[n] = buf;
          nmax = std::max(nmax, w);
        }
        const hipError_t e = launch_contract(OP_NONE, PREC_FP64, c, 1, nmax, ctx->stream);
        if (e != hipSuccess) {
          release();
          return set_err(ctx, ACI_E_HIP, std::string("patch restriction: ") + hipGetErrorString(e));
        }
        next.push_back(std::move(ch));
      }
    }
    level = std::move(next);
  }
  if (rc < 0) {
    const std::string keep = ctx->err;
    release();
    ctx->err = keep;
    return rc;
  }
  // gather the kept patches into one buffer of the context's allocator
  const int np = (int)kept.size();
  int64_t total = 0;
  for (const PatchNode& nd : kept) total += nd.elems;
  void* all = nullptr;
  if (!dev_alloc(ctx, &all, (size_t)std::max<int64_t>(total, 1) * ew * sizeof(double))) {
    release();
    return set_err(ctx, ACI_E_NOMEM, "patch result");
  }
  result->n_patches = np;
  result->L = L;
  result->levels = levels;
  result->prefix_len = (int32_t*)std::calloc(np, sizeof(int32_t));
  result->prefix = (uint8_t*)std::calloc((size_t)np * L, 1);
  result->ranks = (int32_t*)std::calloc((size_t)np * (L + 1), sizeof(int32_t));
  result->core_offset = (int64_t*)std::calloc((size_t)np * L, sizeof(int64_t));
  result->converged = (int32_t*)std::calloc(np, sizeof(int32_t));
  result->sweeps = (int32_t*)std::calloc(np, sizeof(int32_t));
  result->max_eps = (double*)std::calloc(np, sizeof(double));
  result->cores = all;
  result->cores_elems = total;
  if (!result->prefix_len || !result->prefix || !result->ranks || !result->core_offset || !result->converged ||
      !result->sweeps || !result->max_eps) {
    release();
    aci_patched_free(ctx, result);
    return set_err(ctx, ACI_E_NOMEM, "host result arrays");
  }
  int64_t off = 0;
  for (int i = 0; i < np; ++i) {
    const PatchNode& nd = kept[i];
    const int k = (int)nd.prefix.size(), Lp = L - k;
    result->prefix_len[i] = k;
    for (int j = 0; j < k; ++j) result->prefix[(size_t)i * L + j] = nd.prefix[j];
    for (int j = 0; j <= Lp; ++j) result->ranks[(size_t)i * (L + 1) + j] = nd.ranks[j];
    for (int j = 0; j < Lp; ++j) result->core_offset[(size_t)i * L + j] = off + nd.offs[j];
    result->converged[i] = nd.converged;
    result->sweeps[i] = nd.sweeps;
    result->max_eps[i] = nd.eps;
    if (nd.elems > 0) {
      const hipError_t e = hipMemcpyAsync((double*)all + (size_t)off * ew, nd.out, (size_t)nd.elems * ew * sizeof(double),
                                          hipMemcpyDeviceToDevice, ctx->stream);
      if (e != hipSuccess) {
        release();
        aci_patched_free(ctx, result);
        return set_err(ctx, ACI_E_HIP, std::string("patch copy: ") + hipGetErrorString(e));
      }
    }
    off += nd.elems;
  }
  release();
  return worst;
}

}  // extern "C"
