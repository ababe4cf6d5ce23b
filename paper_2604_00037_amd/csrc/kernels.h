// Internal launch interface of the ACI kernels (host side).
#pragma once

#include "aci_common.h"

namespace aci {

// ---------------------------------------------------------------- contractions
// One product term A (M x K, row-major, lda) times B (K x N, row-major, ldb).
struct Term {
  const double* A;
  const double* B;
  Dim K;
  Dim lda;
  Dim ldb;
};

// A group writes C = f(term_0, ..., term_{nterm-1}) (elementwise f) into one
// M x N output.  Groups of one launch run side by side (grid z).
struct Group {
  Term t[ACI_MAX_INPUTS];
  int nterm;
  double* C;
  Dim M;
  Dim N;
  Dim ldc;
};

struct ContractArgs {
  Group g[ACI_MAX_INPUTS];
  int ngroup;
  int* err;  // ERR_NONFINITE is or-ed in when an output is NaN/Inf (may be null)
  int cplx;  // 1: operands and result are complex (interleaved re, im); dims
             // and leading dimensions count complex elements
  // OP_LINEAR_CUBIC: a_1..a_N, b as (re, im) pairs (im ignored when real)
  double coef[2 * (ACI_MAX_INPUTS + 1)];
};

// op: OP_NONE (single term, plain GEMM), OP_PRODUCT, OP_SUM, OP_ABS2_MUL.
// mmax/nmax bound the (possibly device-resident) output sizes of every group.
// prec: PREC_FP64, PREC_FP32 or PREC_BF16X3 (operands and result FP64 in HBM).
// tile: TILE_64x64, TILE_32x64, TILE_32x32 output tiles per workgroup, or
// -1 for contract_default_tile.  The tile never changes a result.
enum { TILE_64x64 = 0, TILE_32x64 = 1, TILE_32x32 = 2, NUM_TILES = 3 };
hipError_t launch_contract(int op, int prec, const ContractArgs& args, int mmax, int nmax, hipStream_t s,
                           int tile = -1);
// workgroups of a launch with this tile; the default: the largest tile
// that still gives every CU a workgroup
int contract_tiles(int tile, int mmax, int nmax, int ngroup, int cplx);
int contract_default_tile(int mmax, int nmax, int ngroup, int cplx);

// ------------------------------------------------------------------- prrLU
struct PrrluArgs {
  const double* M;
  Dim m, n, ldm;
  double tol;
  // noise floor relative to the first pivot (0: none): the stop rules
  // compare pivots with max(tol, tol_rel |first pivot|), for two-site
  // tensors contracted in low precision
  double tol_rel;
  int maxrank;
  int rule;
  int P;            // cooperating workgroups
  int stride;       // launch stride: workgroup b is active iff b % stride == 0
  uint64_t* xbuf;   // exchange words, 2 * P * xwords
  size_t xbuf_words;  // capacity of xbuf
  int xwords;       // words per exchange slot
  uint32_t flag_base;
  uint32_t spin_limit;
  // failure-handling tests: from pivot step stall_from on, readers of the
  // exchange wait for flag ^ poll_xor, which no group publishes, so each
  // wait ends at its spin limit (poll_xor 0: off)
  uint32_t poll_xor;
  int stall_from;
  // groups spread over several XCDs publish their candidate's row with the
  // candidate only when its key is at least eager_frac times the predicted
  // next pivot key (0: always); the winner publishes late otherwise
  double eager_frac;
  int* rows;        // out: pivot rows, pivot order
  int* cols;        // out: pivot columns
  int* rank;        // out: rank
  int* rank2;       // out: optional second copy of the rank (bond state)
  double* eps;      // out: error estimate
  double* eps2;     // out: optional second copy
  double* Y;        // out: optional U_JJ^{-1} U (rank x n, ldy)
  Dim ldy;
  int* meta;        // out: optional {rank, m, n}
  int* meta2;       // out: optional second copy (trace)
  int* err;
  int* abort_word;
  // placement and launch (host side unless noted)
  int xcd;            // XCD whose CUs run the groups (0..7); -1: exactly P
                      // workgroups dealt over all XCDs (plain launches only)
  int max_groups;     // cap on P (0: one XCD's CUs)
  int cooperative;    // 1: hipLaunchCooperativeKernel; 0: plain launch (graph capture)
  uint32_t* epoch;    // device word holding flag_base (nullptr: use flag_base);
                      // the kernel advances it for the next launch
  const int* skip;    // optional: the launch does nothing when *skip != 0
  int cplx;           // 1: complex entries (interleaved re, im): M, Y and the
                      // leading dimensions count complex elements
};

// Chooses the workgroup shape for mmax x nmax and launches.
hipError_t launch_prrlu(const PrrluArgs& a, int mmax, int nmax, hipStream_t s);
// Exchange-buffer words needed for matrices up to mmax x nmax.
size_t prrlu_xbuf_words(int mmax, int nmax, int cplx = 0);
// Exchange-buffer words one launch_prrlu call for exactly these bounds and
// group cap reads and writes (both parities), or 0 if out of range.
size_t prrlu_xbuf_used(int mmax, int nmax, int max_groups, int cplx = 0);
// Instance launch_prrlu picks for these bounds: 100000*cplx + 10000*solo +
// 100*RS + CS, or -1 if the bounds are out of range.
int prrlu_variant(int mmax, int nmax, int max_groups = 0, int cplx = 0);
// CUs of one XCD (the most groups one LDU launch places on an XCD)
int prrlu_xcd_cus();
// Cooperating groups (P) launch_prrlu uses for these bounds and group cap.
int prrlu_groups(int mmax, int nmax, int max_groups, int cplx = 0);
// flag_base advance per launch (steps and the XCD check stay below it)
constexpr uint32_t kFlagStride = 2048;

// Factorisations of several products in one launch, each product's groups
// on one XCD.  prod[x][s] is the product slot s of XCD x works for (-1:
// idle), group[x][s] its group index there.
constexpr int kBatchMaxProducts = 12;
constexpr int kBatchSlots = 32;
struct PrrluBatchArgs {
  PrrluArgs a[kBatchMaxProducts];
  int8_t prod[8][kBatchSlots];
  uint8_t group[8][kBatchSlots];
};
static_assert(sizeof(PrrluBatchArgs) <= 4096, "batched LDU arguments exceed 4 KiB");
// Placement and launch of count <= kBatchMaxProducts factorisations of
// matrices up to mmax[i] x nmax (one dtype).  Returns hipErrorInvalidValue
// when the products do not fit one XCD share each.
hipError_t launch_prrlu_batch(const PrrluArgs* a, const int* mmax, int count, int nmax, hipStream_t s);
// Instance code of that launch (200000 + 100000*cplx + 100*RS + CS), or -1
// when the products do not fit.
int prrlu_batch_variant(const int* mmax, int count, int nmax, int cplx);

// ------------------------------------------------------ learned proposal
constexpr int MLP_FEATURES = 7;
constexpr int MLP_HIDDEN = 64;
// flat parameter array: W1 (7 x 64), b1, W2 (64 x 64), b2, w3, b3
constexpr int MLP_PARAMS =
    MLP_FEATURES * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN + 1;

struct FeatureArgs {
  const double* M;
  Dim m, n, ldm;
  const double* env[2];   // left environments A^n (rows a*d + s), row-major
  Dim env_w[2], env_ld[2];
  int n_env;
  const int* prev_rows;   // pivot rows of the previous update of this bond
  const int* prev_rank;   // their number (device), may be null
  float* X;               // m x 7 out
};

struct TrainArgs {
  float* params;
  float* adam_m;
  float* adam_v;
  const float* X;         // count x 7
  const float* y;         // count labels (0 / 1)
  int count;
  float lr, beta1, beta2, one_minus_beta1, one_minus_beta2, c1, c2, eps;
  float* scratch;         // (6 * 64 + 1) * count floats
  float* grads;           // optional MLP_PARAMS out
  float* loss;            // optional mean loss out
};

struct RookArgs {
  const double* M;
  Dim m, n, ldm;
  double tol;
  int maxrank;
  int max_iter;
  const float* scores;    // m, may be null
  double* L;              // m x maxrank, row-major, leading dim ldl
  int ldl;
  double* Up;             // maxrank x n, leading dim ldu
  int ldu;
  int *rows, *cols, *rank;
  double* eps;
  int* scans;             // optional
};

struct CheckArgs {
  const double* M;
  Dim m, n, ldm;
  const double* C;        // L Up
  int ldc;
  double tol;
  double* eps;
  int* accepted;          // [0] = eps <= tol, [1] = its negation
  int* count;             // optional: incremented when accepted
};

// Copies an accepted proposal into the outputs of the LDU it replaces.
struct CommitArgs {
  const int* accepted;
  const int *src_rows, *src_cols, *src_rank;
  const double* src_eps;
  int *rows, *cols, *rank, *rank2;
  double *eps, *eps2;
  int *meta, *meta2;
  Dim m, n;
  int maxrank;
  // optional: scan_total[0] += *src_scans, scan_total[1] += *src_rank (every
  // proposal, accepted or not)
  const int* src_scans;
  int* scan_total;
};

// dst[0 .. *rank) = src, *dst_rank = *rank
struct CopyRowsArgs {
  const int* src;
  const int* rank;
  int* dst;
  int* dst_rank;
  int maxrank;
};

// Appends one local update's rows to a training set of the scoring network:
// X[count + i] = feat[i] (7 floats), y[count + i] = 1 for the first
// max(1, rank / 2) pivot rows, else 0, for i < m; then count += m.  An update
// that would pass `capacity` writes nothing and sets count[1] (and so does
// every later one).
struct RecordArgs {
  const float* feat;    // m x 7 features of the update
  Dim m;
  const int* rows;      // pivot rows of the update, in pivot order
  const int* rank;
  float* X;             // capacity x 7
  float* y;             // capacity
  int64_t capacity;
  long long* count;     // [0] rows so far, [1] overflow flag
};

struct SolveArgs {
  const double* Up;
  int ldu;
  const int* cols;
  const int* rank;
  Dim n;
  double* Y;
  Dim ldy;
  const int* skip;        // optional: return at once when *skip != 0
};

hipError_t launch_features(const FeatureArgs& a, hipStream_t s);
hipError_t launch_mlp_forward(const float* params, const float* X, int count, float* out, hipStream_t s);
hipError_t launch_mlp_train(const TrainArgs& a, hipStream_t s);
hipError_t launch_rook(const RookArgs& a, hipStream_t s);
hipError_t launch_check(const CheckArgs& a, hipStream_t s);
hipError_t launch_rook_solve(const SolveArgs& a, hipStream_t s);
hipError_t launch_commit(const CommitArgs& a, hipStream_t s);
hipError_t launch_copy_rows(const CopyRowsArgs& a, hipStream_t s);
hipError_t launch_record(const RecordArgs& a, hipStream_t s);

// ----------------------------------------------------------------- gathers
struct GatherItem {
  const double* src;
  double* dst;
  Dim ld_src;
  Dim ld_dst;
  Dim extent;        // side 0: row length; side 1: number of rows
  Dim src_n;         // side 0: rows of src; side 1: columns of src (index bound)
};
struct GatherArgs {
  GatherItem it[ACI_MAX_INPUTS + 1];
  int count;
  int side;          // 0: rows of src (dst row k = src row idx[k]); 1: columns
  const int* idx;
  const int* rank;   // number of gathered rows/columns (device)
  int* err;          // ERR_LIMIT is or-ed in for an index out of range (may be null)
  int esz;           // doubles per element (1 real, 2 complex; 0 counts as 1)
};
hipError_t launch_gather(const GatherArgs& a, int rmax, int extent_max, hipStream_t s);

// ------------------------------------------------------------ 2-site TCI
struct TciPointsArgs {
  const int32_t* I_prev;   // |I_{l-1}| digit rows of length L
  const int32_t* J_next;   // |J_{l+2}| digit rows of length L
  int32_t* pts;            // m n rows of L digits out
  int m, n, d, cR, l, L;   // m = |I_{l-1}| d, n = d' cR
};
struct TciSetsArgs {
  const int* rows;         // pivot rows / columns of the bond's LDU
  const int* cols;
  const int* rank;         // their number (device)
  const int32_t* I_prev;
  const int32_t* J_next;
  int32_t* I_out;          // I_l digit rows out
  int32_t* J_out;          // J_{l+1} digit rows out
  int d, cR, l, L;
};
hipError_t launch_tci_points(const TciPointsArgs& a, hipStream_t s);
hipError_t launch_tci_sets(const TciSetsArgs& a, int rmax, hipStream_t s);

// ------------------------------------------------------- TT operators
// One site of an MPO-TT contraction Z = W X (real W; X and Z in real units:
// a complex core is a real one whose right bond counts re and im).
struct MpoSite {
  const double* W;   // wa x d x d x wb
  const double* X;   // ra x d x xe     (xe = right rank in doubles)
  double* Z;         // (wa ra) x d x (wb xe)
  int wa, wb, ra, xe, d;
  int vec;           // 1: xe even and X, Z 16-byte aligned (two doubles per access)
  int block0;        // first workgroup of this site within the launch
};
constexpr int kMpoSitesPerLaunch = 32;
struct MpoArgs {
  MpoSite site[kMpoSitesPerLaunch];
  int nsite;
};
// workgroups one site needs (4 row groups (a, c, s) of wb x xe doubles each)
int mpo_site_blocks(const MpoSite& m);
hipError_t launch_mpo_apply(const MpoArgs& a, int blocks, hipStream_t s);

// Fill `count` doubles with `value` (used instead of a memset so the sweep can
// be captured in a graph).
hipError_t launch_fill(double* p, size_t count, double value, hipStream_t s);
hipError_t launch_fill_int(int* p, size_t count, int value, hipStream_t s);

}  // namespace aci
