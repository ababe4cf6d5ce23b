// Dense contractions of the local update on the matrix cores.
//
// Environment contractions A = L_{l-1} X_l and B = X_{l+1} R_{l+2} and the
// two-site tensors Pi^n = A^n B^n (Eq. pifromframes), with the elementwise f
// of Eq. (localupdate) applied in the epilogue so that Pi = f(Pi^1..Pi^N) is
// written once.  Each workgroup computes a TM x TN output tile (64x64, 32x64
// or 32x32, picked per shape by a heuristic or the autotuner); its four
// waves each own a quarter made of 16x16 MFMA blocks.  Every output element
// is accumulated by the same MFMA sequence (k ascending) whatever the tile,
// so the tile shape never changes a result.  Operands are FP64 in HBM and
// the result is written in FP64 in every precision:
//
// * FP64: v_mfma_f64_16x16x4f64; 64x16 (A, k-major) and 16x64 (B) tiles in
//   LDS so that every lane of an MFMA reads consecutive doubles.
// * FP32: operands rounded to FP32 while staged, v_mfma_f32_16x16x4f32,
//   FP32 accumulation.
// * BF16x3: each operand x is split while staged into hi = bf16(x) and
//   lo = bf16(x - hi) (x first rounded to FP32); the product uses
//   hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16 with FP32
//   accumulation (about 16 significant bits per operand).
//
// Complex operands (interleaved re, im) use the same kernels on real views:
// A (m x K complex) is read as the real m x 2K matrix [re im re im ...], and
// B (K x N complex) is expanded while staged into the real 2K x 2N matrix
// with b[2t][2j] = re, b[2t][2j+1] = im, b[2t+1][2j] = -im,
// b[2t+1][2j+1] = re of B[t][j], so the real product is C interleaved (the
// same 8 mkn real flops as a complex GEMM).  An f that couples re and im
// (products of several terms, |z|^2 z) pairs each accumulator value with the
// one of the neighbouring lane, which holds the other part of the element.
//
// Lane layouts (measured on gfx950), lane l, r = l % 16, g = l / 16:
//   f64 16x16x4:   A[r][g], B[g][r];            acc item v = C[g + 4v][r]
//   f32 16x16x4:   A[r][g], B[g][r];            acc item v = C[4g + v][r]
//   bf16 16x16x32: A[r][8g + e], B[8g + e][r];  acc item v = C[4g + v][r]
#include "kernels.h"

namespace aci {

namespace {

constexpr int KC = 32;        // k per load chunk (FP64 stages one, FP32 / BF16x3 two)

// Shape of a TM x TN output tile (TM, TN in {32, 64}).  One chunk of A (TM x
// 32) and B (32 x TN, real view) is loaded by the 256 threads into
// registers, EA and EB values per thread, while the previous chunk is
// multiplied from LDS.  Two assignments of values to threads (MAP):
//   MAP_SPREAD (FP64, FP32; LDS tiles [k][row] and [k][col]):
//     A value e of thread t: row t / TPA, k (t % TPA) + TPA e;
//     B value e, real: k t / 16 + 16 (e / NC), column t % 16 + 16 (e % NC)
//     (NC = TN / 16): a wave's stores of one value index cover 64 distinct
//     banks of the padded tiles, and each load instruction reads whole
//     segments of consecutive entries;
//   MAP_PACKED (BF16x3; LDS tiles [row][k] and [col][k]): a thread holds
//     consecutive k of one row of A (k EA (t % TPA) + e) and of one column
//     of B (column t % TN, k EB (t / TN) + e), stored as one vector.
//   Complex B is read once per element and expanded in registers into its
//   2 x 2 real block (values 2q, 2q + 1: row 2 ct, columns 2 cj, 2 cj + 1;
//   values EB/2 + 2q, EB/2 + 2q + 1: row 2 ct + 1, same columns), CE
//   elements per thread: MAP_SPREAD: element q of thread t at complex k
//   t / (TN/2) + (512/TN) q, complex column t % (TN/2) (a wave reads whole
//   rows of elements and stores each real row pair as one vector);
//   MAP_PACKED: k ct = t / TPC, columns cj0 + q with cj0 = CE (t % TPC).
constexpr int MAP_SPREAD = 0, MAP_PACKED = 1;

template <int TM_, int TN_>
struct Tile {
  static constexpr int TM = TM_, TN = TN_;
  static constexpr int EA = TM * KC / 256;
  static constexpr int EB = TN * KC / 256;
  static constexpr int TPA = KC / EA;
  static constexpr int TPB = TN / EB;
  static constexpr int NC = TN / 16;
  static constexpr int CE = EB / 4;
  static constexpr int TPC = (TN / 2) / CE;
  static constexpr int MI = TM / 32;   // 16-row blocks per wave (waves are 2 x 2)
  static constexpr int NJ = TN / 32;   // 16-column blocks per wave
  // FP64 LDS pitches ([k][row], [k][col]), in doubles: rows of the tile 16
  // doubles (128 bytes) apart modulo 256 bytes, so that the four k rows an
  // MFMA operand read touches fall on distinct banks
  static constexpr int LDA = TM + 16;
  static constexpr int LDB = TN + 16;
  __device__ static int a_row(int t) { return t / TPA; }
  template <int MAP>
  __device__ static int a_k(int t, int e) { return MAP == MAP_SPREAD ? (t % TPA) + TPA * e : (t % TPA) * EA + e; }
  // complex B, MAP_SPREAD: element q of thread t
  __device__ static int cb_k(int t, int q) { return t / (TN / 2) + (512 / TN) * q; }
  __device__ static int cb_col(int t) { return t % (TN / 2); }
  template <bool CPLX, int MAP>
  __device__ static int b_k(int t, int e) {
    if (CPLX) return 2 * (t / TPC) + e / (EB / 2);
    return MAP == MAP_SPREAD ? t / 16 + 16 * (e / NC) : (t / TN) * EB + e;
  }
  template <bool CPLX, int MAP>
  __device__ static int b_col(int t, int e) {
    if (CPLX) return 2 * CE * (t % TPC) + e % (EB / 2);
    return MAP == MAP_SPREAD ? t % 16 + 16 * (e % NC) : t % TN;
  }
};

template <class TL, bool CPLX, int MAP>
__device__ __forceinline__ void load_chunk(const Term& T, int M, int N, int K, int lda, int ldb, int m0, int n0,
                                           int k0, int t, double (&av)[TL::EA], double (&bv)[TL::EB]) {
  const int gr = m0 + TL::a_row(t);
#pragma unroll
  for (int e = 0; e < TL::EA; ++e) {
    const int gk = k0 + TL::template a_k<MAP>(t, e);
    av[e] = (gr < M && gk < K) ? T.A[(size_t)gr * lda + gk] : 0.0;
  }
  if (!CPLX) {
#pragma unroll
    for (int e = 0; e < TL::EB; ++e) {
      const int gk = k0 + TL::template b_k<false, MAP>(t, e);
      const int gc = n0 + TL::template b_col<false, MAP>(t, e);
      bv[e] = (gk < K && gc < N) ? T.B[(size_t)gk * ldb + gc] : 0.0;
    }
  } else {
#pragma unroll
    for (int q = 0; q < TL::CE; ++q) {
      const int ct = (k0 >> 1) + (MAP == MAP_SPREAD ? TL::cb_k(t, q) : t / TL::TPC);
      const int cjq = (n0 >> 1) + (MAP == MAP_SPREAD ? TL::cb_col(t) : TL::CE * (t % TL::TPC) + q);
      double re = 0.0, im = 0.0;
      if (2 * ct < K && 2 * cjq < N) {
        const double* e = T.B + 2 * ((size_t)ct * ldb + cjq);
        re = e[0];
        im = e[1];
      }
      bv[2 * q] = re;                    // real row 2ct:     (re, im)
      bv[2 * q + 1] = im;
      bv[TL::EB / 2 + 2 * q] = -im;      // real row 2ct + 1: (-im, re)
      bv[TL::EB / 2 + 2 * q + 1] = re;
    }
  }
}

template <int OP>
__device__ __forceinline__ v4d combine(v4d r, v4d a) {
  if (OP == OP_PRODUCT) return r * a;
  return r + a;  // OP_SUM
}

// f applied to one accumulator value of a complex result, given the value
// the neighbouring lane holds for the same element (even lane: real part).
template <int OP>
__device__ __forceinline__ double cplx_combine(double res, double res_o, double acc, double acc_o, bool even) {
  const double rr = even ? res : res_o, ri = even ? res_o : res;
  const double ar = even ? acc : acc_o, ai = even ? acc_o : acc;
  if (OP == OP_PRODUCT) return even ? rr * ar - ri * ai : rr * ai + ri * ar;
  return res + acc;
}
template <bool CPLX>
__device__ __forceinline__ double abs2_mul(double x, double x_o, bool even) {
  if (!CPLX) return (x * x) * x;
  const double re = even ? x : x_o, im = even ? x_o : x;
  const double a = re * re + im * im;
  return a * x;
}

// c x for a constant c = (cr, ci) of the dtype; xo is the neighbouring
// lane's value (the other part of the same complex element).
template <bool CPLX>
__device__ __forceinline__ double scale(double cr, double ci, double x, double xo, bool even) {
  if (!CPLX) return cr * x;
  return even ? cr * x - ci * xo : cr * x + ci * xo;
}

// Epilogue of one term: fold the term's accumulators into the running
// result (f of Eq. localupdate), element by element.  coef (OP_LINEAR_CUBIC
// only): b, then a_1, a_2, ... as (re, im) pairs.
template <int OP, bool CPLX, int MI, int NJ>
__device__ __forceinline__ void fold_term(v4d (&res)[MI][NJ], const v4d (&x)[MI][NJ], int t, bool even,
                                          const double* coef) {
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      if (OP == OP_LINEAR_CUBIC) {
        const double ar = coef[2 * t + 2], ai = coef[2 * t + 3];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double xv = x[i][j][v];
          const double xo = CPLX ? __shfl_xor(xv, 1) : xv;
          const double y = scale<CPLX>(ar, ai, xv, xo, even);
          if (t == 0) {
            // a_1 x_1 + b |x_1|^2 x_1
            const double c = abs2_mul<CPLX>(xv, xo, even);
            const double co = CPLX ? __shfl_xor(c, 1) : c;
            res[i][j][v] = y + scale<CPLX>(coef[0], coef[1], c, co, even);
          } else {
            res[i][j][v] = res[i][j][v] + y;
          }
        }
      } else if (OP == OP_ABS2_MUL) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double xv = x[i][j][v];
          const double xo = CPLX ? __shfl_xor(xv, 1) : xv;
          res[i][j][v] = abs2_mul<CPLX>(xv, xo, even);
        }
      } else if (OP == OP_NONE || t == 0) {
        res[i][j] = x[i][j];
      } else if (CPLX && OP == OP_PRODUCT) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double r0 = res[i][j][v], a0 = x[i][j][v];
          const double ro = __shfl_xor(r0, 1), ao = __shfl_xor(a0, 1);
          res[i][j][v] = cplx_combine<OP>(r0, ro, a0, ao, even);
        }
      } else {
        res[i][j] = combine<OP>(res[i][j], x[i][j]);
      }
    }
}

// Store of the result tile; row of accumulator item v of a 16x16 block is
// rowbase + RSTEP v (FP64 layout: lk + 4v; FP32: 4 lg + v).
template <int OP, int MI, int NJ>
__device__ __forceinline__ void store_tile(const Group& g, const v4d (&res)[MI][NJ], int M, int N, int ldc,
                                           int row0, int col0, int rstep, int* err) {
  bool bad = false;
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = row0 + i * 16 + rstep * v;
        const int col = col0 + j * 16;
        if (row < M && col < N) {
          const double x = res[i][j][v];
          if (OP != OP_NONE && !__builtin_isfinite(x)) bad = true;
          g.C[(size_t)row * ldc + col] = x;
        }
      }
  if (OP != OP_NONE && bad && err) atomicOr(err, ERR_NONFINITE);
}

template <int OP, bool CPLX, class TL>
__global__ __launch_bounds__(256) void contract_kernel(ContractArgs args) {
  __shared__ __align__(16) double sA[KC * TL::LDA];
  __shared__ __align__(16) double sB[KC * TL::LDB];
  constexpr int W = CPLX ? 2 : 1;
  constexpr int MI = TL::MI, NJ = TL::NJ;
  const Group& g = args.g[blockIdx.z];
  const int M = dget(g.M);
  const int N = W * dget(g.N);
  const int m0 = blockIdx.y * TL::TM;
  const int n0 = blockIdx.x * TL::TN;
  if (m0 >= M || n0 >= N) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15, lk = lane >> 4;
  const bool even = (lr & 1) == 0;

  v4d res[MI][NJ];
  for (int t = 0; t < g.nterm; ++t) {
    const Term& T = g.t[t];
    const int K = W * dget(T.K);
    const int lda = W * dget(T.lda);
    const int ldb = dget(T.ldb);
    v4d acc[MI][NJ];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    double av[TL::EA], bv[TL::EB];
    load_chunk<TL, CPLX, MAP_SPREAD>(T, M, N, K, lda, ldb, m0, n0, 0, tid, av, bv);
    for (int k0 = 0; k0 < K; k0 += KC) {
#pragma unroll
      for (int e = 0; e < TL::EA; ++e) sA[TL::template a_k<MAP_SPREAD>(tid, e) * TL::LDA + TL::a_row(tid)] = av[e];
      if constexpr (CPLX) {
#pragma unroll
        for (int q = 0; q < TL::CE; ++q) {
          const int r = 2 * TL::cb_k(tid, q), c = 2 * TL::cb_col(tid);
          *reinterpret_cast<double2*>(&sB[r * TL::LDB + c]) = double2{bv[2 * q], bv[2 * q + 1]};
          *reinterpret_cast<double2*>(&sB[(r + 1) * TL::LDB + c]) =
              double2{bv[TL::EB / 2 + 2 * q], bv[TL::EB / 2 + 2 * q + 1]};
        }
      } else {
#pragma unroll
        for (int e = 0; e < TL::EB; ++e)
          sB[TL::template b_k<false, MAP_SPREAD>(tid, e) * TL::LDB + TL::template b_col<false, MAP_SPREAD>(tid, e)] =
              bv[e];
      }
      __syncthreads();
      // the next chunk's loads are in flight while this one is multiplied
      if (k0 + KC < K) load_chunk<TL, CPLX, MAP_SPREAD>(T, M, N, K, lda, ldb, m0, n0, k0 + KC, tid, av, bv);
      // operands of step ks + 1 are read while step ks is multiplied (two
      // register sets, so the reads need not wait for the MFMAs that use the
      // previous set)
      double a[2][MI], b[2][NJ];
#pragma unroll
      for (int i = 0; i < MI; ++i) a[0][i] = sA[lk * TL::LDA + wm * (TL::TM / 2) + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < NJ; ++j) b[0][j] = sB[lk * TL::LDB + wn * (TL::TN / 2) + j * 16 + lr];
#pragma unroll
      for (int ks = 0; ks < KC / 4; ++ks) {
        const int cur = ks & 1, nxt = cur ^ 1;
        if (ks + 1 < KC / 4) {
          const int kr = (ks + 1) * 4 + lk;
#pragma unroll
          for (int i = 0; i < MI; ++i) a[nxt][i] = sA[kr * TL::LDA + wm * (TL::TM / 2) + i * 16 + lr];
#pragma unroll
          for (int j = 0; j < NJ; ++j) b[nxt][j] = sB[kr * TL::LDB + wn * (TL::TN / 2) + j * 16 + lr];
        }
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < NJ; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[cur][i], b[cur][j], acc[i][j], 0, 0, 0);
        // keep that order: the next step's LDS reads, then this step's MFMAs
        if (ks + 1 < KC / 4) __builtin_amdgcn_sched_group_barrier(0x100, MI + NJ, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, MI * NJ, 0);
      }
      __syncthreads();
    }
    fold_term<OP, CPLX, MI, NJ>(res, acc, t, even, args.coef);
  }
  store_tile<OP, MI, NJ>(g, res, M, N, W * dget(g.ldc), m0 + wm * (TL::TM / 2) + lk,
                         n0 + wn * (TL::TN / 2) + lr, 4, args.err);
}

// ---------------------------------------------------------------- FP32 / BF16x3
constexpr int KL = 2 * KC;    // k per staged chunk: two load chunks (the
                              // low-precision products are cheaper per k)
constexpr int LDH = KL + 8;   // bf16 tiles, 64 k per row/column (+pad; 16-byte rows)

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// Round-to-nearest-even FP32 -> bf16 bits (finite inputs; a non-finite
// input stays non-finite, which the epilogue flags).
__device__ __forceinline__ unsigned short bf16_bits(float x) {
  const unsigned int u = __float_as_uint(x);
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_value(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

template <int PREC, class TL>
struct alignas(16) LpTiles;

template <class TL>
struct alignas(16) LpTiles<PREC_FP32, TL> {
  float A[KL * (TL::TM + 16)];   // [k][row]
  float B[KL * (TL::TN + 16)];   // [k][col]
};

// N bf16 bit patterns as one LDS store (N = 4 or 8; dst aligned to 2N bytes)
template <int N>
__device__ __forceinline__ void store_bf16s(unsigned short* dst, const unsigned short (&v)[N]) {
  typedef unsigned short vec __attribute__((ext_vector_type(N)));
  vec x;
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = v[i];
  *reinterpret_cast<vec*>(dst) = x;
}

template <class TL>
struct alignas(16) LpTiles<PREC_BF16X3, TL> {
  unsigned short Ah[TL::TM * LDH], Al[TL::TM * LDH];   // [row][k]
  unsigned short Bh[TL::TN * LDH], Bl[TL::TN * LDH];   // [col][k]
};

template <int OP, int PREC, bool CPLX, class TL>
__global__ __launch_bounds__(256) void contract_lp_kernel(ContractArgs args) {
  __shared__ LpTiles<PREC, TL> sh;
  constexpr int W = CPLX ? 2 : 1;
  constexpr int MI = TL::MI, NJ = TL::NJ;
  // FP32 pitches: k rows 16 words apart modulo 64 banks (MFMA operand reads
  // conflict-free); the spread assignment makes the staging stores so too
  constexpr int LDFA = TL::TM + 16, LDFB = TL::TN + 16;
  constexpr int MAP = PREC == PREC_FP32 ? MAP_SPREAD : MAP_PACKED;
  const Group& g = args.g[blockIdx.z];
  const int M = dget(g.M);
  const int N = W * dget(g.N);
  const int m0 = blockIdx.y * TL::TM;
  const int n0 = blockIdx.x * TL::TN;
  if (m0 >= M || n0 >= N) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15, lg = lane >> 4;
  const bool even = (lr & 1) == 0;

  v4d res[MI][NJ];
  for (int t = 0; t < g.nterm; ++t) {
    const Term& T = g.t[t];
    const int K = W * dget(T.K);
    const int lda = W * dget(T.lda);
    const int ldb = dget(T.ldb);
    v4f acc[MI][NJ];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

    double av[2][TL::EA], bv[2][TL::EB];
    load_chunk<TL, CPLX, MAP>(T, M, N, K, lda, ldb, m0, n0, 0, tid, av[0], bv[0]);
    load_chunk<TL, CPLX, MAP>(T, M, N, K, lda, ldb, m0, n0, KC, tid, av[1], bv[1]);
    for (int k0 = 0; k0 < K; k0 += KL) {
      const int ar = TL::a_row(tid);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int kh = KC * h;
        if (PREC == PREC_FP32) {
          auto& S = reinterpret_cast<LpTiles<PREC_FP32, TL>&>(sh);
#pragma unroll
          for (int e = 0; e < TL::EA; ++e) S.A[(kh + TL::template a_k<MAP>(tid, e)) * LDFA + ar] = (float)av[h][e];
          if constexpr (CPLX) {
#pragma unroll
            for (int q = 0; q < TL::CE; ++q) {
              const int r = kh + 2 * TL::cb_k(tid, q), c = 2 * TL::cb_col(tid);
              *reinterpret_cast<float2*>(&S.B[r * LDFB + c]) = float2{(float)bv[h][2 * q], (float)bv[h][2 * q + 1]};
              *reinterpret_cast<float2*>(&S.B[(r + 1) * LDFB + c]) =
                  float2{(float)bv[h][TL::EB / 2 + 2 * q], (float)bv[h][TL::EB / 2 + 2 * q + 1]};
            }
          } else {
#pragma unroll
            for (int e = 0; e < TL::EB; ++e)
              S.B[(kh + TL::template b_k<false, MAP>(tid, e)) * LDFB + TL::template b_col<false, MAP>(tid, e)] =
                  (float)bv[h][e];
          }
        } else {
          auto& S = reinterpret_cast<LpTiles<PREC_BF16X3, TL>&>(sh);
          // this thread's EA consecutive k of one row: one vector store each
          unsigned short ah_[TL::EA], al_[TL::EA];
#pragma unroll
          for (int e = 0; e < TL::EA; ++e) {
            const float fa = (float)av[h][e];
            ah_[e] = bf16_bits(fa);
            al_[e] = bf16_bits(fa - bf16_value(ah_[e]));
          }
          const int ak0 = kh + TL::template a_k<MAP_PACKED>(tid, 0);
          store_bf16s<TL::EA>(&S.Ah[ar * LDH + ak0], ah_);
          store_bf16s<TL::EA>(&S.Al[ar * LDH + ak0], al_);
          if constexpr (!CPLX) {
            // EB consecutive k of one column
            unsigned short bh_[TL::EB], bl_[TL::EB];
#pragma unroll
            for (int e = 0; e < TL::EB; ++e) {
              const float fb = (float)bv[h][e];
              bh_[e] = bf16_bits(fb);
              bl_[e] = bf16_bits(fb - bf16_value(bh_[e]));
            }
            const int bk0 = kh + TL::template b_k<false, MAP_PACKED>(tid, 0);
            const int bc = TL::template b_col<false, MAP_PACKED>(tid, 0);
            store_bf16s<TL::EB>(&S.Bh[bc * LDH + bk0], bh_);
            store_bf16s<TL::EB>(&S.Bl[bc * LDH + bk0], bl_);
          } else {
            // value e and EB/2 + e share a column and are consecutive in k
            // (real rows 2 ct and 2 ct + 1): one 32-bit store per column
            const int bk = kh + TL::template b_k<true, MAP_PACKED>(tid, 0);
#pragma unroll
            for (int e = 0; e < TL::EB / 2; ++e) {
              const int bc = TL::template b_col<true, MAP_PACKED>(tid, e);
              const float f0 = (float)bv[h][e], f1 = (float)bv[h][TL::EB / 2 + e];
              const unsigned short h0 = bf16_bits(f0), h1 = bf16_bits(f1);
              const unsigned short l0 = bf16_bits(f0 - bf16_value(h0)), l1 = bf16_bits(f1 - bf16_value(h1));
              *reinterpret_cast<unsigned int*>(&S.Bh[bc * LDH + bk]) = (unsigned int)h0 | ((unsigned int)h1 << 16);
              *reinterpret_cast<unsigned int*>(&S.Bl[bc * LDH + bk]) = (unsigned int)l0 | ((unsigned int)l1 << 16);
            }
          }
        }
      }
      __syncthreads();
      // the next chunk's loads are in flight while this one is multiplied
      if (k0 + KL < K) {
        load_chunk<TL, CPLX, MAP>(T, M, N, K, lda, ldb, m0, n0, k0 + KL, tid, av[0], bv[0]);
        load_chunk<TL, CPLX, MAP>(T, M, N, K, lda, ldb, m0, n0, k0 + KL + KC, tid, av[1], bv[1]);
      }
      if (PREC == PREC_FP32) {
        auto& S = reinterpret_cast<LpTiles<PREC_FP32, TL>&>(sh);
        // operands of step ks + 1 read while step ks is multiplied
        float a[2][MI], b[2][NJ];
#pragma unroll
        for (int i = 0; i < MI; ++i) a[0][i] = S.A[lg * LDFA + wm * (TL::TM / 2) + i * 16 + lr];
#pragma unroll
        for (int j = 0; j < NJ; ++j) b[0][j] = S.B[lg * LDFB + wn * (TL::TN / 2) + j * 16 + lr];
#pragma unroll
        for (int ks = 0; ks < KL / 4; ++ks) {
          const int cur = ks & 1, nxt = cur ^ 1;
          if (ks + 1 < KL / 4) {
            const int kr = (ks + 1) * 4 + lg;
#pragma unroll
            for (int i = 0; i < MI; ++i) a[nxt][i] = S.A[kr * LDFA + wm * (TL::TM / 2) + i * 16 + lr];
#pragma unroll
            for (int j = 0; j < NJ; ++j) b[nxt][j] = S.B[kr * LDFB + wn * (TL::TN / 2) + j * 16 + lr];
          }
#pragma unroll
          for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[cur][i], b[cur][j], acc[i][j], 0, 0, 0);
          if (ks + 1 < KL / 4) __builtin_amdgcn_sched_group_barrier(0x100, MI + NJ, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, MI * NJ, 0);
        }
      } else {
        auto& S = reinterpret_cast<LpTiles<PREC_BF16X3, TL>&>(sh);
#pragma unroll
        for (int ks = 0; ks < KL / 32; ++ks) {
          v8bf ah[MI], al[MI], bh[NJ], bl[NJ];
#pragma unroll
          for (int i = 0; i < MI; ++i) {
            const int row = wm * (TL::TM / 2) + i * 16 + lr;
            ah[i] = *reinterpret_cast<const v8bf*>(&S.Ah[row * LDH + 32 * ks + 8 * lg]);
            al[i] = *reinterpret_cast<const v8bf*>(&S.Al[row * LDH + 32 * ks + 8 * lg]);
          }
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            const int col = wn * (TL::TN / 2) + j * 16 + lr;
            bh[j] = *reinterpret_cast<const v8bf*>(&S.Bh[col * LDH + 32 * ks + 8 * lg]);
            bl[j] = *reinterpret_cast<const v8bf*>(&S.Bl[col * LDH + 32 * ks + 8 * lg]);
          }
#pragma unroll
          for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
            }
        }
      }
      __syncthreads();
    }
    v4d x[MI][NJ];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        x[i][j] = v4d{(double)acc[i][j][0], (double)acc[i][j][1], (double)acc[i][j][2], (double)acc[i][j][3]};
    fold_term<OP, CPLX, MI, NJ>(res, x, t, even, args.coef);
  }
  store_tile<OP, MI, NJ>(g, res, M, N, W * dget(g.ldc), m0 + wm * (TL::TM / 2) + 4 * lg,
                         n0 + wn * (TL::TN / 2) + lr, 1, args.err);
}

using T64x64 = Tile<64, 64>;
using T32x64 = Tile<32, 64>;
using T32x32 = Tile<32, 32>;

template <int OP, int PREC, bool CPLX, class TL>
const void* kernel_of() {
  if constexpr (PREC == PREC_FP64) return (const void*)contract_kernel<OP, CPLX, TL>;
  else return (const void*)contract_lp_kernel<OP, PREC, CPLX, TL>;
}

template <int PREC, bool CPLX, class TL>
const void* pick_op(int op) {
  switch (op) {
    case OP_NONE: return kernel_of<OP_NONE, PREC, CPLX, TL>();
    case OP_PRODUCT: return kernel_of<OP_PRODUCT, PREC, CPLX, TL>();
    case OP_SUM: return kernel_of<OP_SUM, PREC, CPLX, TL>();
    case OP_ABS2_MUL: return kernel_of<OP_ABS2_MUL, PREC, CPLX, TL>();
    case OP_LINEAR_CUBIC: return kernel_of<OP_LINEAR_CUBIC, PREC, CPLX, TL>();
    default: return nullptr;
  }
}

template <int PREC, bool CPLX>
const void* pick_tile(int op, int tile) {
  switch (tile) {
    case TILE_64x64: return pick_op<PREC, CPLX, T64x64>(op);
    case TILE_32x64: return pick_op<PREC, CPLX, T32x64>(op);
    case TILE_32x32: return pick_op<PREC, CPLX, T32x32>(op);
    default: return nullptr;
  }
}

const int kTileM[3] = {64, 32, 32};
const int kTileN[3] = {64, 64, 32};

}  // namespace

int contract_tiles(int tile, int mmax, int nmax, int ngroup, int cplx) {
  if (tile < 0 || tile >= NUM_TILES) return -1;
  const int nreal = cplx ? 2 * nmax : nmax;
  return ((nreal + kTileN[tile] - 1) / kTileN[tile]) * ((mmax + kTileM[tile] - 1) / kTileM[tile]) * ngroup;
}

int contract_default_tile(int mmax, int nmax, int ngroup, int cplx) {
  // the largest tile that still gives every CU two workgroups (one cannot
  // hide its own staging; measured 3 % more contraction throughput on the
  // complex 512-row products than with one per CU)
  for (int t = 0; t < NUM_TILES; ++t)
    if (contract_tiles(t, mmax, nmax, ngroup, cplx) >= 512) return t;
  return NUM_TILES - 1;
}

hipError_t launch_contract(int op, int prec, const ContractArgs& args, int mmax, int nmax, hipStream_t s, int tile) {
  if (mmax <= 0 || nmax <= 0 || args.ngroup <= 0) return hipSuccess;
  const bool cplx = args.cplx != 0;
  if (tile < 0) tile = contract_default_tile(mmax, nmax, args.ngroup, cplx);
  if (tile >= NUM_TILES) return hipErrorInvalidValue;
  const void* fn = nullptr;
  if (prec == PREC_FP64) fn = cplx ? pick_tile<PREC_FP64, true>(op, tile) : pick_tile<PREC_FP64, false>(op, tile);
  else if (prec == PREC_FP32) fn = cplx ? pick_tile<PREC_FP32, true>(op, tile) : pick_tile<PREC_FP32, false>(op, tile);
  else if (prec == PREC_BF16X3) fn = cplx ? pick_tile<PREC_BF16X3, true>(op, tile) : pick_tile<PREC_BF16X3, false>(op, tile);
  if (!fn) return hipErrorInvalidValue;
  const int nreal = cplx ? 2 * nmax : nmax;
  dim3 grid((nreal + kTileN[tile] - 1) / kTileN[tile], (mmax + kTileM[tile] - 1) / kTileM[tile], args.ngroup);
  ContractArgs a = args;
  void* kp[] = {&a};
  const hipError_t e = hipLaunchKernel(fn, grid, dim3(256), kp, 0, s);
  if (e != hipSuccess) (void)hipGetLastError();
  return e;
}

}  // namespace aci
