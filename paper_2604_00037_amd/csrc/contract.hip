// Dense contractions of the local update on the matrix cores.
//
// Environment contractions A = L_{l-1} X_l and B = X_{l+1} R_{l+2} and the
// two-site tensors Pi^n = A^n B^n (Eq. pifromframes), with the elementwise f
// of Eq. (localupdate) applied in the epilogue so that Pi = f(Pi^1..Pi^N) is
// written once.  Each workgroup computes a 64x64 output tile; its four waves
// each own a 32x32 quarter made of 2x2 blocks of 16x16 MFMA tiles.  Operands
// are FP64 in HBM and the result is written in FP64 in every precision:
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

constexpr int TM = 64;
constexpr int TN = 64;
constexpr int KC = 32;        // k per staged chunk (every precision)
constexpr int LDA_S = TM + 2;
constexpr int LDB_S = TN + 2;

// One staged chunk (64 x 32 of A, 32 x 64 of B in the real view) is loaded
// by the 256 threads into registers, eight values of each operand per
// thread, while the previous chunk is multiplied from LDS.
//   A value e of thread t: row t / 4, k 8 (t % 4) + e.
//   B value e, real:    k t / 8,               column 8 (t % 8) + e.
//   B value e, complex: k 2 (t / 16) + e / 4,  column 4 (t % 16) + e % 4;
// complex B is read once per element (two neighbouring elements per thread)
// and expanded in registers into its 2 x 2 real block.
__device__ __forceinline__ int a_row(int t) { return t >> 2; }
__device__ __forceinline__ int a_k(int t, int e) { return ((t & 3) << 3) + e; }
template <bool CPLX>
__device__ __forceinline__ int b_k(int t, int e) { return CPLX ? 2 * (t >> 4) + (e >> 2) : t >> 3; }
template <bool CPLX>
__device__ __forceinline__ int b_col(int t, int e) { return CPLX ? ((t & 15) << 2) + (e & 3) : ((t & 7) << 3) + e; }

template <bool CPLX>
__device__ __forceinline__ void load_chunk(const Term& T, int M, int N, int K, int lda, int ldb, int m0, int n0,
                                           int k0, int t, double (&av)[8], double (&bv)[8]) {
  const int gr = m0 + a_row(t);
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int gk = k0 + a_k(t, e);
    av[e] = (gr < M && gk < K) ? T.A[(size_t)gr * lda + gk] : 0.0;
  }
  if (!CPLX) {
    const int gk = k0 + b_k<false>(t, 0);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int gc = n0 + b_col<false>(t, e);
      bv[e] = (gk < K && gc < N) ? T.B[(size_t)gk * ldb + gc] : 0.0;
    }
  } else {
    // complex row (k0 + 2 (t / 16)) / 2, columns (n0 + 4 (t % 16)) / 2 + q
    const int ct = (k0 >> 1) + (t >> 4);
    const int cj = (n0 >> 1) + ((t & 15) << 1);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      double re = 0.0, im = 0.0;
      if (2 * ct < K && 2 * (cj + q) < N) {
        const double* e = T.B + 2 * ((size_t)ct * ldb + cj + q);
        re = e[0];
        im = e[1];
      }
      bv[2 * q] = re;         // real row 2ct:     (re, im)
      bv[2 * q + 1] = im;
      bv[4 + 2 * q] = -im;    // real row 2ct + 1: (-im, re)
      bv[4 + 2 * q + 1] = re;
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

template <int OP, bool CPLX>
__global__ __launch_bounds__(256) void contract_kernel(ContractArgs args) {
  __shared__ double sA[KC * LDA_S];
  __shared__ double sB[KC * LDB_S];
  constexpr int W = CPLX ? 2 : 1;
  const Group& g = args.g[blockIdx.z];
  const int M = dget(g.M);
  const int N = W * dget(g.N);
  const int m0 = blockIdx.y * TM;
  const int n0 = blockIdx.x * TN;
  if (m0 >= M || n0 >= N) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15, lk = lane >> 4;

  const bool even = (lr & 1) == 0;
  v4d res[2][2];
  for (int t = 0; t < g.nterm; ++t) {
    const Term& T = g.t[t];
    const int K = W * dget(T.K);
    const int lda = W * dget(T.lda);
    const int ldb = dget(T.ldb);
    v4d acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    double av[8], bv[8];
    load_chunk<CPLX>(T, M, N, K, lda, ldb, m0, n0, 0, tid, av, bv);
    for (int k0 = 0; k0 < K; k0 += KC) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        sA[a_k(tid, e) * LDA_S + a_row(tid)] = av[e];
        sB[b_k<CPLX>(tid, e) * LDB_S + b_col<CPLX>(tid, e)] = bv[e];
      }
      __syncthreads();
      // the next chunk's loads are in flight while this one is multiplied
      if (k0 + KC < K) load_chunk<CPLX>(T, M, N, K, lda, ldb, m0, n0, k0 + KC, tid, av, bv);
#pragma unroll
      for (int ks = 0; ks < KC / 4; ++ks) {
        const int kr = ks * 4 + lk;
        double a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = sA[kr * LDA_S + wm * 32 + i * 16 + lr];
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = sB[kr * LDB_S + wn * 32 + j * 16 + lr];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
      }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        if (OP == OP_ABS2_MUL) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double x = acc[i][j][v];
            const double xo = CPLX ? __shfl_xor(x, 1) : x;
            res[i][j][v] = abs2_mul<CPLX>(x, xo, even);
          }
        } else if (OP == OP_NONE || t == 0) {
          res[i][j] = acc[i][j];
        } else if (CPLX && OP == OP_PRODUCT) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double r0 = res[i][j][v], a0 = acc[i][j][v];
            const double ro = __shfl_xor(r0, 1), ao = __shfl_xor(a0, 1);
            res[i][j][v] = cplx_combine<OP>(r0, ro, a0, ao, even);
          }
        } else {
          res[i][j] = combine<OP>(res[i][j], acc[i][j]);
        }
      }
  }

  const int ldc = W * dget(g.ldc);
  bool bad = false;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * 32 + i * 16 + lk + 4 * v;
        const int col = n0 + wn * 32 + j * 16 + lr;
        if (row < M && col < N) {
          const double x = res[i][j][v];
          if (OP != OP_NONE && !__builtin_isfinite(x)) bad = true;
          g.C[(size_t)row * ldc + col] = x;
        }
      }
  if (OP != OP_NONE && bad && args.err) atomicOr(args.err, ERR_NONFINITE);
}

// ---------------------------------------------------------------- FP32 / BF16x3
constexpr int KL = 2 * KC;    // k per staged chunk: two load chunks (the
                              // low-precision products are cheaper per k)
constexpr int LDF = TM + 4;   // FP32 tiles, k-major rows of 64 (+pad)
constexpr int LDH = KL + 8;   // bf16 tiles, 64 k per row/column (+pad; 16-byte rows)

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// Round-to-nearest-even FP32 -> bf16 bits (finite inputs; a non-finite
// input stays non-finite, which the epilogue flags).
__device__ __forceinline__ unsigned short bf16_bits(float x) {
  const unsigned int u = __float_as_uint(x);
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_value(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

template <int PREC>
struct LpTiles;

template <>
struct LpTiles<PREC_FP32> {
  float A[KL * LDF];   // [k][row]
  float B[KL * LDF];   // [k][col]
};

template <>
struct LpTiles<PREC_BF16X3> {
  unsigned short Ah[TM * LDH], Al[TM * LDH];   // [row][k]
  unsigned short Bh[TN * LDH], Bl[TN * LDH];   // [col][k]
};

template <int OP, int PREC, bool CPLX>
__global__ __launch_bounds__(256) void contract_lp_kernel(ContractArgs args) {
  __shared__ LpTiles<PREC> sh;
  constexpr int W = CPLX ? 2 : 1;
  const Group& g = args.g[blockIdx.z];
  const int M = dget(g.M);
  const int N = W * dget(g.N);
  const int m0 = blockIdx.y * TM;
  const int n0 = blockIdx.x * TN;
  if (m0 >= M || n0 >= N) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15, lg = lane >> 4;
  const bool even = (lr & 1) == 0;

  v4d res[2][2];
  for (int t = 0; t < g.nterm; ++t) {
    const Term& T = g.t[t];
    const int K = W * dget(T.K);
    const int lda = W * dget(T.lda);
    const int ldb = dget(T.ldb);
    v4f acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

    double av[2][8], bv[2][8];
    load_chunk<CPLX>(T, M, N, K, lda, ldb, m0, n0, 0, tid, av[0], bv[0]);
    load_chunk<CPLX>(T, M, N, K, lda, ldb, m0, n0, KC, tid, av[1], bv[1]);
    for (int k0 = 0; k0 < K; k0 += KL) {
      const int ar = a_row(tid);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int kh = KC * h;
        if (PREC == PREC_FP32) {
          auto& S = reinterpret_cast<LpTiles<PREC_FP32>&>(sh);
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            S.A[(kh + a_k(tid, e)) * LDF + ar] = (float)av[h][e];
            S.B[(kh + b_k<CPLX>(tid, e)) * LDF + b_col<CPLX>(tid, e)] = (float)bv[h][e];
          }
        } else {
          auto& S = reinterpret_cast<LpTiles<PREC_BF16X3>&>(sh);
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int ak = kh + a_k(tid, e);
            const float fa = (float)av[h][e];
            const unsigned short ha = bf16_bits(fa);
            S.Ah[ar * LDH + ak] = ha;
            S.Al[ar * LDH + ak] = bf16_bits(fa - bf16_value(ha));
            const int bk = kh + b_k<CPLX>(tid, e), bc = b_col<CPLX>(tid, e);
            const float fb = (float)bv[h][e];
            const unsigned short hb = bf16_bits(fb);
            S.Bh[bc * LDH + bk] = hb;
            S.Bl[bc * LDH + bk] = bf16_bits(fb - bf16_value(hb));
          }
        }
      }
      __syncthreads();
      // the next chunk's loads are in flight while this one is multiplied
      if (k0 + KL < K) {
        load_chunk<CPLX>(T, M, N, K, lda, ldb, m0, n0, k0 + KL, tid, av[0], bv[0]);
        load_chunk<CPLX>(T, M, N, K, lda, ldb, m0, n0, k0 + KL + KC, tid, av[1], bv[1]);
      }
      if (PREC == PREC_FP32) {
        auto& S = reinterpret_cast<LpTiles<PREC_FP32>&>(sh);
#pragma unroll
        for (int ks = 0; ks < KL / 4; ++ks) {
          const int kr = ks * 4 + lg;
          float a[2], b[2];
#pragma unroll
          for (int i = 0; i < 2; ++i) a[i] = S.A[kr * LDF + wm * 32 + i * 16 + lr];
#pragma unroll
          for (int j = 0; j < 2; ++j) b[j] = S.B[kr * LDF + wn * 32 + j * 16 + lr];
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
      } else {
        auto& S = reinterpret_cast<LpTiles<PREC_BF16X3>&>(sh);
#pragma unroll
        for (int ks = 0; ks < KL / 32; ++ks) {
          v8bf ah[2], al[2], bh[2], bl[2];
#pragma unroll
          for (int i = 0; i < 2; ++i) {
            const int row = wm * 32 + i * 16 + lr;
            ah[i] = *reinterpret_cast<const v8bf*>(&S.Ah[row * LDH + 32 * ks + 8 * lg]);
            al[i] = *reinterpret_cast<const v8bf*>(&S.Al[row * LDH + 32 * ks + 8 * lg]);
          }
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            const int col = wn * 32 + j * 16 + lr;
            bh[j] = *reinterpret_cast<const v8bf*>(&S.Bh[col * LDH + 32 * ks + 8 * lg]);
            bl[j] = *reinterpret_cast<const v8bf*>(&S.Bl[col * LDH + 32 * ks + 8 * lg]);
          }
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
            }
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const v4d x = v4d{(double)acc[i][j][0], (double)acc[i][j][1], (double)acc[i][j][2], (double)acc[i][j][3]};
        if (OP == OP_ABS2_MUL) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double xv = x[v];
            const double xo = CPLX ? __shfl_xor(xv, 1) : xv;
            res[i][j][v] = abs2_mul<CPLX>(xv, xo, even);
          }
        } else if (OP == OP_NONE || t == 0) {
          res[i][j] = x;
        } else if (CPLX && OP == OP_PRODUCT) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double r0 = res[i][j][v], a0 = x[v];
            const double ro = __shfl_xor(r0, 1), ao = __shfl_xor(a0, 1);
            res[i][j][v] = cplx_combine<OP>(r0, ro, a0, ao, even);
          }
        } else {
          res[i][j] = combine<OP>(res[i][j], x);
        }
      }
  }

  const int ldc = W * dget(g.ldc);
  bool bad = false;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * 32 + i * 16 + 4 * lg + v;
        const int col = n0 + wn * 32 + j * 16 + lr;
        if (row < M && col < N) {
          const double x = res[i][j][v];
          if (OP != OP_NONE && !__builtin_isfinite(x)) bad = true;
          g.C[(size_t)row * ldc + col] = x;
        }
      }
  if (OP != OP_NONE && bad && args.err) atomicOr(args.err, ERR_NONFINITE);
}

template <int PREC, bool CPLX>
hipError_t launch_prec(int op, const ContractArgs& args, dim3 grid, dim3 block, hipStream_t s) {
  switch (op) {
    case OP_NONE: hipLaunchKernelGGL((contract_lp_kernel<OP_NONE, PREC, CPLX>), grid, block, 0, s, args); break;
    case OP_PRODUCT: hipLaunchKernelGGL((contract_lp_kernel<OP_PRODUCT, PREC, CPLX>), grid, block, 0, s, args); break;
    case OP_SUM: hipLaunchKernelGGL((contract_lp_kernel<OP_SUM, PREC, CPLX>), grid, block, 0, s, args); break;
    case OP_ABS2_MUL: hipLaunchKernelGGL((contract_lp_kernel<OP_ABS2_MUL, PREC, CPLX>), grid, block, 0, s, args); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <bool CPLX>
hipError_t launch_fp64(int op, const ContractArgs& args, dim3 grid, dim3 block, hipStream_t s) {
  switch (op) {
    case OP_NONE: hipLaunchKernelGGL((contract_kernel<OP_NONE, CPLX>), grid, block, 0, s, args); break;
    case OP_PRODUCT: hipLaunchKernelGGL((contract_kernel<OP_PRODUCT, CPLX>), grid, block, 0, s, args); break;
    case OP_SUM: hipLaunchKernelGGL((contract_kernel<OP_SUM, CPLX>), grid, block, 0, s, args); break;
    case OP_ABS2_MUL: hipLaunchKernelGGL((contract_kernel<OP_ABS2_MUL, CPLX>), grid, block, 0, s, args); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_contract(int op, int prec, const ContractArgs& args, int mmax, int nmax, hipStream_t s) {
  if (mmax <= 0 || nmax <= 0 || args.ngroup <= 0) return hipSuccess;
  const bool cplx = args.cplx != 0;
  const int nreal = cplx ? 2 * nmax : nmax;
  dim3 grid((nreal + TN - 1) / TN, (mmax + TM - 1) / TM, args.ngroup);
  dim3 block(256);
  if (prec == PREC_FP32) return cplx ? launch_prec<PREC_FP32, true>(op, args, grid, block, s)
                                     : launch_prec<PREC_FP32, false>(op, args, grid, block, s);
  if (prec == PREC_BF16X3) return cplx ? launch_prec<PREC_BF16X3, true>(op, args, grid, block, s)
                                       : launch_prec<PREC_BF16X3, false>(op, args, grid, block, s);
  if (prec != PREC_FP64) return hipErrorInvalidValue;
  return cplx ? launch_fp64<true>(op, args, grid, block, s) : launch_fp64<false>(op, args, grid, block, s);
}

}  // namespace aci
