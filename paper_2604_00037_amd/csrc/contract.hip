// Dense contractions of the local update on the FP64 matrix cores.
//
// Environment contractions A = L_{l-1} X_l and B = X_{l+1} R_{l+2} and the
// two-site tensors Pi^n = A^n B^n (Eq. pifromframes), with the elementwise f
// of Eq. (localupdate) applied in the epilogue so that Pi = f(Pi^1..Pi^N) is
// written once.  Each workgroup computes a 64x64 output tile; its four waves
// each own a 32x32 quarter made of 2x2 blocks of v_mfma_f64_16x16x4f64.
// Operand tiles of 64x16 (A, stored k-major) and 16x64 (B) are staged through
// LDS so that every lane of an MFMA reads consecutive doubles.
//
// v_mfma_f64_16x16x4f64 lane layout (measured on gfx950): lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; accumulator item v of lane l is
// C[l/16 + 4v][l%16].
#include "kernels.h"

namespace aci {

namespace {

constexpr int TM = 64;
constexpr int TN = 64;
constexpr int KC = 16;
constexpr int LDA_S = TM + 2;
constexpr int LDB_S = TN + 2;

template <int OP>
__device__ __forceinline__ v4d combine(v4d r, v4d a) {
  if (OP == OP_PRODUCT) return r * a;
  return r + a;  // OP_SUM
}

template <int OP>
__global__ __launch_bounds__(256) void contract_kernel(ContractArgs args) {
  __shared__ double sA[KC * LDA_S];
  __shared__ double sB[KC * LDB_S];
  const Group& g = args.g[blockIdx.z];
  const int M = dget(g.M);
  const int N = dget(g.N);
  const int m0 = blockIdx.y * TM;
  const int n0 = blockIdx.x * TN;
  if (m0 >= M || n0 >= N) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = lane & 15, lk = lane >> 4;

  v4d res[2][2];
  for (int t = 0; t < g.nterm; ++t) {
    const Term& T = g.t[t];
    const int K = dget(T.K);
    const int lda = dget(T.lda);
    const int ldb = dget(T.ldb);
    v4d acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    for (int k0 = 0; k0 < K; k0 += KC) {
      // A tile: 64 rows x 16 k, thread -> row tid/4, k (tid%4)*4 .. +3
      {
        const int r = tid >> 2;
        const int kq = (tid & 3) * 4;
        const int gr = m0 + r;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int gk = k0 + kq + e;
          double v = 0.0;
          if (gr < M && gk < K) v = T.A[(size_t)gr * lda + gk];
          sA[(kq + e) * LDA_S + r] = v;
        }
      }
      // B tile: 16 k x 64 cols, thread -> k tid/16, cols (tid%16)*4 .. +3
      {
        const int kk = tid >> 4;
        const int cq = (tid & 15) * 4;
        const int gk = k0 + kk;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int gc = n0 + cq + e;
          double v = 0.0;
          if (gk < K && gc < N) v = T.B[(size_t)gk * ldb + gc];
          sB[kk * LDB_S + cq + e] = v;
        }
      }
      __syncthreads();
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
          res[i][j] = (acc[i][j] * acc[i][j]) * acc[i][j];
        } else if (OP == OP_NONE || t == 0) {
          res[i][j] = acc[i][j];
        } else {
          res[i][j] = combine<OP>(res[i][j], acc[i][j]);
        }
      }
  }

  const int ldc = dget(g.ldc);
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

}  // namespace

hipError_t launch_contract(int op, const ContractArgs& args, int mmax, int nmax, hipStream_t s) {
  if (mmax <= 0 || nmax <= 0 || args.ngroup <= 0) return hipSuccess;
  dim3 grid((nmax + TN - 1) / TN, (mmax + TM - 1) / TM, args.ngroup);
  dim3 block(256);
  switch (op) {
    case OP_NONE: hipLaunchKernelGGL(contract_kernel<OP_NONE>, grid, block, 0, s, args); break;
    case OP_PRODUCT: hipLaunchKernelGGL(contract_kernel<OP_PRODUCT>, grid, block, 0, s, args); break;
    case OP_SUM: hipLaunchKernelGGL(contract_kernel<OP_SUM>, grid, block, 0, s, args); break;
    case OP_ABS2_MUL: hipLaunchKernelGGL(contract_kernel<OP_ABS2_MUL>, grid, block, 0, s, args); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace aci
