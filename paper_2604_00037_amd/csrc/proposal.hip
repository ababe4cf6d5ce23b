// Learned pivot proposal (an extension of the method): row features of the
// two-site matrix, a 7 -> 64 -> 64 -> 1 scoring network (inference and one
// Adam training step), a rook search with lazy residuals seeded by the
// scores, the dense residual check that accepts or rejects its result, and
// the right factor B = T^{-1} Up of an accepted search.
//
// Every reduction here runs in a fixed index order inside one workgroup, so
// results do not depend on timing.  Floating-point contraction is off: the
// network layers accumulate fp32(x16 * w16) products in index order (the
// products of two float16 values are exact in float32), and the residuals
// are M[i, j] - L[i, t] Up[t, j] term by term with the product rounded first.
#include <climits>

#include <hip/hip_fp16.h>

#include "kernels.h"

#pragma clang fp contract(off)

namespace aci {

namespace {

constexpr int NT = 256;
constexpr int NF = MLP_FEATURES;
constexpr int HD = MLP_HIDDEN;

__device__ __forceinline__ float f16r(float x) { return __half2float(__float2half_rn(x)); }

// parameter blocks of the flat network array
struct Net {
  const float* W1;  // NF x HD
  const float* b1;  // HD
  const float* W2;  // HD x HD
  const float* b2;  // HD
  const float* w3;  // HD
  const float* b3;  // 1
};
__device__ __forceinline__ Net net_of(const float* p) {
  Net n;
  n.W1 = p;
  n.b1 = n.W1 + NF * HD;
  n.W2 = n.b1 + HD;
  n.b2 = n.W2 + HD * HD;
  n.w3 = n.b2 + HD;
  n.b3 = n.w3 + HD;
  return n;
}

// ---------------------------------------------------------------- features
// One workgroup.  f0, f1: row 2-norms of the environments over their
// maxima; f2: previous pivot rows; f3..f6: |M| at four sample columns over
// their maximum.  Norms in float64, features rounded to float32.
__global__ __launch_bounds__(NT) void features_kernel(FeatureArgs a) {
  __shared__ double red[NT];
  const int m = dget(a.m), n = dget(a.n), ldm = dget(a.ldm);
  const int tid = threadIdx.x;
  for (int i = tid; i < m; i += NT)
    for (int f = 0; f < NF; ++f) a.X[(size_t)i * NF + f] = 0.f;
  __syncthreads();
  for (int t = 0; t < 2; ++t) {
    if (t >= a.n_env) break;
    const int w = dget(a.env_w[t]);
    const int lde = dget(a.env_ld[t]);
    double mx = 0.0;
    for (int i = tid; i < m; i += NT) {
      double s = 0.0;
      for (int c = 0; c < w; ++c) {
        const double v = a.env[t][(size_t)i * lde + c];
        s = s + v * v;
      }
      mx = fmax(mx, sqrt(s));
    }
    red[tid] = mx;
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
      if (tid < h) red[tid] = fmax(red[tid], red[tid + h]);
      __syncthreads();
    }
    const double gmax = red[0];
    __syncthreads();
    if (gmax > 0.0)
      for (int i = tid; i < m; i += NT) {
        double s = 0.0;
        for (int c = 0; c < w; ++c) {
          const double v = a.env[t][(size_t)i * lde + c];
          s = s + v * v;
        }
        a.X[(size_t)i * NF + t] = (float)(sqrt(s) / gmax);
      }
  }
  const int np = a.prev_rank ? *a.prev_rank : 0;
  for (int q = tid; q < np; q += NT) {
    const int i = a.prev_rows[q];
    if (i >= 0 && i < m) a.X[(size_t)i * NF + 2] = 1.f;
  }
  int cols[4];
  for (int t = 0; t < 4; ++t) cols[t] = ((2 * t + 1) * n) / 8;
  double mx = 0.0;
  for (int i = tid; i < m; i += NT)
    for (int t = 0; t < 4; ++t) mx = fmax(mx, fabs(a.M[(size_t)i * ldm + cols[t]]));
  red[tid] = mx;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] = fmax(red[tid], red[tid + h]);
    __syncthreads();
  }
  const double gmax = red[0];
  if (gmax > 0.0)
    for (int i = tid; i < m; i += NT)
      for (int t = 0; t < 4; ++t) a.X[(size_t)i * NF + 3 + t] = (float)(fabs(a.M[(size_t)i * ldm + cols[t]]) / gmax);
}

// ---------------------------------------------------------------- network
// Forward pass of one sample (thread), weights staged in LDS as float16
// values.  Writes the pre-activations and rounded activations when asked.
struct Stage {
  float W1[NF * HD];
  float b1[HD];
  float W2[HD * HD];
  float b2[HD];
  float w3[HD];
  float b3;
};

__device__ void stage_weights(const float* params, Stage& S) {
  const Net p = net_of(params);
  for (int i = threadIdx.x; i < NF * HD; i += blockDim.x) S.W1[i] = f16r(p.W1[i]);
  for (int i = threadIdx.x; i < HD * HD; i += blockDim.x) S.W2[i] = f16r(p.W2[i]);
  for (int i = threadIdx.x; i < HD; i += blockDim.x) {
    S.b1[i] = p.b1[i];
    S.b2[i] = p.b2[i];
    S.w3[i] = f16r(p.w3[i]);
  }
  if (threadIdx.x == 0) S.b3 = p.b3[0];
}

// z1, a1_16, z2, a2_16 may be null
__device__ float forward_one(const Stage& S, const float* x, float* z1o, float* a1o, float* z2o, float* a2o) {
  float xi[NF];
  for (int k = 0; k < NF; ++k) xi[k] = f16r(x[k]);
  float a1[HD];
  for (int o = 0; o < HD; ++o) {
    float acc = 0.f;
    for (int k = 0; k < NF; ++k) acc = acc + xi[k] * S.W1[k * HD + o];
    const float z = acc + S.b1[o];
    if (z1o) z1o[o] = z;
    a1[o] = f16r(z > 0.f ? z : 0.f);
    if (a1o) a1o[o] = a1[o];
  }
  float acc3 = 0.f;
  for (int o = 0; o < HD; ++o) {
    float acc = 0.f;
    for (int k = 0; k < HD; ++k) acc = acc + a1[k] * S.W2[k * HD + o];
    const float z = acc + S.b2[o];
    if (z2o) z2o[o] = z;
    const float a2 = f16r(z > 0.f ? z : 0.f);
    if (a2o) a2o[o] = a2;
    acc3 = acc3 + a2 * S.w3[o];
  }
  return acc3 + S.b3;
}

__global__ __launch_bounds__(NT) void mlp_forward_kernel(const float* params, const float* X, int count,
                                                         float* out) {
  __shared__ Stage S;
  stage_weights(params, S);
  __syncthreads();
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < count; s += gridDim.x * blockDim.x)
    out[s] = forward_one(S, X + (size_t)s * NF, nullptr, nullptr, nullptr, nullptr);
}

// One Adam step on a minibatch, in one workgroup.  scratch holds per
// sample z1, a1_16, z2, a2_16, dz2 and dz1 (6 * HD floats) and dz3.
__global__ __launch_bounds__(NT) void mlp_train_kernel(TrainArgs a) {
  __shared__ Stage S;
  __shared__ float lossred[NT];
  stage_weights(a.params, S);
  __syncthreads();
  const int B = a.count;
  const int tid = threadIdx.x;
  float* z1 = a.scratch;
  float* a1 = z1 + (size_t)B * HD;
  float* z2 = a1 + (size_t)B * HD;
  float* a2 = z2 + (size_t)B * HD;
  float* dz2 = a2 + (size_t)B * HD;
  float* dz1 = dz2 + (size_t)B * HD;
  float* dz3 = dz1 + (size_t)B * HD;
  const float om1 = a.one_minus_beta1, om2 = a.one_minus_beta2;
  float lsum = 0.f;
  for (int s = tid; s < B; s += NT) {
    const float z = forward_one(S, a.X + (size_t)s * NF, z1 + (size_t)s * HD, a1 + (size_t)s * HD,
                                z2 + (size_t)s * HD, a2 + (size_t)s * HD);
    const double zd = (double)z;
    const float sig = (float)(1.0 / (1.0 + exp(-zd)));
    dz3[s] = (sig - a.y[s]) / (float)B;
    lsum += (float)(fmax(zd, 0.0) - zd * (double)a.y[s] + log1p(exp(-fabs(zd))));
  }
  lossred[tid] = lsum;
  __syncthreads();
  // dz2[s, o] = relu'(z2) * dz3[s] * w3_16[o]
  for (int idx = tid; idx < B * HD; idx += NT) {
    const int s = idx / HD, o = idx % HD;
    const float d = dz3[s] * S.w3[o];
    dz2[idx] = z2[idx] > 0.f ? d : 0.f;
  }
  __syncthreads();
  // dz1[s, k] = relu'(z1) * sum_o dz2[s, o] W2_16[k, o]  (o order)
  for (int idx = tid; idx < B * HD; idx += NT) {
    const int s = idx / HD, k = idx % HD;
    float acc = 0.f;
    for (int o = 0; o < HD; ++o) acc = acc + dz2[(size_t)s * HD + o] * S.W2[k * HD + o];
    dz1[idx] = z1[idx] > 0.f ? acc : 0.f;
  }
  __syncthreads();
  // gradients (sums over samples in order) and the Adam update, parameter
  // by parameter in the flat layout
  const int total = MLP_PARAMS;
  const float b1c = a.beta1, b2c = a.beta2;
  for (int q = tid; q < total; q += NT) {
    float g = 0.f;
    if (q < NF * HD) {                       // W1[k, o]
      const int k = q / HD, o = q % HD;
      for (int s = 0; s < B; ++s) g = g + f16r(a.X[(size_t)s * NF + k]) * dz1[(size_t)s * HD + o];
    } else if (q < NF * HD + HD) {           // b1[o]
      const int o = q - NF * HD;
      for (int s = 0; s < B; ++s) g = g + dz1[(size_t)s * HD + o];
    } else if (q < NF * HD + HD + HD * HD) {  // W2[k, o]
      const int r = q - NF * HD - HD;
      const int k = r / HD, o = r % HD;
      for (int s = 0; s < B; ++s) g = g + a1[(size_t)s * HD + k] * dz2[(size_t)s * HD + o];
    } else if (q < NF * HD + 2 * HD + HD * HD) {  // b2[o]
      const int o = q - NF * HD - HD - HD * HD;
      for (int s = 0; s < B; ++s) g = g + dz2[(size_t)s * HD + o];
    } else if (q < NF * HD + 3 * HD + HD * HD) {  // w3[o]
      const int o = q - NF * HD - 2 * HD - HD * HD;
      for (int s = 0; s < B; ++s) g = g + a2[(size_t)s * HD + o] * dz3[s];
    } else {                                  // b3
      for (int s = 0; s < B; ++s) g = g + dz3[s];
    }
    if (a.grads) a.grads[q] = g;
    float& m = a.adam_m[q];
    float& v = a.adam_v[q];
    m = b1c * m + om1 * g;
    v = b2c * v + om2 * (g * g);
    const float mh = m / a.c1;
    const float vh = v / a.c2;
    a.params[q] = a.params[q] - (a.lr * mh) / (sqrtf(vh) + a.eps);
  }
  __syncthreads();
  if (tid == 0 && a.loss) {
    float t = 0.f;
    for (int i = 0; i < NT; ++i) t += lossred[i];
    *a.loss = t / (float)B;
  }
}

// --------------------------------------------------------------- rook LDU
// Argmax of |v| over the workgroup: largest value, then smallest index.
__device__ void block_argmax(double v, int i, double* sv, int* si, double& bv, int& bi) {
  const int tid = threadIdx.x;
  sv[tid] = v;
  si[tid] = i;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if (tid < h) {
      const double ov = sv[tid + h];
      const int oi = si[tid + h];
      if (ov > sv[tid] || (ov == sv[tid] && oi < si[tid])) {
        sv[tid] = ov;
        si[tid] = oi;
      }
    }
    __syncthreads();
  }
  bv = sv[0];
  bi = si[0];
  __syncthreads();
}

__global__ __launch_bounds__(NT) void rook_kernel(RookArgs a) {
  __shared__ double sv[NT];
  __shared__ int si[NT];
  extern __shared__ unsigned char flags_lds[];
  unsigned char* prow = flags_lds;                  // m
  unsigned char* pcol = flags_lds + ACI_MAX_MATRIX;  // n
  const int m = dget(a.m), n = dget(a.n), ldm = dget(a.ldm);
  const int ldl = a.ldl, ldu = a.ldu;
  const int tid = threadIdx.x;
  for (int i = tid; i < m; i += NT) prow[i] = 0;
  for (int j = tid; j < n; j += NT) pcol[j] = 0;
  __syncthreads();
  const int kstop = m < n ? m : n;
  int k = 0, scans = 0;
  double eps = 0.0;
  while (k < kstop) {
    // start row: best score among free rows (ties: smallest), or the first free row
    double sb = -INFINITY;
    int ib = INT_MAX;
    for (int i = tid; i < m; i += NT)
      if (!prow[i]) {
        const double sc = a.scores ? (double)a.scores[i] : 0.0;
        if (sc > sb || (sc == sb && i < ib)) {
          sb = sc;
          ib = i;
        }
      }
    double bv;
    int i0;
    block_argmax(sb, ib, sv, si, bv, i0);
    int j0 = 0;
    double piv = 0.0;
    for (int it = 0;;) {
      // residual row i0 into Up[k, :]; its argmax over free columns
      double rb = -1.0;
      int jb = INT_MAX;
      for (int j = tid; j < n; j += NT) {
        double acc = 0.0;
        if (!pcol[j]) {
          acc = a.M[(size_t)i0 * ldm + j];
          for (int t = 0; t < k; ++t) acc = acc - a.L[(size_t)i0 * ldl + t] * a.Up[(size_t)t * ldu + j];
        }
        if (k < a.maxrank) a.Up[(size_t)k * ldu + j] = acc;
        const double av = fabs(acc);
        if (av > rb || (av == rb && j < jb)) {
          rb = av;
          jb = j;
        }
      }
      block_argmax(rb, jb, sv, si, bv, j0);
      // residual column j0 into L[:, k]; its argmax over free rows
      double cb = -1.0;
      int ic = INT_MAX;
      for (int i = tid; i < m; i += NT) {
        double acc = 0.0;
        if (!prow[i] && !pcol[j0]) {
          acc = a.M[(size_t)i * ldm + j0];
          for (int t = 0; t < k; ++t) acc = acc - a.L[(size_t)i * ldl + t] * a.Up[(size_t)t * ldu + j0];
        }
        if (k < a.maxrank) a.L[(size_t)i * ldl + k] = acc;
        const double av = fabs(acc);
        if (av > cb || (av == cb && i < ic)) {
          cb = av;
          ic = i;
        }
      }
      int i1;
      block_argmax(cb, ic, sv, si, bv, i1);
      scans += 2;
      ++it;
      if (i1 == i0 || it >= a.max_iter) break;
      i0 = i1;
    }
    // pivot value: the residual of (i0, j0) as held in L[:, k] (column scan)
    if (k < a.maxrank) piv = a.L[(size_t)i0 * ldl + k];
    else {
      // at the rank cap the column was not stored: recompute the entry
      double acc = a.M[(size_t)i0 * ldm + j0];
      for (int t = 0; t < k; ++t) acc = acc - a.L[(size_t)i0 * ldl + t] * a.Up[(size_t)t * ldu + j0];
      piv = acc;
    }
    __syncthreads();
    const double v = fabs(piv);
    if (k == a.maxrank) { eps = v; break; }
    if (k >= 1 && v <= a.tol) { eps = v; break; }
    if (v == 0.0) {
      // all-zero matrix at k == 0: one pivot, L = e_i0, Up = 0
      for (int i = tid; i < m; i += NT) a.L[(size_t)i * ldl] = (i == i0) ? 1.0 : 0.0;
      for (int j = tid; j < n; j += NT) a.Up[j] = 0.0;
      if (tid == 0) {
        a.rows[0] = i0;
        a.cols[0] = j0;
      }
      k = 1;
      eps = 0.0;
      break;
    }
    for (int i = tid; i < m; i += NT) {
      const double c = a.L[(size_t)i * ldl + k];
      a.L[(size_t)i * ldl + k] = (i == i0) ? 1.0 : c / piv;
    }
    if (tid == 0) {
      a.rows[k] = i0;
      a.cols[k] = j0;
      prow[i0] = 1;
      pcol[j0] = 1;
    }
    __syncthreads();
    ++k;
  }
  if (tid == 0) {
    *a.rank = k;
    *a.eps = eps;
    if (a.scans) *a.scans = scans;
  }
}

// ------------------------------------------------------- residual check
// eps = max |M - C| over the m x n block (C = L Up from the contraction);
// accepted = (eps <= tol).
__global__ __launch_bounds__(NT) void check_kernel(CheckArgs a) {
  __shared__ double red[NT];
  const int m = dget(a.m), n = dget(a.n), ldm = dget(a.ldm);
  double mx = 0.0;
  for (size_t q = threadIdx.x; q < (size_t)m * n; q += NT) {
    const size_t i = q / n, j = q % n;
    mx = fmax(mx, fabs(a.M[i * ldm + j] - a.C[i * a.ldc + j]));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int ok = red[0] <= a.tol ? 1 : 0;
    *a.eps = red[0];
    a.accepted[0] = ok;
    a.accepted[1] = 1 - ok;
    if (ok && a.count) atomicAdd(a.count, 1);
  }
}

__global__ void commit_kernel(CommitArgs a) {
  if (a.scan_total && threadIdx.x == 0) {
    a.scan_total[0] += *a.src_scans;
    a.scan_total[1] += *a.src_rank;
  }
  if (!*a.accepted) return;
  const int r = *a.src_rank;
  for (int k = threadIdx.x; k < r && k < a.maxrank; k += blockDim.x) {
    a.rows[k] = a.src_rows[k];
    a.cols[k] = a.src_cols[k];
  }
  if (threadIdx.x == 0) {
    const double e = *a.src_eps;
    *a.rank = r;
    *a.eps = e;
    if (a.rank2) *a.rank2 = r;
    if (a.eps2) *a.eps2 = e;
    if (a.meta) {
      a.meta[0] = r;
      a.meta[1] = dget(a.m);
      a.meta[2] = dget(a.n);
    }
    if (a.meta2) {
      a.meta2[0] = r;
      a.meta2[1] = dget(a.m);
      a.meta2[2] = dget(a.n);
    }
  }
}

__global__ void copy_rows_kernel(CopyRowsArgs a) {
  const int r = *a.rank;
  for (int k = threadIdx.x; k < r && k < a.maxrank; k += blockDim.x) a.dst[k] = a.src[k];
  if (threadIdx.x == 0) *a.dst_rank = r < a.maxrank ? r : a.maxrank;
}

// Training rows of one local update (one workgroup): features and pivot
// labels appended at the dataset's current end.
__global__ __launch_bounds__(NT) void record_kernel(RecordArgs a) {
  const long long off = a.count[0];
  const int m = dget(a.m);
  if (a.count[1] != 0 || off + m > a.capacity) {
    if (threadIdx.x == 0) a.count[1] = 1;
    return;
  }
  for (int i = threadIdx.x; i < m; i += NT) {
    for (int f = 0; f < NF; ++f) a.X[(size_t)(off + i) * NF + f] = a.feat[(size_t)i * NF + f];
    a.y[off + i] = 0.f;
  }
  __syncthreads();
  const int r = *a.rank;
  const int npos = r / 2 > 1 ? r / 2 : 1;
  for (int k = threadIdx.x; k < npos && k < r; k += NT) {
    const int i = a.rows[k];
    if (i >= 0 && i < m) a.y[off + i] = 1.f;
  }
  if (threadIdx.x == 0) a.count[0] = off + m;
}

// ------------------------------------------------------- right factor
// Y = T^{-1} Up with T = Up[:, J] upper triangular, by back substitution:
// Y[t, j] = (Up[t, j] - sum_{s > t} T[t, s] Y[s, j]) / T[t, t], s ascending.
__global__ __launch_bounds__(NT) void rook_solve_kernel(SolveArgs a) {
  if (a.skip && *a.skip) return;
  const int r = *a.rank;
  const int n = dget(a.n);
  const int ldy = dget(a.ldy);
  for (int t = r - 1; t >= 0; --t) {
    const double d = a.Up[(size_t)t * a.ldu + a.cols[t]];
    for (int j = threadIdx.x; j < n; j += NT) {
      double acc = a.Up[(size_t)t * a.ldu + j];
      for (int s = t + 1; s < r; ++s) acc = acc - a.Up[(size_t)t * a.ldu + a.cols[s]] * a.Y[(size_t)s * ldy + j];
      a.Y[(size_t)t * ldy + j] = d != 0.0 ? acc / d : 0.0;
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_features(const FeatureArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(features_kernel, dim3(1), dim3(NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* params, const float* X, int count, float* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int blocks = (count + NT - 1) / NT;
  if (blocks > 256) blocks = 256;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(blocks), dim3(NT), 0, s, params, X, count, out);
  return hipGetLastError();
}

hipError_t launch_mlp_train(const TrainArgs& a, hipStream_t s) {
  if (a.count <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mlp_train_kernel, dim3(1), dim3(NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_rook(const RookArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(rook_kernel, dim3(1), dim3(NT), 2 * ACI_MAX_MATRIX, s, a);
  return hipGetLastError();
}

hipError_t launch_check(const CheckArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(check_kernel, dim3(1), dim3(NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_rook_solve(const SolveArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(rook_solve_kernel, dim3(1), dim3(NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_commit(const CommitArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(commit_kernel, dim3(1), dim3(NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_copy_rows(const CopyRowsArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(copy_rows_kernel, dim3(1), dim3(NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_record(const RecordArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(record_kernel, dim3(1), dim3(NT), 0, s, a);
  return hipGetLastError();
}

}  // namespace aci
