// 2-site TCI of a function given point by point (the construction of the
// inputs in Sec. 3; the index-set optimisation of Sec. 2.6 with the two-site
// tensor evaluated directly): the multi-indices of a bond's two-site tensor,
// and the update of the nested index sets from the pivots of its LDU.
//
// Index sets live on the device as digit rows of length L (int32): row k of
// I_l holds sigma_1..sigma_l of its k-th multi-index in positions 0..l-1;
// row k of J_l holds sigma_l..sigma_L in positions 0..L-l.
#include <algorithm>

#include "kernels.h"

namespace aci {

namespace {

constexpr int NT = 256;

// pts[p][t], p = row * n + col, row = a d + s, col = s' cR + b:
// I_{l-1}[a] ++ (s, s') ++ J_{l+2}[b]
__global__ __launch_bounds__(NT) void tci_points_kernel(TciPointsArgs a) {
  const int64_t count = (int64_t)a.m * a.n;
  const int L = a.L;
  for (int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x; p < count; p += (int64_t)gridDim.x * NT) {
    const int row = (int)(p / a.n), col = (int)(p % a.n);
    const int ia = row / a.d, s = row % a.d;
    const int s2 = col / a.cR, jb = col % a.cR;
    int32_t* out = a.pts + p * L;
    const int l = a.l;
    for (int t = 0; t < l - 1; ++t) out[t] = a.I_prev[(size_t)ia * L + t];
    out[l - 1] = s;
    out[l] = s2;
    for (int t = l + 1; t < L; ++t) out[t] = a.J_next[(size_t)jb * L + (t - l - 1)];
  }
}

// I_l[k] = I_{l-1}[p_k / d] ++ (p_k mod d);  J_{l+1}[k] = (q_k / cR) ++ J_{l+2}[q_k mod cR]
__global__ __launch_bounds__(NT) void tci_sets_kernel(TciSetsArgs a) {
  const int r = *a.rank;
  const int L = a.L, l = a.l;
  for (int k = blockIdx.x; k < r; k += gridDim.x) {
    const int p = a.rows[k], q = a.cols[k];
    const int ia = p / a.d, s = p % a.d;
    const int s2 = q / a.cR, jb = q % a.cR;
    for (int t = threadIdx.x; t < L; t += NT) {
      a.I_out[(size_t)k * L + t] = t < l - 1 ? a.I_prev[(size_t)ia * L + t] : (t == l - 1 ? s : 0);
      a.J_out[(size_t)k * L + t] = t == 0 ? s2 : (t < L - l ? a.J_next[(size_t)jb * L + t - 1] : 0);
    }
  }
}

}  // namespace

hipError_t launch_tci_points(const TciPointsArgs& a, hipStream_t s) {
  const int64_t count = (int64_t)a.m * a.n;
  if (count <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((count + NT - 1) / NT, 8192);
  hipLaunchKernelGGL(tci_points_kernel, dim3((unsigned)blocks), dim3(NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_tci_sets(const TciSetsArgs& a, int rmax, hipStream_t s) {
  if (rmax <= 0) return hipSuccess;
  hipLaunchKernelGGL(tci_sets_kernel, dim3((unsigned)std::min(rmax, 1024)), dim3(NT), 0, s, a);
  return hipGetLastError();
}

}  // namespace aci
