// Exact contraction of a TT operator (MPO) with a tensor train, the operator
// half of an explicit step of a nonlinear equation (the use of ACI named in
// Sec. 5).  Core by core,
//   Z[(a, c), s, (b, e)] = sum_t W[a, s, t, b] X[c, t, e],
// so the output is w^2 times the input: the kernel is bound by its HBM
// writes.  One wave writes one output row (a, c, s, b), xe contiguous
// doubles; the rows are dealt in the order (c, a, s, b) so that the
// workgroups running together read the same rows of X from L2.
#include "kernels.h"

namespace aci {
namespace {

constexpr int kRowsPerGroup = 4;   // one row per wave of a 256-thread workgroup

__global__ __launch_bounds__(256) void mpo_apply_kernel(MpoArgs args) {
  int si = 0;
  for (int k = 1; k < args.nsite; ++k)
    if ((int)blockIdx.x >= args.site[k].block0) si = k;
  const MpoSite& m = args.site[si];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = ((int)blockIdx.x - m.block0) * kRowsPerGroup + wave;
  if (row >= m.ra * m.wa * m.d * m.wb) return;
  int q = row;
  const int b = q % m.wb;
  q /= m.wb;
  const int s = q % m.d;
  q /= m.d;
  const int a = q % m.wa;
  const int c = q / m.wa;
  double w[ACI_MAX_DIM];
#pragma unroll
  for (int t = 0; t < ACI_MAX_DIM; ++t)
    w[t] = t < m.d ? m.W[((size_t)(a * m.d + s) * m.d + t) * m.wb + b] : 0.0;
  const double* x = m.X + (size_t)c * m.d * m.xe;
  double* z = m.Z + ((size_t)((a * m.ra + c) * m.d + s) * m.wb + b) * m.xe;
  for (int e = lane; e < m.xe; e += 64) {
    double acc = w[0] * x[e];
    for (int t = 1; t < m.d; ++t) acc += w[t] * x[(size_t)t * m.xe + e];
    z[e] = acc;
  }
}

}  // namespace

int mpo_site_blocks(const MpoSite& m) {
  const long long rows = (long long)m.ra * m.wa * m.d * m.wb;
  return (int)((rows + kRowsPerGroup - 1) / kRowsPerGroup);
}

hipError_t launch_mpo_apply(const MpoArgs& a, int blocks, hipStream_t s) {
  if (blocks <= 0 || a.nsite <= 0) return hipSuccess;
  MpoArgs args = a;
  void* kp[] = {&args};
  const hipError_t e = hipLaunchKernel((const void*)mpo_apply_kernel, dim3(blocks), dim3(256), kp, 0, s);
  if (e != hipSuccess) (void)hipGetLastError();
  return e;
}

}  // namespace aci
