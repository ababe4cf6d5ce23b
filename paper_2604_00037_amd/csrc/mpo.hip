// Exact contraction of a TT operator (MPO) with a tensor train, the operator
// half of an explicit step of a nonlinear equation (the use of ACI named in
// Sec. 4).  Core by core,
//   Z[(a, c), s, (b, e)] = sum_t W[a, s, t, b] X[c, t, e],
// so the output is w^2 times the input: the kernel is bound by its HBM
// writes.  One wave produces the wb output rows (a, c, s, 0..wb-1), which
// are contiguous (wb xe doubles), from the d rows X[c, t, :]: every element
// of X is loaded once per (a, s) and every output element stored once,
// 16 bytes per lane and access, with non-temporal stores (the output is not
// read again by this kernel).  Row groups are dealt in the order (c, a, s)
// so that the workgroups running together read the same rows of X from L2.
#include "kernels.h"

namespace aci {
namespace {

constexpr int kRowsPerGroup = 4;   // one row group per wave of a 256-thread workgroup

typedef double v2d __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void mpo_apply_kernel(MpoArgs args) {
  int si = 0;
  for (int k = 1; k < args.nsite; ++k)
    if ((int)blockIdx.x >= args.site[k].block0) si = k;
  const MpoSite& m = args.site[si];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = ((int)blockIdx.x - m.block0) * kRowsPerGroup + wave;
  if (row >= m.ra * m.wa * m.d) return;
  const int s = row % m.d;
  const int a = (row / m.d) % m.wa;
  const int c = row / (m.d * m.wa);
  const int d = m.d, wb = m.wb, xe = m.xe;
  const double* x = m.X + (size_t)c * d * xe;
  const double* w = m.W + (size_t)(a * d + s) * d * wb;   // w[t wb + b] = W[a, s, t, b]
  double* z = m.Z + ((size_t)(a * m.ra + c) * d + s) * wb * xe;
  if (m.vec) {
    const int n2 = xe / 2;
    for (int e = lane; e < n2; e += 64) {
      v2d xv[ACI_MAX_DIM];
#pragma unroll
      for (int t = 0; t < ACI_MAX_DIM; ++t)
        if (t < d) xv[t] = reinterpret_cast<const v2d*>(x + (size_t)t * xe)[e];
      for (int b = 0; b < wb; ++b) {
        v2d acc = w[b] * xv[0];
#pragma unroll
        for (int t = 1; t < ACI_MAX_DIM; ++t)
          if (t < d) acc += w[t * wb + b] * xv[t];
        __builtin_nontemporal_store(acc, reinterpret_cast<v2d*>(z + (size_t)b * xe) + e);
      }
    }
  } else {
    for (int e = lane; e < xe; e += 64) {
      double xv[ACI_MAX_DIM];
#pragma unroll
      for (int t = 0; t < ACI_MAX_DIM; ++t)
        if (t < d) xv[t] = x[(size_t)t * xe + e];
      for (int b = 0; b < wb; ++b) {
        double acc = w[b] * xv[0];
#pragma unroll
        for (int t = 1; t < ACI_MAX_DIM; ++t)
          if (t < d) acc += w[t * wb + b] * xv[t];
        __builtin_nontemporal_store(acc, z + (size_t)b * xe + e);
      }
    }
  }
}

}  // namespace

int mpo_site_blocks(const MpoSite& m) {
  const long long rows = (long long)m.ra * m.wa * m.d;
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
