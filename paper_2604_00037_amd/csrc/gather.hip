// Frame truncation of Alg. 5 (L' = (L X)[I, :], R' = (X R)[:, J]) as gathers
// of pivot rows / columns from the cached environment products, and small
// fill kernels.
#include "kernels.h"

namespace aci {

namespace {

// side 0: dst[k][c] = src[idx[k]][c], k < rank, c < extent
// side 1: dst[h][k] = src[h][idx[k]], h < extent, k < rank
// grid: x over the gathered index k (64 per block), y over the extent, z item
__global__ __launch_bounds__(256) void gather_kernel(GatherArgs a) {
  const GatherItem& it = a.it[blockIdx.z];
  const int r = *a.rank;
  // elements of esz doubles (2: complex, interleaved re, im)
  const int es = a.esz > 1 ? a.esz : 1;
  const int ext = dget(it.extent);
  const int lds = dget(it.ld_src) * es;
  const int ldd = dget(it.ld_dst) * es;
  const int nsrc = dget(it.src_n);
  if (a.side == 0) {
    // one row per (k), threads along the row
    const int k = blockIdx.x;
    if (k >= r) return;
    const int src_row = a.idx[k];
    if (src_row < 0 || src_row >= nsrc) {
      if (threadIdx.x == 0 && a.err) atomicOr(a.err, ERR_LIMIT);
      return;
    }
    for (int c = blockIdx.y * 256 + threadIdx.x; c < ext * es; c += gridDim.y * 256)
      it.dst[(size_t)k * ldd + c] = it.src[(size_t)src_row * lds + c];
  } else {
    // threads along k (destination row is contiguous in k)
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= r) return;
    const int sc = a.idx[k];
    if (sc < 0 || sc >= nsrc) {
      if (a.err) atomicOr(a.err, ERR_LIMIT);
      return;
    }
    for (int h = blockIdx.y; h < ext; h += gridDim.y)
      for (int e = 0; e < es; ++e) it.dst[(size_t)h * ldd + (size_t)k * es + e] = it.src[(size_t)h * lds + (size_t)sc * es + e];
  }
}

__global__ void fill_kernel(double* p, size_t n, double v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void fill_int_kernel(int* p, size_t n, int v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

}  // namespace

hipError_t launch_gather(const GatherArgs& a, int rmax, int extent_max, hipStream_t s) {
  if (rmax <= 0 || extent_max <= 0 || a.count <= 0) return hipSuccess;
  if (a.side == 0) {
    dim3 grid(rmax, (extent_max + 255) / 256 > 8 ? 8 : (extent_max + 255) / 256, a.count);
    hipLaunchKernelGGL(gather_kernel, grid, dim3(256), 0, s, a);
  } else {
    dim3 grid((rmax + 255) / 256, extent_max > 256 ? 256 : extent_max, a.count);
    hipLaunchKernelGGL(gather_kernel, grid, dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_fill(double* p, size_t count, double value, hipStream_t s) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, count, value);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* p, size_t count, int value, hipStream_t s) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, count, value);
  return hipGetLastError();
}

}  // namespace aci
