// Shared definitions of the ACI HIP library (device side and host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/aci.h"

namespace aci {

// A size or leading dimension that is either a constant or is read from
// device memory when the kernel runs (value = (*ptr) * mul + add).  Ranks
// found by one prrLU feed the shapes of the next kernels without a host
// round trip.
struct Dim {
  const int32_t* ptr;
  int32_t mul;
  int32_t add;
};

inline Dim dconst(int v) { return Dim{nullptr, 0, v}; }
inline Dim ddev(const int32_t* p, int mul = 1, int add = 0) { return Dim{p, mul, add}; }

__device__ __forceinline__ int dget(const Dim& d) {
  return d.ptr ? (*d.ptr) * d.mul + d.add : d.add;
}

// Device error flags (bitwise or-ed into one int of the workspace).
enum : int { ERR_NONFINITE = 1, ERR_TIMEOUT = 2, ERR_LIMIT = 4 };

// Stop rules of the LDU factorisation.
enum : int { RULE_EXCLUSIVE = 0, RULE_LITERAL = 1 };

// Elementwise operations of the two-site tensor.
enum : int { OP_NONE = -1, OP_PRODUCT = ACI_OP_PRODUCT, OP_SUM = ACI_OP_SUM,
             OP_ABS2_MUL = ACI_OP_ABS2_MUL, OP_LINEAR_CUBIC = ACI_OP_LINEAR_CUBIC };
// contraction precision (same values as aci_precision)
enum : int { PREC_FP64 = ACI_PREC_FP64, PREC_FP32 = ACI_PREC_FP32, PREC_BF16X3 = ACI_PREC_BF16X3 };

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// ---- low-latency exchange words --------------------------------------------
// A 64-bit word carries 32 bits of payload and a 32-bit flag.  A reader knows
// the word is current when the flag equals the value it expects, so a
// producer needs no memory fence between payload and flag: each word is its
// own flag.  Stores and loads are relaxed atomics at agent scope (single-copy
// atomic and coherent across the XCDs).
__device__ __forceinline__ void xw_store(uint64_t* p, uint32_t data, uint32_t flag) {
  uint64_t v = ((uint64_t)flag << 32) | (uint64_t)data;
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Poll until the flag matches.  Gives up (returns false) once the shared abort
// word is set; a wave that has polled `limit` times sets the abort word itself,
// so every waiting wave leaves within a bounded time.
__device__ __forceinline__ bool xw_load(const uint64_t* p, uint32_t flag, int* abort_word,
                                        uint32_t limit, uint32_t* out) {
  uint32_t spins = 0;
  while (true) {
    uint64_t v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((uint32_t)(v >> 32) == flag) {
      *out = (uint32_t)v;
      return true;
    }
    ++spins;
    if ((spins & 1023u) == 0u) {
      if (__hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
      if (spins >= limit) {
        __hip_atomic_store(abort_word, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
      }
    }
  }
}

__device__ __forceinline__ uint32_t lo32(double x) {
  return (uint32_t)(__double_as_longlong(x) & 0xffffffffull);
}
__device__ __forceinline__ uint32_t hi32(double x) {
  return (uint32_t)((unsigned long long)__double_as_longlong(x) >> 32);
}
__device__ __forceinline__ double join64(uint32_t lo, uint32_t hi) {
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

}  // namespace aci
