// LDU factorisation with full pivoting (Alg. 2, "greedy maxvol" pivot
// search) of a matricised two-site tensor, with the right-interpolative
// factor B = U_JJ^{-1} U of Alg. 3 formed on the fly.
//
// Layout.  P cooperating workgroups of WAVES waves share the m x n matrix by
// rows: global row i lives in workgroup i % P, wave (i / P) % WAVES, register
// slot (i / P) / WAVES; lane l holds columns l, l+64, ...  The residual never
// leaves the registers.
//
// One pivot step.  Each workgroup reduces the largest |residual| of its alive
// entries (ties: smallest row, then smallest column) and publishes that
// candidate together with the candidate's whole row as flagged 64-bit words
// (see aci_common.h).  Every workgroup reads all P candidates, picks the same
// winner (p, q, pivot) and takes row p from the winner's slot, so one
// exchange per pivot replaces a grid barrier.  With P == 1 the exchange goes
// through LDS.  The Schur complement update of Alg. 2 is applied to the alive
// rows as s - (s_q / pivot) * u_j with the product rounded before the
// subtraction (floating-point contraction is off in this file), which is the
// rounding of the CPU reference, so pivots agree bit for bit on equal input.
// Column q of the alive rows is set to zero; the row p either dies (left-to-
// right updates) or becomes the next row of B, normalised by the pivot.  Rows
// of B are kept reduced against every later pivot row (Gauss-Jordan), which
// gives U_JJ^{-1} U with B[:, J] = identity.
#include <climits>

#include "kernels.h"

#pragma clang fp contract(off)

namespace aci {

namespace {

enum : int { ROW_ALIVE = 0, ROW_PIVOT = 1, ROW_DEAD = 2 };

__device__ __forceinline__ void amax_combine(double& k1, int& i1, double k2, int i2) {
  if (k2 > k1 || (k2 == k1 && i2 < i1)) {
    k1 = k2;
    i1 = i2;
  }
}

__device__ __forceinline__ void wave_amax(double& k, int& i) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    double k2 = __shfl_xor(k, off);
    int i2 = __shfl_xor(i, off);
    amax_combine(k, i, k2, i2);
  }
}

template <int CS>
__device__ __forceinline__ double pick(const double (&row)[CS], int b) {
  double r = 0.0;
#pragma unroll
  for (int c = 0; c < CS; ++c)
    if (c == b) r = row[c];
  return r;
}

template <int WAVES, int RS, int CS, bool SOLO>
__global__ __launch_bounds__(WAVES * 64) void prrlu_kernel(PrrluArgs a) {
  if (blockIdx.x % a.stride) return;
  const int w = blockIdx.x / a.stride;
  const int P = a.P;
  const int m = dget(a.m), n = dget(a.n), ldm = dget(a.ldm);
  const int kmax = m < n ? m : n;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool needY = a.Y != nullptr;
  const int ldy = needY ? dget(a.ldy) : 0;

  __shared__ double red_k[2][WAVES];
  __shared__ int red_i[2][WAVES];
  __shared__ int red_f[2][WAVES];
  __shared__ double srow[SOLO ? 64 * CS : 1];

  double s[RS][CS];
  int state[RS], rowid[RS], pstep[RS];
  bool cv[CS];
#pragma unroll
  for (int b = 0; b < CS; ++b) cv[b] = (lane + 64 * b) < n;

  double bk = -1.0;
  int bi = INT_MAX;
#pragma unroll
  for (int r = 0; r < RS; ++r) {
    const int i = w + P * (wv + WAVES * r);
    rowid[r] = i;
    state[r] = i < m ? ROW_ALIVE : ROW_DEAD;
    pstep[r] = -1;
#pragma unroll
    for (int b = 0; b < CS; ++b) {
      const int j = lane + 64 * b;
      double v = 0.0;
      if (i < m && cv[b]) v = a.M[(size_t)i * ldm + j];
      s[r][b] = v;
      if (i < m && cv[b]) {
        const double kv = fabs(v);
        if (kv > bk) {
          bk = kv;
          bi = (i << 16) | j;
        }
      }
    }
  }

  int k = 0;
  double eps = 0.0;
  bool failed = false;
  int final_rank = 0;
  while (true) {
    if (k == kmax) {
      if (a.rule == RULE_EXCLUSIVE) eps = 0.0;
      final_rank = k;
      break;
    }
    const int par = k & 1;
    // ---- workgroup candidate
    wave_amax(bk, bi);
    if (lane == 0) {
      red_k[par][wv] = bk;
      red_i[par][wv] = bi;
      red_f[par][wv] = failed ? 1 : 0;
    }
    __syncthreads();
    double ck = -1.0;
    int ci = INT_MAX;
    int anyfail = 0;
    if (lane < WAVES) {
      ck = red_k[par][lane];
      ci = red_i[par][lane];
      anyfail = red_f[par][lane];
    }
    wave_amax(ck, ci);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) anyfail |= __shfl_xor(anyfail, off);
    if (anyfail) {
      // an exchange timed out: leave with an error (uniform across the group)
      final_rank = k;
      eps = 0.0;
      if (threadIdx.x == 0 && a.err) atomicOr(a.err, ERR_TIMEOUT);
      break;
    }

    // ---- global winner (v, p, q) and pivot row u
    double v;
    int widx;
    double u[CS];
    if (SOLO) {
      v = ck;
      widx = ci;
      const int p = widx >> 16;
      if (v >= 0.0) {
        const int rho = p / P;
        if (wv == rho % WAVES) {
          const int r0 = rho / WAVES;
#pragma unroll
          for (int r = 0; r < RS; ++r)
            if (r == r0) {
#pragma unroll
              for (int b = 0; b < CS; ++b) srow[lane + 64 * b] = s[r][b];
            }
        }
      }
      __syncthreads();
#pragma unroll
      for (int b = 0; b < CS; ++b) u[b] = srow[lane + 64 * b];
    } else {
      const uint32_t flag = a.flag_base + (uint32_t)k;
      uint64_t* slot_base = a.xbuf + (size_t)par * P * a.xwords;
      uint64_t* mine = slot_base + (size_t)w * a.xwords;
      if (wv == 0 && lane < 3) {
        const uint32_t d = lane == 0 ? lo32(ck) : (lane == 1 ? hi32(ck) : (uint32_t)ci);
        xw_store(mine + lane, d, flag);
      }
      if (ck >= 0.0) {
        const int rho = ((ci >> 16) - w) / P;
        if (wv == rho % WAVES) {
          const int r0 = rho / WAVES;
#pragma unroll
          for (int r = 0; r < RS; ++r)
            if (r == r0) {
#pragma unroll
              for (int b = 0; b < CS; ++b)
                if (cv[b]) {
                  const int j = lane + 64 * b;
                  xw_store(mine + 4 + 2 * j, lo32(s[r][b]), flag);
                  xw_store(mine + 5 + 2 * j, hi32(s[r][b]), flag);
                }
            }
        }
      }
      // all candidates: lane t < P reads the three words of workgroup t
      double tk = -1.0;
      int ti = INT_MAX;
      bool ok = true;
      if (lane < P) {
        const uint64_t* sl = slot_base + (size_t)lane * a.xwords;
        uint64_t c3[3];
#pragma unroll
        for (int h = 0; h < 3; ++h)
          c3[h] = __hip_atomic_load(sl + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t spins = 0;
        while (true) {
          bool all = true;
#pragma unroll
          for (int h = 0; h < 3; ++h)
            if ((uint32_t)(c3[h] >> 32) != flag) {
              all = false;
              c3[h] = __hip_atomic_load(sl + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
          if (all) break;
          ++spins;
          if ((spins & 1023u) == 0u) {
            if (__hip_atomic_load(a.abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ok = false; break; }
            if (spins >= a.spin_limit) {
              __hip_atomic_store(a.abort_word, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              ok = false;
              break;
            }
          }
        }
        if (ok) {
          tk = join64((uint32_t)c3[0], (uint32_t)c3[1]);
          ti = (int)(uint32_t)c3[2];
        }
      }
      ok = __ballot(!ok) == 0;
      wave_amax(tk, ti);
      v = tk;
      widx = ti;
      int p = widx >> 16;
      if (!(v >= 0.0) || p < 0 || p >= m || (widx & 0xffff) >= n) {
        // only reachable after a timeout; keep every index in range
        ok = false;
        v = 0.0;
        widx = 0;
        p = 0;
      }
      // the winner's row
      const uint64_t* ws = slot_base + (size_t)(p % P) * a.xwords;
      uint64_t raw[2 * CS];
#pragma unroll
      for (int b = 0; b < CS; ++b) {
        const int j = lane + 64 * b;
        if (cv[b]) {
          raw[2 * b] = __hip_atomic_load(ws + 4 + 2 * j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          raw[2 * b + 1] = __hip_atomic_load(ws + 5 + 2 * j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
          raw[2 * b] = (uint64_t)flag << 32;
          raw[2 * b + 1] = (uint64_t)flag << 32;
        }
      }
      uint32_t spins = 0;
      while (ok) {
        bool all = true;
#pragma unroll
        for (int b = 0; b < CS; ++b) {
          const int j = lane + 64 * b;
#pragma unroll
          for (int h = 0; h < 2; ++h)
            if ((uint32_t)(raw[2 * b + h] >> 32) != flag) {
              all = false;
              raw[2 * b + h] = __hip_atomic_load(ws + 4 + 2 * j + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (all) break;
        ++spins;
        if ((spins & 1023u) == 0u) {
          if (__hip_atomic_load(a.abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = false;
          if (spins >= a.spin_limit) {
            __hip_atomic_store(a.abort_word, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = false;
          }
        }
      }
#pragma unroll
      for (int b = 0; b < CS; ++b)
        u[b] = cv[b] ? join64((uint32_t)raw[2 * b], (uint32_t)raw[2 * b + 1]) : 0.0;
      ok = __ballot(!ok) == 0;
      if (!ok) {
        // keep going with zeros until the whole group agrees to stop
        failed = true;
        v = 0.0;
        widx = 0;
#pragma unroll
        for (int b = 0; b < CS; ++b) u[b] = 0.0;
        if (lane == 0 && a.err) atomicOr(a.err, ERR_TIMEOUT);
      }
    }

    const int p = widx >> 16;
    const int q = widx & 0xffff;
    const int qb = q >> 6;
    const int ql = q & 63;

    // ---- stop rules
    if (a.rule == RULE_EXCLUSIVE) {
      if (k == a.maxrank) { eps = v; final_rank = k; break; }
      if (k >= 1 && v <= a.tol) { eps = v; final_rank = k; break; }
    } else if (k >= 1 && v == 0.0) {
      eps = 0.0;
      final_rank = k;
      break;
    }
    const double piv = __shfl(pick<CS>(u, qb), ql);
    if (w == 0 && threadIdx.x == 0) {
      a.rows[k] = p;
      a.cols[k] = q;
    }
    if (piv == 0.0) {
      // all-zero matrix (only possible at k == 0): one pivot at the tie-break
      // cell, B = unit row e_q, error 0
#pragma unroll
      for (int r = 0; r < RS; ++r)
        if (rowid[r] == p && needY) {
          state[r] = ROW_PIVOT;
          pstep[r] = 0;
#pragma unroll
          for (int b = 0; b < CS; ++b) s[r][b] = (lane + 64 * b == q) ? 1.0 : 0.0;
        }
      eps = 0.0;
      final_rank = 1;
      break;
    }

    // ---- elimination, fused with the next step's local argmax
    double uh[CS];
    if (needY) {
#pragma unroll
      for (int b = 0; b < CS; ++b) uh[b] = u[b] / piv;
    }
    bk = -1.0;
    bi = INT_MAX;
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      if (state[r] == ROW_ALIVE) {
        if (rowid[r] == p) {
          if (needY) {
            state[r] = ROW_PIVOT;
            pstep[r] = k;
#pragma unroll
            for (int b = 0; b < CS; ++b) s[r][b] = s[r][b] / piv;
          } else {
            state[r] = ROW_DEAD;
          }
        } else {
          const double c = __shfl(pick<CS>(s[r], qb), ql) / piv;
#pragma unroll
          for (int b = 0; b < CS; ++b) {
            const double t = c * u[b];
            double x = s[r][b] - t;
            if (b == qb && lane == ql) x = 0.0;
            s[r][b] = x;
            const double kv = fabs(x);
            if (cv[b] && kv > bk) {
              bk = kv;
              bi = (rowid[r] << 16) | (lane + 64 * b);
            }
          }
        }
      } else if (state[r] == ROW_PIVOT) {
        const double c = __shfl(pick<CS>(s[r], qb), ql);
#pragma unroll
        for (int b = 0; b < CS; ++b) {
          const double t = c * uh[b];
          s[r][b] = s[r][b] - t;
        }
      }
    }
    ++k;
    if (a.rule == RULE_LITERAL) {
      eps = v;
      if (v <= a.tol || k == a.maxrank) {
        final_rank = k;
        break;
      }
    }
  }

  if (needY) {
#pragma unroll
    for (int r = 0; r < RS; ++r)
      if (state[r] == ROW_PIVOT && pstep[r] >= 0 && pstep[r] < final_rank) {
#pragma unroll
        for (int b = 0; b < CS; ++b)
          if (cv[b]) a.Y[(size_t)pstep[r] * ldy + lane + 64 * b] = s[r][b];
      }
  }
  if (w == 0 && threadIdx.x == 0) {
    *a.rank = final_rank;
    *a.eps = eps;
    if (a.rank2) *a.rank2 = final_rank;
    if (a.eps2) *a.eps2 = eps;
    if (a.meta) {
      a.meta[0] = final_rank;
      a.meta[1] = m;
      a.meta[2] = n;
    }
    if (a.meta2) {
      a.meta2[0] = final_rank;
      a.meta2[1] = m;
      a.meta2[2] = n;
    }
  }
}

// Register shapes: CS column slots per lane (n <= 64 CS), RS row slots per
// wave.  Only shapes that fit the register file without spilling are built:
// with 16 waves a lane has 128 VGPRs, with 8 waves 256.
struct Shape {
  int cs, waves, rs_max;
};
constexpr Shape kShapes[] = {{1, 16, 4}, {2, 16, 4}, {4, 16, 2}, {6, 16, 2}, {8, 16, 1}, {12, 8, 2}, {16, 8, 1}};

// Resident workgroups per CU of one kernel instance (cached).
int resident_per_cu(const void* fn, int block) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, block, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return nb < 1 ? 1 : nb;
}

int cus_per_xcd() {
  static int v = 0;
  if (!v) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
      (void)hipGetLastError();
      cus = 256;
    }
    v = cus / 8 > 0 ? cus / 8 : 1;
  }
  return v;
}

template <int WAVES, int RS, int CS>
hipError_t launch_shape(const PrrluArgs& a, hipStream_t s) {
  const void* fn = a.P == 1 ? (const void*)prrlu_kernel<WAVES, RS, CS, true>
                            : (const void*)prrlu_kernel<WAVES, RS, CS, false>;
  static int per_cu = resident_per_cu((const void*)prrlu_kernel<WAVES, RS, CS, false>, WAVES * 64);
  PrrluArgs args = a;
  // Workgroups are dealt to the 8 XCDs round robin, so launching 8x the
  // groups and keeping every 8th puts the cooperating groups on one XCD,
  // which shortens the exchange latency.  Only when they all fit there.
  args.stride = (a.P > 1 && a.P <= per_cu * cus_per_xcd()) ? 8 : 1;
  dim3 block(WAVES * 64);
  dim3 grid(args.P * args.stride);
  void* kp[] = {&args};
  hipError_t e = hipLaunchCooperativeKernel(fn, grid, block, kp, 0, s);
  if (e != hipSuccess) (void)hipGetLastError();
  return e;
}

const Shape* pick_shape(int nmax) {
  for (const Shape& sh : kShapes)
    if (64 * sh.cs >= nmax) return &sh;
  return nullptr;
}

// rows per workgroup: as few register slots as keep the group count small
int pick_rs(const Shape& sh, int mmax) {
  const int target_p = 8;
  int rs = 1;
  while (rs < sh.rs_max && (mmax + sh.waves * rs - 1) / (sh.waves * rs) > target_p) rs *= 2;
  return rs;
}

}  // namespace

size_t prrlu_xbuf_words(int mmax, int nmax) {
  // every launch uses at most 64 groups and the column slots of nmax
  (void)mmax;
  const Shape* sh = pick_shape(nmax < 1 ? 1 : nmax);
  if (!sh) sh = &kShapes[sizeof(kShapes) / sizeof(kShapes[0]) - 1];
  return (size_t)2 * 64 * (4 + 2 * 64 * sh->cs);
}

hipError_t launch_prrlu(const PrrluArgs& a0, int mmax, int nmax, hipStream_t s) {
  if (mmax < 1 || nmax < 1 || mmax > ACI_MAX_MATRIX || nmax > ACI_MAX_MATRIX) return hipErrorInvalidValue;
  const Shape* sh = pick_shape(nmax);
  if (!sh) return hipErrorInvalidValue;
  PrrluArgs a = a0;
  const int rs = pick_rs(*sh, mmax);
  a.P = (mmax + sh->waves * rs - 1) / (sh->waves * rs);
  if (a.P > 64) return hipErrorInvalidValue;
  a.xwords = 4 + 2 * 64 * sh->cs;
  if ((size_t)2 * a.P * a.xwords > a.xbuf_words) return hipErrorInvalidValue;
  switch (sh->cs * 8 + rs) {
    case 1 * 8 + 1: return launch_shape<16, 1, 1>(a, s);
    case 1 * 8 + 2: return launch_shape<16, 2, 1>(a, s);
    case 1 * 8 + 4: return launch_shape<16, 4, 1>(a, s);
    case 2 * 8 + 1: return launch_shape<16, 1, 2>(a, s);
    case 2 * 8 + 2: return launch_shape<16, 2, 2>(a, s);
    case 2 * 8 + 4: return launch_shape<16, 4, 2>(a, s);
    case 4 * 8 + 1: return launch_shape<16, 1, 4>(a, s);
    case 4 * 8 + 2: return launch_shape<16, 2, 4>(a, s);
    case 6 * 8 + 1: return launch_shape<16, 1, 6>(a, s);
    case 6 * 8 + 2: return launch_shape<16, 2, 6>(a, s);
    case 8 * 8 + 1: return launch_shape<16, 1, 8>(a, s);
    case 12 * 8 + 1: return launch_shape<8, 1, 12>(a, s);
    case 12 * 8 + 2: return launch_shape<8, 2, 12>(a, s);
    case 16 * 8 + 1: return launch_shape<8, 1, 16>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace aci
