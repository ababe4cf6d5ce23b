// LDU factorisation with full pivoting (Alg. 2, "greedy maxvol" pivot
// search) of a matricised two-site tensor, with the right-interpolative
// factor B = U_JJ^{-1} U of Alg. 3 formed on the fly.
//
// Layout.  P cooperating workgroups of four waves (one per SIMD, one group
// per CU) share the m x n matrix by rows: global row i lives in workgroup
// i % P, wave (i / P) % 4, register slot (i / P) / 4; lane l holds columns
// l, l+64, ...  The residual never leaves the registers.
//
// One pivot step.  Each workgroup reduces the largest |residual| of its alive
// entries (ties: smallest row, then smallest column) and publishes that
// candidate together with the candidate's row as flagged 64-bit words (see
// aci_common.h).  Every workgroup reads the P candidates, picks the same
// winner (p, q, pivot) and reads row p from the winner's slot: two round
// trips through the XCD's L2 per pivot replace grid barriers.  With P == 1
// the exchange stays in LDS.  The Schur complement update of Alg. 2 is
// applied to the alive rows as s - (s_q / pivot) * u_j with the product
// rounded before the subtraction (floating-point contraction is off in this
// file), which is the rounding of the CPU reference, so pivots agree bit for
// bit on equal input.  Column q of the alive rows is set to zero; row p either
// dies (left-to-right updates) or becomes the next row of B, normalised by the
// pivot.  Rows of B are kept reduced against every later pivot row
// (Gauss-Jordan), which gives U_JJ^{-1} U with B[:, J] = identity.
#include <algorithm>
#include <climits>

#include "kernels.h"

#pragma clang fp contract(off)

namespace aci {

namespace {

constexpr int WAVES = 4;
constexpr int NT = WAVES * 64;

// ---- wave-wide reductions with DPP row shifts and row broadcasts ----------
// After row_shr 1, 2, 4, 8 lane 15 of every 16-lane row holds the row's
// reduction; row_bcast 15 and 31 fold the rows so that lane 63 holds the
// wave's.  Lanes without a DPP source keep their own value (bound_ctrl off).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, ROWMASK, 0xf, false);
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = dpp_i32<CTRL, ROWMASK>(__double2loint(v));
  const int hi = dpp_i32<CTRL, ROWMASK>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_max_f64(double v) {
  v = fmax(v, dpp_f64<0x111, 0xf>(v));
  v = fmax(v, dpp_f64<0x112, 0xf>(v));
  v = fmax(v, dpp_f64<0x114, 0xf>(v));
  v = fmax(v, dpp_f64<0x118, 0xf>(v));
  v = fmax(v, dpp_f64<0x142, 0xa>(v));
  v = fmax(v, dpp_f64<0x143, 0xc>(v));
  return readlane_f64(v, 63);
}

__device__ __forceinline__ int wave_min_i32(int v) {
  v = min(v, dpp_i32<0x111, 0xf>(v));
  v = min(v, dpp_i32<0x112, 0xf>(v));
  v = min(v, dpp_i32<0x114, 0xf>(v));
  v = min(v, dpp_i32<0x118, 0xf>(v));
  v = min(v, dpp_i32<0x142, 0xa>(v));
  v = min(v, dpp_i32<0x143, 0xc>(v));
  return __builtin_amdgcn_readlane(v, 63);
}

// Largest key over the wave; among equal keys the smallest packed index
// (row << 16 | column).  The result is uniform across the wave.
__device__ __forceinline__ void wave_argmax(double& k, int& i) {
  const double mk = wave_max_f64(k);
  const int c = wave_min_i32(k == mk ? i : INT_MAX);
  k = mk;
  i = c;
}

// Value of column slot qb held by lane ql (both uniform), broadcast to the
// wave.  The slot is chosen by uniform branches, so one readlane pair runs.
template <int CS>
__device__ __forceinline__ double lane_pick(const double (&row)[CS], int qb, int ql) {
  double r = 0.0;
#pragma unroll
  for (int c = 0; c < CS; ++c)
    if (c == qb) r = readlane_f64(row[c], ql);
  return r;
}

// XCD (XCC) the workgroup runs on.
__device__ __forceinline__ int hw_xcc_id() {
  uint32_t v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
  return (int)(v & 0xf);
}

// Exchange store.  Loads are always agent-scope (they bypass the CU's L1 and
// read the XCD's L2).  When every cooperating group runs on the same XCD a
// workgroup-scope store suffices: the L1 is write-through, so the word lands
// in the shared L2 where those loads find it, and it is not pushed further
// out.  Groups spread over several XCDs use agent-scope stores.
__device__ __forceinline__ void xw_put(uint64_t* p, uint32_t data, uint32_t flag, bool same_xcd) {
  const uint64_t v = ((uint64_t)flag << 32) | (uint64_t)data;
  if (same_xcd)
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  else
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Poll `cnt` flagged words src[0 .. cnt) (thread t of NTH takes words t, t + NTH, ...)
// until their flags match, then store the payloads to dst.  Returns false
// after a timeout; the abort word is then set for every waiting wave.
template <int MAXW, int NTH>
__device__ __forceinline__ bool poll_words(const uint64_t* src, int cnt, uint32_t flag, int* abort_word,
                                           uint32_t limit, uint32_t* dst) {
  uint64_t raw[MAXW];
#pragma unroll
  for (int i = 0; i < MAXW; ++i) {
    const int t = threadIdx.x + NTH * i;
    raw[i] = t < cnt ? __hip_atomic_load(src + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                     : ((uint64_t)flag << 32);
  }
  uint32_t spins = 0;
  bool ok = true;
  while (true) {
    bool all = true;
#pragma unroll
    for (int i = 0; i < MAXW; ++i) {
      const int t = threadIdx.x + NTH * i;
      if (t < cnt && (uint32_t)(raw[i] >> 32) != flag) {
        all = false;
        raw[i] = __hip_atomic_load(src + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (all) break;
    ++spins;
    if ((spins & 255u) == 0u) {
      if (__hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ok = false; break; }
      if (spins >= limit) {
        __hip_atomic_store(abort_word, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = false;
        break;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < MAXW; ++i) {
    const int t = threadIdx.x + NTH * i;
    if (t < cnt) dst[t] = (uint32_t)raw[i];
  }
  return ok;
}

// Publish register row slot r0 of this wave (lane l: columns l, l + 64, ...)
// as flagged words after the candidate words of its slot.
template <int RS, int CS, bool CX>
__device__ __forceinline__ void publish_row(uint64_t* mine, const double (&s)[RS][CS],
                                            const double (&si)[CX ? RS : 1][CX ? CS : 1], int r0,
                                            const bool (&cv)[CS], uint32_t flag, bool same_xcd) {
  constexpr int EW = CX ? 2 : 1;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < RS; ++r)
    if (r == r0) {
#pragma unroll
      for (int b = 0; b < CS; ++b)
        if (cv[b]) {
          const int j = lane + 64 * b;
          xw_put(mine + 3 + 2 * EW * j, lo32(s[r][b]), flag, same_xcd);
          xw_put(mine + 4 + 2 * EW * j, hi32(s[r][b]), flag, same_xcd);
          if constexpr (CX) {
            xw_put(mine + 5 + 4 * j, lo32(si[r][b]), flag, same_xcd);
            xw_put(mine + 6 + 4 * j, hi32(si[r][b]), flag, same_xcd);
          }
        }
    }
}

// Most workgroups one factorisation may use (one per CU).
constexpr int kMaxGroups = 128;
// LDS of a cooperative launch: candidate words at [0, kCandWords) (three per
// group), the winner's row after them.
constexpr int kCandWords = 3 * kMaxGroups;
// LDS words of a launch: the candidates, the winner's row (flagged-word
// payloads) and, for real rows, that row divided by the pivot (doubles).
template <int CS, bool CX>
constexpr int lds_words() { return kCandWords + 2 * 128 * (CX ? 2 : 1) * CS; }
// a step index no pivot step uses (steps stay below ACI_MAX_MATRIX)
constexpr uint32_t kXccFlagOffset = 1536;

// Squared magnitude of a complex entry (two roundings, no fused multiply-add:
// the key of the complex pivot search).
__device__ __forceinline__ double cabs2(double re, double im) {
  const double a = re * re;
  const double b = im * im;
  return a + b;
}

// Complex entries (CX) are held as two register arrays, real and imaginary
// parts; the search key is re^2 + im^2 and the pivot magnitude its square
// root; the elimination spells the complex arithmetic out as
//   l = s_q conj(pi) / |pi|^2,  s_j -= l u_j  (re: (l.re u.re - l.im u.im),
//   im: (l.re u.im + l.im u.re)),
// every product and sum rounded on its own.
//
// The factorisation itself, run by group w (0 <= w < a.P) of the
// cooperating groups.
template <int RS, int CS, bool SOLO, bool CX, int WAVES, bool CROSS = false>
__device__ __forceinline__ void prrlu_body(const PrrluArgs& a, const int w) {
  constexpr int NT = 64 * WAVES;   // threads of the workgroup
  // flags of this launch: step k uses fbase + k
  const uint32_t fbase = a.epoch ? __hip_atomic_load(a.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                 : a.flag_base;
  constexpr int EW = CX ? 2 : 1;   // doubles per entry
  // real groups of eight waves (two per SIMD) and complex groups share the
  // division of the pivot row for the rows of B through LDS; for real rows
  // in four waves the extra barrier costs more than the divisions it saves
  constexpr bool kShareNorm = !SOLO && (CX || WAVES == 8);
  // only complex rows of 1024 columns (two rows per wave) need more than 64
  // groups; every other shape keeps P <= 64, one candidate per lane
  constexpr bool WIDE = CX && CS == 16;
  const int P = a.P;
  const int m = dget(a.m), n = dget(a.n), ldm = dget(a.ldm);
  const int kmax = m < n ? m : n;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool needY = a.Y != nullptr;
  const int ldy = needY ? dget(a.ldy) : 0;
  // slot of group g in the exchange buffer: words [g per, g per + 3) hold the
  // candidate (key lo, key hi, index), then 2 EW n words its row (lo, hi of
  // each double)
  const int per = 3 + 2 * EW * n;

  __shared__ double red_k[2][WAVES];
  __shared__ int red_i[2][WAVES];
  __shared__ int red_f[2][WAVES];
  // set once any thread of the group saw a wait time out (only ever 0 -> 1)
  __shared__ int gfail;
  if (threadIdx.x == 0) gfail = 0;
  // 16-byte aligned, so that the winner's row is read from LDS with wide
  // loads (complex rows: 14.4 against 15.2 us per 1024 x 1024 pivot step)
  extern __shared__ __align__(16) uint32_t xs[];
  uint32_t* xrow = xs + kCandWords;
  // real rows of B: the winner's row divided by the pivot, once per group
  double* xrn = reinterpret_cast<double*>(xs + kCandWords + 128 * EW * CS);

  double s[RS][CS];
  double si[CX ? RS : 1][CX ? CS : 1];
  // row slot r of this wave holds global row w + P (wv + 4 r).  Row states
  // are wave-uniform bit sets: alive rows take part in the pivot search and
  // the Schur update, B rows (right-to-left updates only) in the
  // Gauss-Jordan reduction; pstep[r] is the pivot step of a B row.
  uint32_t alive = 0u, brows = 0u;
  int pstep[RS];
  const int row0 = w + P * wv, rstride = P * WAVES;
  bool cv[CS];
#pragma unroll
  for (int b = 0; b < CS; ++b) cv[b] = (lane + 64 * b) < n;

  // rm[r]: largest key of row slot r in this lane (-1 when the row is not
  // alive).  Entries of columns >= n and of eliminated columns are zero.
  double rm[RS];
#pragma unroll
  for (int r = 0; r < RS; ++r) {
    const int i = row0 + rstride * r;
    if (i < m) alive |= 1u << r;
    pstep[r] = -1;
    rm[r] = -1.0;
#pragma unroll
    for (int b = 0; b < CS; ++b) {
      const int j = lane + 64 * b;
      double v = 0.0, vi = 0.0;
      if (i < m && cv[b]) {
        v = a.M[EW * ((size_t)i * ldm + j)];
        if constexpr (CX) vi = a.M[2 * ((size_t)i * ldm + j) + 1];
      }
      s[r][b] = v;
      if constexpr (CX) si[r][b] = vi;
      if (i < m) rm[r] = fmax(rm[r], CX ? cabs2(v, vi) : fabs(v));
    }
  }

  alive = __builtin_amdgcn_readfirstlane(alive);
  bool failed = false;
  bool same_xcd = false;
  if (!SOLO) {
    // which XCD each group runs on, exchanged once at agent scope through
    // word 0 of the parity-1 slots (overwritten by step 1 only after every
    // group has passed step 0, hence this exchange)
    const uint32_t xf = fbase + kXccFlagOffset;
    uint64_t* slots1 = a.xbuf + (size_t)P * a.xwords;
    if (threadIdx.x == 0) xw_put(slots1 + (size_t)w * per, (uint32_t)hw_xcc_id(), xf, false);
    bool ok = true;
    if (threadIdx.x < P) {
      const uint64_t* src = slots1 + (size_t)threadIdx.x * per;
      uint64_t v = __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      uint32_t spins = 0;
      while ((uint32_t)(v >> 32) != xf) {
        ++spins;
        if ((spins & 255u) == 0u) {
          if (__hip_atomic_load(a.abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) || spins >= a.spin_limit) {
            __hip_atomic_store(a.abort_word, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = false;
            break;
          }
        }
        v = __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      xs[threadIdx.x] = ok ? (uint32_t)v : 0xffffffffu - threadIdx.x;
    }
    if (!ok) failed = true;
    __syncthreads();
    same_xcd = __ballot((lane < P && xs[lane] != xs[0]) || (lane + 64 < P && xs[lane + 64] != xs[0])) == 0;
  }

  int k = 0;
  double eps = 0.0;
  int final_rank = 0;
  double tol = a.tol;   // raised to the noise floor after the first pivot
  // across XCDs: keys of the last two pivots, and the candidate key from
  // which a group publishes its row eagerly (see the exchange below)
  double last_key = 0.0, prev_key = 1.0, eager_key = 0.0;
  while (true) {
    if (k == kmax) {
      if (a.rule == RULE_EXCLUSIVE) eps = 0.0;
      final_rank = k;
      break;
    }
    const int par = k & 1;
    // ---- wave candidate: the largest key, then the smallest index holding
    // it.  Only rows in which some lane holds the wave's maximum are scanned.
    double bk = rm[0];
#pragma unroll
    for (int r = 1; r < RS; ++r) bk = fmax(bk, rm[r]);
    bk = wave_max_f64(bk);
    int bi = INT_MAX;
    bool found = false;
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      if (!found && __ballot(rm[r] == bk) != 0) {
        if (rm[r] == bk) {
#pragma unroll
          for (int b = CS - 1; b >= 0; --b) {
            const double kb = CX ? cabs2(s[r][b], si[CX ? r : 0][CX ? b : 0]) : fabs(s[r][b]);
            if (kb == bk) bi = ((row0 + rstride * r) << 16) | (lane + 64 * b);
          }
        }
        found = true;
      }
    }
    bi = wave_min_i32(bi);
    if (lane == 0) {
      red_k[par][wv] = bk;
      red_i[par][wv] = bi;
      red_f[par][wv] = failed ? 1 : 0;
    }
    __syncthreads();
    double ck = lane < WAVES ? red_k[par][lane] : -1.0;
    int ci = lane < WAVES ? red_i[par][lane] : INT_MAX;
    const bool anyfail = __ballot(lane < WAVES && red_f[par][lane] != 0) != 0;
    wave_argmax(ck, ci);
    if (anyfail) {
      // an exchange timed out: leave with an error (uniform across the group)
      final_rank = k;
      eps = 0.0;
      if (threadIdx.x == 0 && a.err) atomicOr(a.err, ERR_TIMEOUT);
      break;
    }

    // ---- global winner (key, p, q) and pivot row u (+ ui)
    double v;
    int widx;
    double u[CS];
    double ui[CX ? CS : 1];
    if (SOLO) {
      double* srow = reinterpret_cast<double*>(xrow);
      v = ck;
      widx = ci;
      if (v >= 0.0) {
        const int rho = widx >> 16;
        if (wv == rho % WAVES) {
          const int r0 = rho / WAVES;
#pragma unroll
          for (int r = 0; r < RS; ++r)
            if (r == r0) {
#pragma unroll
              for (int b = 0; b < CS; ++b) {
                srow[EW * (lane + 64 * b)] = s[r][b];
                if constexpr (CX) srow[2 * (lane + 64 * b) + 1] = si[r][b];
              }
            }
        }
      }
      __syncthreads();
#pragma unroll
      for (int b = 0; b < CS; ++b) {
        u[b] = srow[EW * (lane + 64 * b)];
        if constexpr (CX) ui[b] = srow[2 * (lane + 64 * b) + 1];
      }
    } else {
      const uint32_t flag = fbase + (uint32_t)k;
      // the flag readers wait for: the published one, unless a test stalls
      // this step (then no word ever carries it)
      const uint32_t want = k >= a.stall_from ? (flag ^ a.poll_xor) : flag;
      uint64_t* slot_base = a.xbuf + (size_t)par * P * a.xwords;
      uint64_t* mine = slot_base + (size_t)w * per;
      if (wv == 0 && lane < 3) {
        const uint32_t d = lane == 0 ? lo32(ck) : (lane == 1 ? hi32(ck) : (uint32_t)ci);
        xw_put(mine + lane, d, flag, same_xcd);
      }
      // The candidate's row goes out with the candidate (saving a round
      // trip for the winner) when the groups share one XCD: those stores
      // end in its L2.  Across XCDs they travel further and up to 128 groups
      // publish, so only groups whose candidate may win do: key at least
      // a.eager_frac of the pivot key predicted from the last two (last key
      // times the last ratio, at most 1).  A winner that did not publish
      // does so once it knows; readers poll the row's flags either way, so
      // the rule moves stores in time and changes no result.
      const bool eager = !CROSS || same_xcd || k < 2 || ck >= eager_key;
      if (eager && ck >= 0.0) {
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
                  xw_put(mine + 3 + 2 * EW * j, lo32(s[r][b]), flag, same_xcd);
                  xw_put(mine + 4 + 2 * EW * j, hi32(s[r][b]), flag, same_xcd);
                  if constexpr (CX) {
                    xw_put(mine + 5 + 4 * j, lo32(si[r][b]), flag, same_xcd);
                    xw_put(mine + 6 + 4 * j, hi32(si[r][b]), flag, same_xcd);
                  }
                }
            }
        }
      }
      // round trip 1: the P candidates (thread t reads word t, and t + NT
      // when more than 85 groups cooperate)
      bool ok = true;
#pragma unroll
      for (int i = 0; i < WIDE + 1; ++i) {
        const int t = threadIdx.x + NT * i;
        if (!ok || t >= 3 * P) continue;
        const int g = t / 3;
        const uint64_t* src = slot_base + (size_t)g * per + (t - 3 * g);
        uint64_t raw = __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t spins = 0;
        while ((uint32_t)(raw >> 32) != want) {
          ++spins;
          if ((spins & 255u) == 0u) {
            if (__hip_atomic_load(a.abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) || spins >= a.spin_limit) {
              __hip_atomic_store(a.abort_word, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              ok = false;
              break;
            }
          }
          raw = __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        xs[t] = (uint32_t)raw;
      }
      if (!ok) failed = true;
      __syncthreads();
      // lane l takes the candidate of group l (and folds in group l + 64 in
      // the order of the wave reduction: larger key, then smaller index)
      double tk = -1.0;
      int ti = INT_MAX;
      if (lane < P) {
        tk = join64(xs[3 * lane], xs[3 * lane + 1]);
        ti = (int)xs[3 * lane + 2];
      }
      if constexpr (WIDE) {
        const int g = lane + 64;
        if (g < P) {
          const double gk = join64(xs[3 * g], xs[3 * g + 1]);
          const int gi = (int)xs[3 * g + 2];
          if (gk > tk || (gk == tk && gi < ti)) {
            tk = gk;
            ti = gi;
          }
        }
      }
      wave_argmax(tk, ti);
      v = tk;
      widx = ti;
      const int p0 = widx >> 16;
      if (!(v >= 0.0) || p0 < 0 || p0 >= m || (widx & 0xffff) >= n) {
        // only reachable after a timeout; keep every index in range
        failed = true;
        v = 0.0;
        widx = 0;
      }
      // round trip 2: the winner's row (published with its candidate, or
      // now by the winner)
      const int wg = (widx >> 16) % P;
      if (CROSS && !same_xcd) {
        // next step's threshold: eager_frac of last key times last ratio
        // (at most 1), computed off the exchange's critical path
        prev_key = last_key;
        last_key = v;
        eager_key = a.eager_frac * last_key * fmin(1.0, last_key / prev_key);
      }
      if (CROSS && !eager && w == wg && !failed) {
        const int rho = ((widx >> 16) - w) / P;
        if (wv == rho % WAVES) publish_row<RS, CS, CX>(mine, s, si, rho / WAVES, cv, flag, same_xcd);
      }
      ok = poll_words<(128 * EW * CS + NT - 1) / NT, NT>(slot_base + (size_t)wg * per + 3, 2 * EW * n, want,
                                                     a.abort_word, a.spin_limit, xrow);
      if (!ok) failed = true;
      if (failed) gfail = 1;
      __syncthreads();
      // a failed wait anywhere in the group fails the whole group, so that
      // every lane takes the same path out
      failed = gfail != 0;
      if (kShareNorm && needY) {
        // the pivot row divided by the pivot, for the rows of B: one division
        // per entry for the whole group instead of one per entry and wave
        const int qq = widx & 0xffff;
        if constexpr (CX) {
          const double pr = join64(xrow[4 * qq], xrow[4 * qq + 1]), pm = join64(xrow[4 * qq + 2], xrow[4 * qq + 3]);
          const double dd = cabs2(pr, pm);
          for (int j = threadIdx.x; j < n; j += NT) {
            const double ur = join64(xrow[4 * j], xrow[4 * j + 1]), um = join64(xrow[4 * j + 2], xrow[4 * j + 3]);
            const double a1 = ur * pr, a2 = um * pm, b1 = um * pr, b2 = ur * pm;
            xrn[2 * j] = (a1 + a2) / dd;
            xrn[2 * j + 1] = (b1 - b2) / dd;
          }
        } else {
          const double pv = join64(xrow[2 * qq], xrow[2 * qq + 1]);
          for (int j = threadIdx.x; j < n; j += NT) xrn[j] = join64(xrow[2 * j], xrow[2 * j + 1]) / pv;
        }
        __syncthreads();
      }
#pragma unroll
      for (int b = 0; b < CS; ++b) {
        const int j = lane + 64 * b;
        u[b] = cv[b] ? join64(xrow[2 * EW * j], xrow[2 * EW * j + 1]) : 0.0;
        if constexpr (CX) ui[b] = cv[b] ? join64(xrow[4 * j + 2], xrow[4 * j + 3]) : 0.0;
      }
      if (failed) {
        v = 0.0;
        widx = 0;
#pragma unroll
        for (int b = 0; b < CS; ++b) {
          u[b] = 0.0;
          if constexpr (CX) ui[b] = 0.0;
        }
        if (threadIdx.x == 0 && a.err) atomicOr(a.err, ERR_TIMEOUT);
      }
    }
    // pivot magnitude: the key itself (real) or its square root (complex)
    if constexpr (CX) v = sqrt(v);

    const int p = widx >> 16;
    const int q = widx & 0xffff;
    const int qb = q >> 6;
    const int ql = q & 63;

    // ---- stop rules
    if (k == 0) tol = fmax(a.tol, a.tol_rel * v);
    if (a.rule == RULE_EXCLUSIVE) {
      if (k == a.maxrank) { eps = v; final_rank = k; break; }
      if (k >= 1 && v <= tol) { eps = v; final_rank = k; break; }
    } else if (k >= 1 && v == 0.0) {
      eps = 0.0;
      final_rank = k;
      break;
    }
    const double piv = lane_pick<CS>(u, qb, ql);
    double pivi = 0.0;
    if constexpr (CX) pivi = lane_pick<CS>(ui, qb, ql);
    if (w == 0 && threadIdx.x == 0) {
      a.rows[k] = p;
      a.cols[k] = q;
    }
    if (piv == 0.0 && pivi == 0.0) {
      // all-zero matrix (only possible at k == 0): one pivot at the tie-break
      // cell, B = unit row e_q, error 0
#pragma unroll
      for (int r = 0; r < RS; ++r)
        if (row0 + rstride * r == p && needY) {
          brows |= 1u << r;
          pstep[r] = 0;
#pragma unroll
          for (int b = 0; b < CS; ++b) {
            s[r][b] = (lane + 64 * b == q) ? 1.0 : 0.0;
            if constexpr (CX) si[r][b] = 0.0;
          }
        }
      eps = 0.0;
      final_rank = 1;
      break;
    }
    const double den = CX ? cabs2(piv, pivi) : 0.0;

    // ---- elimination, fused with the next step's local maxima
    // slot of the pivot row in this wave (-1: another wave or group owns it)
    const int rp = ((p - row0) % rstride == 0 && p >= row0) ? (p - row0) / rstride : -1;
    // multipliers s_iq / pivot of the rows: one vector division with lane r
    // dividing row r's entry (correctly rounded, like a scalar division)
    double quo, quoi = 0.0;
    {
      double num = 0.0, numi = 0.0;
#pragma unroll
      for (int c = 0; c < CS; ++c)
        if (c == qb) {
#pragma unroll
          for (int r = 0; r < RS; ++r) {
            const double sq = readlane_f64(s[r][c], ql);
            num = lane == r ? sq : num;
            if constexpr (CX) {
              const double sqi = readlane_f64(si[r][c], ql);
              numi = lane == r ? sqi : numi;
            }
          }
        }
      if constexpr (CX) {
        // (num + i numi) conj(pivot) / |pivot|^2
        const double a1 = num * piv, a2 = numi * pivi;
        const double b1 = numi * piv, b2 = num * pivi;
        quo = (a1 + a2) / den;
        quoi = (b1 - b2) / den;
      } else {
        quo = num / piv;
      }
    }
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      if ((alive >> r) & 1u) {
        if (r == rp) {
          rm[r] = -1.0;
          alive &= ~(1u << r);
          if (needY) {
            brows |= 1u << r;
            pstep[r] = k;
#pragma unroll
            for (int b = 0; b < CS; ++b) {
              if constexpr (CX) {
                const double sr = s[r][b], sm = si[r][b];
                const double a1 = sr * piv, a2 = sm * pivi, b1 = sm * piv, b2 = sr * pivi;
                s[r][b] = (a1 + a2) / den;
                si[r][b] = (b1 - b2) / den;
              } else {
                s[r][b] = s[r][b] / piv;
              }
            }
          }
        } else {
          const double c = readlane_f64(quo, r);
          double cim = 0.0;
          if constexpr (CX) cim = readlane_f64(quoi, r);
#pragma unroll
          for (int b = 0; b < CS; ++b) {
            if constexpr (CX) {
              const double t1 = c * u[b], t2 = cim * ui[b];
              const double tr = t1 - t2;
              const double t3 = c * ui[b], t4 = cim * u[b];
              const double tim = t3 + t4;
              s[r][b] = s[r][b] - tr;
              si[r][b] = si[r][b] - tim;
            } else {
              const double t = c * u[b];
              s[r][b] = s[r][b] - t;
            }
          }
          // eliminated column q: exactly zero from now on
#pragma unroll
          for (int b = 0; b < CS; ++b)
            if (b == qb) {
              s[r][b] = lane == ql ? 0.0 : s[r][b];
              if constexpr (CX) si[r][b] = lane == ql ? 0.0 : si[r][b];
            }
          double mx = 0.0;
#pragma unroll
          for (int b = 0; b < CS; ++b) mx = fmax(mx, CX ? cabs2(s[r][b], si[CX ? r : 0][CX ? b : 0]) : fabs(s[r][b]));
          rm[r] = mx;
        }
      }
    }
    alive = __builtin_amdgcn_readfirstlane(alive);
    if (needY) {
      brows = __builtin_amdgcn_readfirstlane(brows);
      // rows of B chosen at earlier steps: reduce them against the new pivot
      // row normalised by the pivot (Gauss-Jordan), so that B[:, J] = I
#pragma unroll
      for (int b = 0; b < CS; ++b) {
        if constexpr (CX && kShareNorm) {
          const int j = lane + 64 * b;
          u[b] = cv[b] ? xrn[2 * j] : 0.0;
          ui[b] = cv[b] ? xrn[2 * j + 1] : 0.0;
        } else if constexpr (CX) {
          const double ur = u[b], um = ui[b];
          const double a1 = ur * piv, a2 = um * pivi, b1 = um * piv, b2 = ur * pivi;
          u[b] = (a1 + a2) / den;
          ui[b] = (b1 - b2) / den;
        } else if (!kShareNorm) {
          u[b] = u[b] / piv;
        } else {
          // divided once per group after the row arrived; columns past n
          // are never read
          u[b] = cv[b] ? xrn[lane + 64 * b] : 0.0;
        }
      }
#pragma unroll
      for (int r = 0; r < RS; ++r) {
        if (((brows >> r) & 1u) && r != rp) {
          const double c = lane_pick<CS>(s[r], qb, ql);
          if constexpr (CX) {
            const double cim = lane_pick<CS>(si[r], qb, ql);
#pragma unroll
            for (int b = 0; b < CS; ++b) {
              const double t1 = c * u[b], t2 = cim * ui[b];
              const double tr = t1 - t2;
              const double t3 = c * ui[b], t4 = cim * u[b];
              const double tim = t3 + t4;
              s[r][b] = s[r][b] - tr;
              si[r][b] = si[r][b] - tim;
            }
          } else {
#pragma unroll
            for (int b = 0; b < CS; ++b) {
              const double t = c * u[b];
              s[r][b] = s[r][b] - t;
            }
          }
        }
      }
    }
    ++k;
    if (a.rule == RULE_LITERAL) {
      eps = v;
      if (v <= tol || k == a.maxrank) {
        final_rank = k;
        break;
      }
    }
  }

  if (needY) {
#pragma unroll
    for (int r = 0; r < RS; ++r)
      if (((brows >> r) & 1u) && pstep[r] >= 0 && pstep[r] < final_rank) {
#pragma unroll
        for (int b = 0; b < CS; ++b)
          if (cv[b]) {
            const size_t o = (size_t)pstep[r] * ldy + lane + 64 * b;
            a.Y[EW * o] = s[r][b];
            if constexpr (CX) a.Y[2 * o + 1] = si[r][b];
          }
      }
  }
  if (w == 0 && threadIdx.x == 0) {
    if (a.epoch) {
      // every group read the epoch before its first candidate, and group 0
      // has seen all of them, so the next launch's flags can be published
      uint32_t next = fbase + kFlagStride;
      if (next < kFlagStride) next = 1;
      __hip_atomic_store(a.epoch, next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
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

template <int RS, int CS, bool SOLO, bool CX, int W>
__global__ __launch_bounds__(64 * W) void prrlu_kernel(PrrluArgs a) {
  if ((int)(blockIdx.x % a.stride) != (a.stride == 8 ? a.xcd : 0)) return;
  // a proposal already supplied this factorisation (every group reads the
  // same word, so the whole launch leaves together; the epoch is untouched)
  if (a.skip && *a.skip) return;
  prrlu_body<RS, CS, SOLO, CX, W>(a, blockIdx.x / a.stride);
}

// The same for launches whose groups may span several XCDs (stride 1), with
// the late row publication; launches kept on one XCD (stride 8) use
// prrlu_kernel, whose exchange code is shorter without it.
template <int RS, int CS, bool CX, int W>
__global__ __launch_bounds__(64 * W) void prrlu_cross_kernel(PrrluArgs a) {
  if ((int)(blockIdx.x % a.stride) != (a.stride == 8 ? a.xcd : 0)) return;
  if (a.skip && *a.skip) return;
  prrlu_body<RS, CS, false, CX, W, true>(a, blockIdx.x / a.stride);
}

// Several products' factorisations in one launch.  Workgroup b runs on XCD
// b % 8 (the dispatcher deals workgroups round robin over the XCDs); slot
// b / 8 of that XCD belongs to the product and group the placement names, or
// is idle.  Every product's groups share one XCD, so its exchange stays in
// that XCD's L2.
template <int RS, int CS, bool CX, int W>
__global__ __launch_bounds__(64 * W) void prrlu_batch_kernel(PrrluBatchArgs bt) {
  const int x = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int prod = bt.prod[x][slot];
  if (prod < 0) return;
  const PrrluArgs& a = bt.a[prod];
  if (a.skip && *a.skip) return;
  prrlu_body<RS, CS, false, CX, W>(a, bt.group[x][slot]);
}

// Resident workgroups per CU of one kernel instance.
int resident_per_cu(const void* fn, int threads, size_t lds) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, lds) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return nb < 1 ? 1 : nb;
}

// LDS a cooperative launch requests: more than half of a CU's LDS when a
// group may take that much, so that no two cooperating groups share a CU (and
// its SIMDs); otherwise just what the kernel uses.
size_t group_lds(size_t need) {
  static size_t v = 0;
  if (!v) {
    int dev = 0, per_block = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess) {
      (void)hipGetLastError();
      per_block = per_cu = 0;
    }
    const size_t want = (size_t)per_cu / 2 + 1024;
    v = (per_cu > 0 && (size_t)per_block >= want) ? want : 1;
  }
  return v > need ? v : need;
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

// Register shapes: CS column slots per lane (n <= 64 CS), RS row slots per
// wave (rows per group = 4 RS).
struct Shape {
  int cs, rs_max;
};
constexpr Shape kShapes[] = {{1, 16}, {2, 16}, {4, 16}, {6, 8}, {8, 8}, {12, 4}, {16, 4}};

hipError_t do_launch(const void* fn, dim3 grid, int threads, size_t lds, PrrluArgs& args, hipStream_t s) {
  hipError_t e;
  if (args.cooperative) {
    void* kp[] = {&args};
    e = hipLaunchCooperativeKernel(fn, grid, dim3(threads), kp, (unsigned)lds, s);
  } else {
    // plain launch (stream capture): at most one XCD's worth of groups, one
    // per CU, so all of them become resident once the CUs are free
    void* kp[] = {&args};
    e = hipLaunchKernel(fn, grid, dim3(threads), kp, lds, s);
  }
  if (e != hipSuccess) (void)hipGetLastError();
  return e;
}

// Real groups of at least 16 rows run as eight waves of half the row slots
// (same rows per group, same exchange): two waves per SIMD hide each other's
// latencies in the in-CU part of a step.  Complex groups, smaller groups and
// rows too wide for half the registers keep four waves.
template <int RS, int CS, bool CX>
constexpr bool eight_waves() { return !CX && RS >= 4 && CS < 16 && (RS / 2) * CS <= 32; }

template <int RS, int CS, bool CX>
hipError_t launch_shape(const PrrluArgs& a, hipStream_t s) {
  PrrluArgs args = a;
  constexpr int EW = CX ? 2 : 1;
  constexpr bool W8 = eight_waves<RS, CS, CX>();
  constexpr int RSG = W8 ? RS / 2 : RS, WG = W8 ? 8 : WAVES;
  // xcd < 0 ("spread"): exactly P workgroups, dealt round robin over the
  // XCDs, for launches that overlap with other spinning launches: a launch
  // of 8P workgroups would also need CUs on the other XCDs for its idle
  // workgroups, and two such launches can each wait for the other's CUs
  const bool spread = a.xcd < 0;
  if (a.P == 1) {
    // one group: 8 workgroups of which the one on the requested XCD runs
    args.stride = (a.cooperative || spread) ? 1 : 8;
    const size_t lds = (size_t)lds_words<CS, CX>() * 4;
    return do_launch((const void*)prrlu_kernel<RS, CS, true, CX, WAVES>, dim3(args.stride), NT, lds, args, s);
  }
  const void* fn = (const void*)prrlu_kernel<RSG, CS, false, CX, WG>;
  const void* fn_cross = (const void*)prrlu_cross_kernel<RSG, CS, CX, WG>;
  const size_t lds = group_lds((size_t)lds_words<CS, CX>() * 4);
  if (spread) {
    args.stride = 1;
    return do_launch(fn_cross, dim3(args.P), 64 * WG, lds, args, s);
  }
  static int per_cu = resident_per_cu(fn, 64 * WG, lds);
  // Workgroups are dealt to the 8 XCDs round robin, so launching 8x the
  // groups and keeping every 8th (offset by the XCD index) puts the
  // cooperating groups on one XCD, which lets the exchange stay in that
  // XCD's L2.  Only when they all fit.
  args.stride = (a.P <= per_cu * cus_per_xcd()) ? 8 : 1;
  if (!a.cooperative && args.stride != 8) return hipErrorInvalidValue;
  return do_launch(args.stride == 8 ? fn : fn_cross, dim3(args.P * args.stride), 64 * WG, lds, args, s);
}

// Register shapes of complex matrices (two doubles per entry).
// Columns up to 1024 take 16 slots of two doubles: two rows per wave fill the
// registers, so a 1024-row matrix spreads over 128 groups.
constexpr Shape kShapesC[] = {{1, 8}, {2, 8}, {4, 8}, {8, 4}, {16, 2}};

const Shape* pick_shape(int nmax, bool cx = false) {
  if (cx) {
    for (const Shape& sh : kShapesC)
      if (64 * sh.cs >= nmax) return &sh;
    return nullptr;
  }
  for (const Shape& sh : kShapes)
    if (64 * sh.cs >= nmax) return &sh;
  return nullptr;
}

// Rows per group: the fewest register slots that keep the group count within
// one XCD (one group per CU), unless one group can hold all rows.  More
// groups spread the elimination over more CUs; past one XCD the exchange has
// to go through device-scope memory, which costs more than the shorter
// update saves.
int pick_rs(const Shape& sh, int mmax, int max_groups) {
  // one workgroup when the rows fit in its registers: the exchange then
  // stays in LDS, which beats any split of so few rows over several CUs
  int rs = 1;
  while (rs < sh.rs_max && WAVES * rs < mmax) rs *= 2;
  if (WAVES * rs >= mmax) return rs;
  int target_p = cus_per_xcd();
  if (max_groups > 0 && max_groups < target_p) target_p = max_groups;
  rs = 1;
  while (rs < sh.rs_max && (mmax + WAVES * rs - 1) / (WAVES * rs) > target_p) rs *= 2;
  return rs;
}

template <bool CX>
hipError_t launch_instance(const PrrluArgs& a, int cs, int rs, hipStream_t s) {
  if (CX) {
    switch (cs * 32 + rs) {
      case 1 * 32 + 1: return launch_shape<1, 1, true>(a, s);
      case 1 * 32 + 2: return launch_shape<2, 1, true>(a, s);
      case 1 * 32 + 4: return launch_shape<4, 1, true>(a, s);
      case 1 * 32 + 8: return launch_shape<8, 1, true>(a, s);
      case 2 * 32 + 1: return launch_shape<1, 2, true>(a, s);
      case 2 * 32 + 2: return launch_shape<2, 2, true>(a, s);
      case 2 * 32 + 4: return launch_shape<4, 2, true>(a, s);
      case 2 * 32 + 8: return launch_shape<8, 2, true>(a, s);
      case 4 * 32 + 1: return launch_shape<1, 4, true>(a, s);
      case 4 * 32 + 2: return launch_shape<2, 4, true>(a, s);
      case 4 * 32 + 4: return launch_shape<4, 4, true>(a, s);
      case 4 * 32 + 8: return launch_shape<8, 4, true>(a, s);
      case 8 * 32 + 1: return launch_shape<1, 8, true>(a, s);
      case 8 * 32 + 2: return launch_shape<2, 8, true>(a, s);
      case 8 * 32 + 4: return launch_shape<4, 8, true>(a, s);
      case 16 * 32 + 1: return launch_shape<1, 16, true>(a, s);
      case 16 * 32 + 2: return launch_shape<2, 16, true>(a, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (cs * 32 + rs) {
    case 1 * 32 + 1: return launch_shape<1, 1, false>(a, s);
    case 1 * 32 + 2: return launch_shape<2, 1, false>(a, s);
    case 1 * 32 + 4: return launch_shape<4, 1, false>(a, s);
    case 1 * 32 + 8: return launch_shape<8, 1, false>(a, s);
    case 1 * 32 + 16: return launch_shape<16, 1, false>(a, s);
    case 2 * 32 + 1: return launch_shape<1, 2, false>(a, s);
    case 2 * 32 + 2: return launch_shape<2, 2, false>(a, s);
    case 2 * 32 + 4: return launch_shape<4, 2, false>(a, s);
    case 2 * 32 + 8: return launch_shape<8, 2, false>(a, s);
    case 2 * 32 + 16: return launch_shape<16, 2, false>(a, s);
    case 4 * 32 + 1: return launch_shape<1, 4, false>(a, s);
    case 4 * 32 + 2: return launch_shape<2, 4, false>(a, s);
    case 4 * 32 + 4: return launch_shape<4, 4, false>(a, s);
    case 4 * 32 + 8: return launch_shape<8, 4, false>(a, s);
    case 4 * 32 + 16: return launch_shape<16, 4, false>(a, s);
    case 6 * 32 + 1: return launch_shape<1, 6, false>(a, s);
    case 6 * 32 + 2: return launch_shape<2, 6, false>(a, s);
    case 6 * 32 + 4: return launch_shape<4, 6, false>(a, s);
    case 6 * 32 + 8: return launch_shape<8, 6, false>(a, s);
    case 8 * 32 + 1: return launch_shape<1, 8, false>(a, s);
    case 8 * 32 + 2: return launch_shape<2, 8, false>(a, s);
    case 8 * 32 + 4: return launch_shape<4, 8, false>(a, s);
    case 8 * 32 + 8: return launch_shape<8, 8, false>(a, s);
    case 12 * 32 + 1: return launch_shape<1, 12, false>(a, s);
    case 12 * 32 + 2: return launch_shape<2, 12, false>(a, s);
    case 12 * 32 + 4: return launch_shape<4, 12, false>(a, s);
    case 16 * 32 + 1: return launch_shape<1, 16, false>(a, s);
    case 16 * 32 + 2: return launch_shape<2, 16, false>(a, s);
    case 16 * 32 + 4: return launch_shape<4, 16, false>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int prrlu_xcd_cus() { return cus_per_xcd(); }

int prrlu_groups(int mmax, int nmax, int max_groups, int cplx) {
  if (mmax < 1 || nmax < 1 || mmax > ACI_MAX_MATRIX || nmax > ACI_MAX_MATRIX) return -1;
  const Shape* sh = pick_shape(nmax, cplx != 0);
  if (!sh) return -1;
  const int rs = pick_rs(*sh, mmax, max_groups);
  return (mmax + WAVES * rs - 1) / (WAVES * rs);
}

size_t prrlu_xbuf_words(int mmax, int nmax, int cplx) {
  // every launch uses at most kMaxGroups groups of at most 4 + 2 EW n words per parity
  (void)mmax;
  const int ew = cplx ? 2 : 1;
  const Shape* sh = pick_shape(nmax < 1 ? 1 : nmax, cplx != 0);
  if (!sh) sh = cplx ? &kShapesC[sizeof(kShapesC) / sizeof(kShapesC[0]) - 1]
                     : &kShapes[sizeof(kShapes) / sizeof(kShapes[0]) - 1];
  return (size_t)2 * kMaxGroups * (4 + 2 * ew * 64 * sh->cs);
}

size_t prrlu_xbuf_used(int mmax, int nmax, int max_groups, int cplx) {
  if (mmax < 1 || nmax < 1 || mmax > ACI_MAX_MATRIX || nmax > ACI_MAX_MATRIX) return 0;
  const Shape* sh = pick_shape(nmax, cplx != 0);
  if (!sh) return 0;
  const int rs = pick_rs(*sh, mmax, max_groups);
  const int P = (mmax + WAVES * rs - 1) / (WAVES * rs);
  return (size_t)2 * P * (4 + 2 * (cplx ? 2 : 1) * 64 * sh->cs);
}

int prrlu_variant(int mmax, int nmax, int max_groups, int cplx) {
  if (mmax < 1 || nmax < 1 || mmax > ACI_MAX_MATRIX || nmax > ACI_MAX_MATRIX) return -1;
  const Shape* sh = pick_shape(nmax, cplx != 0);
  if (!sh) return -1;
  const int rs = pick_rs(*sh, mmax, max_groups);
  const int P = (mmax + WAVES * rs - 1) / (WAVES * rs);
  if (P > 1 && !cplx && rs >= 4 && sh->cs < 16 && (rs / 2) * sh->cs <= 32)   // eight waves (eight_waves)
    return 1000000 + 100 * (rs / 2) + sh->cs;
  return (cplx ? 100000 : 0) + (P == 1 ? 10000 : 0) + 100 * rs + sh->cs;
}

// Batch placement: the fewest row slots per wave for which every product's
// groups (one per CU) fit on one XCD, products dealt largest first to the
// least loaded XCD.
static bool batch_place(const int* mmax, int count, const Shape& sh, int& rs, int* P, PrrluBatchArgs* out) {
  const int cap = std::min(cus_per_xcd(), kBatchSlots);
  if (count < 1 || count > kBatchMaxProducts) return false;
  for (rs = 1; rs <= sh.rs_max; rs *= 2) {
    bool ok = true;
    int order[kBatchMaxProducts];
    for (int b = 0; b < count; ++b) {
      P[b] = (std::max(mmax[b], 1) + WAVES * rs - 1) / (WAVES * rs);
      ok = ok && P[b] <= cap;
      order[b] = b;
    }
    if (!ok) continue;
    std::stable_sort(order, order + count, [&](int x, int y) { return P[x] > P[y]; });
    int load[8] = {0, 0, 0, 0, 0, 0, 0, 0}, xcd_of[kBatchMaxProducts], start[kBatchMaxProducts];
    for (int i = 0; i < count && ok; ++i) {
      const int b = order[i];
      int x = 0;
      for (int y = 1; y < 8; ++y)
        if (load[y] < load[x]) x = y;
      if (load[x] + P[b] > cap) ok = false;
      xcd_of[b] = x;
      start[b] = load[x];
      load[x] += P[b];
    }
    if (!ok) continue;
    if (out) {
      for (int x = 0; x < 8; ++x)
        for (int t = 0; t < kBatchSlots; ++t) {
          out->prod[x][t] = -1;
          out->group[x][t] = 0;
        }
      for (int b = 0; b < count; ++b)
        for (int g = 0; g < P[b]; ++g) {
          out->prod[xcd_of[b]][start[b] + g] = (int8_t)b;
          out->group[xcd_of[b]][start[b] + g] = (uint8_t)g;
        }
    }
    return true;
  }
  return false;
}

template <int RS, int CS, bool CX>
hipError_t launch_batch_shape(const PrrluBatchArgs& bt, int slots, hipStream_t s) {
  constexpr int EW = CX ? 2 : 1;
  constexpr bool W8 = eight_waves<RS, CS, CX>();
  constexpr int RSG = W8 ? RS / 2 : RS, WG = W8 ? 8 : WAVES;
  const void* fn = (const void*)prrlu_batch_kernel<RSG, CS, CX, WG>;
  const size_t lds = group_lds((size_t)lds_words<CS, CX>() * 4);
  PrrluBatchArgs args = bt;
  void* kp[] = {&args};
  const hipError_t e = hipLaunchKernel(fn, dim3(8 * slots), dim3(64 * WG), kp, lds, s);
  if (e != hipSuccess) (void)hipGetLastError();
  return e;
}

template <bool CX>
hipError_t launch_batch_instance(const PrrluBatchArgs& bt, int slots, int cs, int rs, hipStream_t s) {
  if (CX) {
    switch (cs * 32 + rs) {
      case 1 * 32 + 1: return launch_batch_shape<1, 1, true>(bt, slots, s);
      case 1 * 32 + 2: return launch_batch_shape<2, 1, true>(bt, slots, s);
      case 1 * 32 + 4: return launch_batch_shape<4, 1, true>(bt, slots, s);
      case 1 * 32 + 8: return launch_batch_shape<8, 1, true>(bt, slots, s);
      case 2 * 32 + 1: return launch_batch_shape<1, 2, true>(bt, slots, s);
      case 2 * 32 + 2: return launch_batch_shape<2, 2, true>(bt, slots, s);
      case 2 * 32 + 4: return launch_batch_shape<4, 2, true>(bt, slots, s);
      case 2 * 32 + 8: return launch_batch_shape<8, 2, true>(bt, slots, s);
      case 4 * 32 + 1: return launch_batch_shape<1, 4, true>(bt, slots, s);
      case 4 * 32 + 2: return launch_batch_shape<2, 4, true>(bt, slots, s);
      case 4 * 32 + 4: return launch_batch_shape<4, 4, true>(bt, slots, s);
      case 4 * 32 + 8: return launch_batch_shape<8, 4, true>(bt, slots, s);
      case 8 * 32 + 1: return launch_batch_shape<1, 8, true>(bt, slots, s);
      case 8 * 32 + 2: return launch_batch_shape<2, 8, true>(bt, slots, s);
      case 8 * 32 + 4: return launch_batch_shape<4, 8, true>(bt, slots, s);
      case 16 * 32 + 1: return launch_batch_shape<1, 16, true>(bt, slots, s);
      case 16 * 32 + 2: return launch_batch_shape<2, 16, true>(bt, slots, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (cs * 32 + rs) {
    case 1 * 32 + 1: return launch_batch_shape<1, 1, false>(bt, slots, s);
    case 1 * 32 + 2: return launch_batch_shape<2, 1, false>(bt, slots, s);
    case 1 * 32 + 4: return launch_batch_shape<4, 1, false>(bt, slots, s);
    case 1 * 32 + 8: return launch_batch_shape<8, 1, false>(bt, slots, s);
    case 1 * 32 + 16: return launch_batch_shape<16, 1, false>(bt, slots, s);
    case 2 * 32 + 1: return launch_batch_shape<1, 2, false>(bt, slots, s);
    case 2 * 32 + 2: return launch_batch_shape<2, 2, false>(bt, slots, s);
    case 2 * 32 + 4: return launch_batch_shape<4, 2, false>(bt, slots, s);
    case 2 * 32 + 8: return launch_batch_shape<8, 2, false>(bt, slots, s);
    case 2 * 32 + 16: return launch_batch_shape<16, 2, false>(bt, slots, s);
    case 4 * 32 + 1: return launch_batch_shape<1, 4, false>(bt, slots, s);
    case 4 * 32 + 2: return launch_batch_shape<2, 4, false>(bt, slots, s);
    case 4 * 32 + 4: return launch_batch_shape<4, 4, false>(bt, slots, s);
    case 4 * 32 + 8: return launch_batch_shape<8, 4, false>(bt, slots, s);
    case 4 * 32 + 16: return launch_batch_shape<16, 4, false>(bt, slots, s);
    case 6 * 32 + 1: return launch_batch_shape<1, 6, false>(bt, slots, s);
    case 6 * 32 + 2: return launch_batch_shape<2, 6, false>(bt, slots, s);
    case 6 * 32 + 4: return launch_batch_shape<4, 6, false>(bt, slots, s);
    case 6 * 32 + 8: return launch_batch_shape<8, 6, false>(bt, slots, s);
    case 8 * 32 + 1: return launch_batch_shape<1, 8, false>(bt, slots, s);
    case 8 * 32 + 2: return launch_batch_shape<2, 8, false>(bt, slots, s);
    case 8 * 32 + 4: return launch_batch_shape<4, 8, false>(bt, slots, s);
    case 8 * 32 + 8: return launch_batch_shape<8, 8, false>(bt, slots, s);
    case 12 * 32 + 1: return launch_batch_shape<1, 12, false>(bt, slots, s);
    case 12 * 32 + 2: return launch_batch_shape<2, 12, false>(bt, slots, s);
    case 12 * 32 + 4: return launch_batch_shape<4, 12, false>(bt, slots, s);
    case 16 * 32 + 1: return launch_batch_shape<1, 16, false>(bt, slots, s);
    case 16 * 32 + 2: return launch_batch_shape<2, 16, false>(bt, slots, s);
    case 16 * 32 + 4: return launch_batch_shape<4, 16, false>(bt, slots, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_prrlu(const PrrluArgs& a0, int mmax, int nmax, hipStream_t s) {
  if (mmax < 1 || nmax < 1 || mmax > ACI_MAX_MATRIX || nmax > ACI_MAX_MATRIX) return hipErrorInvalidValue;
  const bool cx = a0.cplx != 0;
  const Shape* sh = pick_shape(nmax, cx);
  if (!sh) return hipErrorInvalidValue;
  PrrluArgs a = a0;
  const int rs = pick_rs(*sh, mmax, a.max_groups);
  a.P = (mmax + WAVES * rs - 1) / (WAVES * rs);
  if (a.xcd > 7 || (a.xcd < 0 && a.cooperative)) return hipErrorInvalidValue;
  if (a.P > ((cx && sh->cs == 16) ? kMaxGroups : 64)) return hipErrorInvalidValue;
  a.xwords = 4 + 2 * (cx ? 2 : 1) * 64 * sh->cs;
  if ((size_t)2 * a.P * a.xwords > a.xbuf_words) return hipErrorInvalidValue;
  return cx ? launch_instance<true>(a, sh->cs, rs, s) : launch_instance<false>(a, sh->cs, rs, s);
}

int prrlu_batch_variant(const int* mmax, int count, int nmax, int cplx) {
  if (count < 1 || count > kBatchMaxProducts || nmax < 1 || nmax > ACI_MAX_MATRIX) return -1;
  for (int b = 0; b < count; ++b)
    if (mmax[b] < 1 || mmax[b] > ACI_MAX_MATRIX) return -1;
  const Shape* sh = pick_shape(nmax, cplx != 0);
  if (!sh) return -1;
  int rs = 0, P[kBatchMaxProducts];
  if (!batch_place(mmax, count, *sh, rs, P, nullptr)) return -1;
  if (!cplx && rs >= 4 && sh->cs < 16 && (rs / 2) * sh->cs <= 32)   // eight waves (eight_waves)
    return 2000000 + 100 * (rs / 2) + sh->cs;
  return 200000 + (cplx ? 100000 : 0) + 100 * rs + sh->cs;
}

hipError_t launch_prrlu_batch(const PrrluArgs* a, const int* mmax, int count, int nmax, hipStream_t s) {
  if (count < 1 || count > kBatchMaxProducts || nmax < 1 || nmax > ACI_MAX_MATRIX) return hipErrorInvalidValue;
  const bool cx = a[0].cplx != 0;
  for (int b = 0; b < count; ++b)
    if (mmax[b] < 1 || mmax[b] > ACI_MAX_MATRIX || (a[b].cplx != 0) != cx) return hipErrorInvalidValue;
  const Shape* sh = pick_shape(nmax, cx);
  if (!sh) return hipErrorInvalidValue;
  PrrluBatchArgs bt{};
  int rs = 0, P[kBatchMaxProducts];
  if (!batch_place(mmax, count, *sh, rs, P, &bt)) return hipErrorInvalidValue;
  const int xwords = 4 + 2 * (cx ? 2 : 1) * 64 * sh->cs;
  int slots = 0;
  for (int x = 0; x < 8; ++x)
    for (int t = 0; t < kBatchSlots; ++t)
      if (bt.prod[x][t] >= 0) slots = std::max(slots, t + 1);
  for (int b = 0; b < count; ++b) {
    bt.a[b] = a[b];
    bt.a[b].P = P[b];
    bt.a[b].stride = 1;
    bt.a[b].xwords = xwords;
    if ((size_t)2 * P[b] * xwords > a[b].xbuf_words) return hipErrorInvalidValue;
  }
  return cx ? launch_batch_instance<true>(bt, slots, sh->cs, rs, s)
            : launch_batch_instance<false>(bt, slots, sh->cs, rs, s);
}

}  // namespace aci
