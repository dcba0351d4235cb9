// mcc_device.hpp -- device building blocks for gfx950 (wave64):
// Philox4x32-10, compensated block reductions, block scans, LDS sorts and
// the scalar math of the scatter (N97 inversion, angle sampling, rotation).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mcc_kernel_args.hpp"

namespace mcc {

constexpr int WAVE = 64;
constexpr double PI_D = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Counter layout:
//   c0 = index (pair k, or particle index >> 2 for the shuffle keys)
//   c1 = global cell id, c2 = step (low 32 bits)
//   c3 = (step >> 32 & 0xFFFF) << 16 | collision << 8 | purpose
// ---------------------------------------------------------------------------
struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2,
                                     uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    // one 32x32 -> 64 product per multiplier (both halves at once)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return U4{c0, c1, c2, c3};
}

enum : uint32_t { PURPOSE_PAIR = 0, PURPOSE_SHUFFLE0 = 1 };

__device__ __forceinline__ uint32_t ctr3(uint64_t step, int coll, uint32_t purpose) {
  return (uint32_t)(((step >> 32) & 0xFFFFu) << 16) | ((uint32_t)(coll & 0xFF) << 8) | purpose;
}

// Copies ndw dwords from global memory into LDS without passing through
// registers (LDS DMA: each lane's dword lands at the wave's LDS base plus 4
// times its lane index).  Wave w copies the 64-dword chunks w, w + TPC/64,
// ...; lds_copy_wait() and a barrier make the data visible to the block.
// Both addresses must be 4-byte aligned.
template <int TPC, class T, class U>
__device__ __forceinline__ void lds_copy(const T *src, U *dst, int ndw) {
  const uint32_t *s = reinterpret_cast<const uint32_t *>(src);
  uint32_t *d = reinterpret_cast<uint32_t *>(dst);
  const int lane = threadIdx.x & 63;
  for (int d0 = (int)(threadIdx.x >> 6) * 64; d0 < ndw; d0 += TPC)
    if (d0 + lane < ndw)
      __builtin_amdgcn_global_load_lds(s + d0 + lane,
                                       (__attribute__((address_space(3))) void *)(d + d0), 4, 0,
                                       0);
}
__device__ __forceinline__ void lds_copy_wait() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// values the whole wave holds alike (read from LDS): kept in scalar registers
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ long long uni(long long x) {
  const uint64_t b = (uint64_t)x;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  return (long long)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double uni(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// uniform in (0,1), exact in FP64
__device__ __forceinline__ double unif64(uint32_t a) { return ((double)a + 0.5) * 0x1p-32; }
// FP32 uniform from the top 23 bits: (2k + 1) 2^-24 is exact in FP32 and
// lies in [2^-24, 1 - 2^-24], so no word maps to 0 or 1 (a 24-bit form
// rounds its top value to 1, and N97's inverse CDF would then take log(0)
// and return a full reversal)
__device__ __forceinline__ float unif32(uint32_t a) {
  return ((float)(a >> 9) + 0.5f) * 0x1p-23f;
}

// ---------------------------------------------------------------------------
// Wave-level exchanges on the VALU (DPP and the gfx950 permlane swaps), with
// no trip through the LDS unit
// ---------------------------------------------------------------------------
template <int CTRL, int ROWMASK = 0xF, bool BOUND = true>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWMASK, 0xF, BOUND);
}
template <int CTRL, int ROWMASK = 0xF, bool BOUND = true>
__device__ __forceinline__ double dpp_f64(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = dpp_u32<CTRL, ROWMASK, BOUND>((uint32_t)b);
  const uint32_t hi = dpp_u32<CTRL, ROWMASK, BOUND>((uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
constexpr int DPP_QP_1032 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int DPP_QP_2301 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int DPP_ROW_SHR1 = 0x111, DPP_ROW_SHR2 = 0x112, DPP_ROW_SHR4 = 0x114,
              DPP_ROW_SHR8 = 0x118;
constexpr int DPP_WAVE_SHR1 = 0x138;
constexpr int DPP_ROW_MIRROR = 0x140, DPP_ROW_HALF_MIRROR = 0x141;
constexpr int DPP_ROW_BCAST15 = 0x142, DPP_ROW_BCAST31 = 0x143;

// The two operands of level L (0..5) of a wave all-reduce: lanes pair up
// within quads (L = 0, 1), then half rows and rows (L = 2, 3: mirrored lane
// orders pair equal-valued groups), then rows of 16 (L = 4) and halves of 32
// (L = 5: permlane swaps, which hand every lane the same two values in the
// same order).  Combined with a commutative operation, every lane of a group
// gets the same bits.
template <int L>
__device__ __forceinline__ void wave_pair(double x, double &a, double &b) {
  if constexpr (L < 4) {
    constexpr int C = L == 0 ? DPP_QP_1032
                             : (L == 1 ? DPP_QP_2301 : (L == 2 ? DPP_ROW_HALF_MIRROR
                                                               : DPP_ROW_MIRROR));
    a = x;
    b = dpp_f64<C>(x);
  } else {
    const uint64_t v = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    uint32_t a0, a1, b0, b1;
    if constexpr (L == 4) {
      const auto r0 = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
      const auto r1 = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
      a0 = r0[0], b0 = r0[1], a1 = r1[0], b1 = r1[1];
    } else {
      const auto r0 = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
      const auto r1 = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
      a0 = r0[0], b0 = r0[1], a1 = r1[0], b1 = r1[1];
    }
    a = __longlong_as_double((long long)(((uint64_t)a1 << 32) | a0));
    b = __longlong_as_double((long long)(((uint64_t)b1 << 32) | b0));
  }
}
template <int L, int N>
__device__ __forceinline__ void wave_sum_level(double v[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double a, b;
    wave_pair<L>(v[i], a, b);
    v[i] = a + b;
  }
}
// sum of N values over the wave, the same bits in every lane
template <int N>
__device__ __forceinline__ void wave_sum(double v[N]) {
  wave_sum_level<0, N>(v);
  wave_sum_level<1, N>(v);
  wave_sum_level<2, N>(v);
  wave_sum_level<3, N>(v);
  wave_sum_level<4, N>(v);
  wave_sum_level<5, N>(v);
}

// inclusive prefix sums over the wave: within rows of 16 by shifted adds,
// then the totals of row 0 (into row 1), row 2 (into row 3) and rows 0-1
// (into rows 2-3) by the row broadcasts
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  x += dpp_u32<DPP_ROW_SHR1>(x);
  x += dpp_u32<DPP_ROW_SHR2>(x);
  x += dpp_u32<DPP_ROW_SHR4>(x);
  x += dpp_u32<DPP_ROW_SHR8>(x);
  x += dpp_u32<DPP_ROW_BCAST15, 0xA, false>(x);
  x += dpp_u32<DPP_ROW_BCAST31, 0xC, false>(x);
  return x;
}
__device__ __forceinline__ double wave_incl_scan(double x) {
  x += dpp_f64<DPP_ROW_SHR1>(x);
  x += dpp_f64<DPP_ROW_SHR2>(x);
  x += dpp_f64<DPP_ROW_SHR4>(x);
  x += dpp_f64<DPP_ROW_SHR8>(x);
  x += dpp_f64<DPP_ROW_BCAST15, 0xA, false>(x);
  x += dpp_f64<DPP_ROW_BCAST31, 0xC, false>(x);
  return x;
}
// the value of the previous lane (0 in lane 0)
__device__ __forceinline__ double wave_shr1(double x) { return dpp_f64<DPP_WAVE_SHR1>(x); }
// the value of lane `lane` (a uniform index), in every lane
__device__ __forceinline__ double wave_bcast(double x, int lane) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, lane);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), lane);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// ---------------------------------------------------------------------------
// Error-free transforms and compensated block sums
// ---------------------------------------------------------------------------
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// accumulate x into (s, c) Neumaier-style, branch-free via TwoSum
__device__ __forceinline__ void csum_add(double &s, double &c, double x) {
  double t, e;
  two_sum(s, x, t, e);
  s = t;
  c += e;
}

// level L of a compensated wave all-reduce of (s, c): TwoSum of the pair's
// sums (its error term does not depend on the operand order) and the sum of
// their compensations
template <int L>
__device__ __forceinline__ void wave_csum_level(double &s, double &c) {
  double sa, sb, ca, cb, t, e;
  wave_pair<L>(s, sa, sb);
  wave_pair<L>(c, ca, cb);
  two_sum(sa, sb, t, e);
  s = t;
  c = ca + cb + e;
}
__device__ __forceinline__ void wave_csum(double &s, double &c) {
  wave_csum_level<0>(s, c);
  wave_csum_level<1>(s, c);
  wave_csum_level<2>(s, c);
  wave_csum_level<3>(s, c);
  wave_csum_level<4>(s, c);
  wave_csum_level<5>(s, c);
}

template <int N>
struct CSum {
  double s[N], c[N];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < N; ++i) s[i] = c[i] = 0.0;
  }
  __device__ __forceinline__ void add(int i, double x) { csum_add(s[i], c[i], x); }
};

// Sum of N compensated values over the block; every thread receives the
// totals.  `red` is LDS scratch of at least 2*N*(TPC/64) doubles.  Ends with a
// barrier so `red` may be reused right after (with TAIL; without it, `red`
// must not be written again before the workgroup's next barrier).
template <int TPC, int N, bool G = false, bool TAIL = true>
__device__ __forceinline__ void block_csum(CSum<N> &v, double *red, double out[N]) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = threadIdx.x / WAVE;
  constexpr int NW = TPC / WAVE;
#pragma unroll
  for (int i = 0; i < N; ++i) wave_csum(v.s[i], v.c[i]);
  if (NW == 1) {
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = v.s[i] + v.c[i];
    __syncthreads();
    return;
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      red[(wid * N + i) * 2] = v.s[i];
      red[(wid * N + i) * 2 + 1] = v.c[i];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double s = red[i * 2], c = red[i * 2 + 1];
    for (int w = 1; w < NW; ++w) {
      double t, e;
      two_sum(s, red[(w * N + i) * 2], t, e);
      s = t;
      c = c + red[(w * N + i) * 2 + 1] + e;
    }
    out[i] = s + c;
  }
  if constexpr (TAIL) __syncthreads();
}

// Plain FP64 sum of N values over the block; every thread receives the same
// totals (the xor butterfly adds the same two operands on both partners).
// `red` is LDS scratch of at least N*(TPC/64) doubles.  Ends with a barrier
// (without TAIL, `red` must not be written again before the next barrier).
template <int TPC, int N, bool TAIL = true>
__device__ __forceinline__ void block_sum(double v[N], double *red, double out[N]) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = threadIdx.x / WAVE;
  constexpr int NW = TPC / WAVE;
  wave_sum<N>(v);
  if (NW == 1) {
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = v[i];
    __syncthreads();
    return;
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) red[wid * N + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double acc = red[i];
    for (int w = 1; w < NW; ++w) acc += red[w * N + i];
    out[i] = acc;
  }
  if constexpr (TAIL) __syncthreads();
}

// One compensated value (s, c) and N plain values summed over the block in
// one pass; every thread receives the totals.  `red` holds at least
// (N+2)*(TPC/64) doubles.  Ends with a barrier (as block_sum with TAIL).
template <int TPC, int N, bool TAIL = true>
__device__ __forceinline__ void block_sum_c1(double &s, double &c, double v[N], double *red,
                                             double &out_c, double out[N]) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = threadIdx.x / WAVE;
  constexpr int NW = TPC / WAVE;
  wave_csum(s, c);
  wave_sum<N>(v);
  if (NW == 1) {
    out_c = s + c;
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = v[i];
    __syncthreads();
    return;
  }
  constexpr int M = N + 2;
  if (lane == 0) {
    red[wid * M] = s;
    red[wid * M + 1] = c;
#pragma unroll
    for (int i = 0; i < N; ++i) red[wid * M + 2 + i] = v[i];
  }
  __syncthreads();
  double ss = red[0], cc = red[1];
  for (int w = 1; w < NW; ++w) {
    double t, e;
    two_sum(ss, red[w * M], t, e);
    ss = t;
    cc = cc + red[w * M + 1] + e;
  }
  out_c = ss + cc;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double acc = red[2 + i];
    for (int w = 1; w < NW; ++w) acc += red[w * M + 2 + i];
    out[i] = acc;
  }
  if constexpr (TAIL) __syncthreads();
}

// Two compensated values summed over the block in one pass, each exactly as
// block_sum_c1 sums its one (same butterfly, same order across waves);
// every thread receives both totals.  `red` holds at least 4*(TPC/64)
// doubles.  Ends with a barrier (as block_sum with TAIL).
template <int TPC, bool TAIL = true>
__device__ __forceinline__ void block_sum_c2(double &s0, double &c0, double &s1, double &c1,
                                             double *red, double &out0, double &out1) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = threadIdx.x / WAVE;
  constexpr int NW = TPC / WAVE;
  wave_csum(s0, c0);
  wave_csum(s1, c1);
  if (NW == 1) {
    out0 = s0 + c0;
    out1 = s1 + c1;
    __syncthreads();
    return;
  }
  if (lane == 0) {
    red[wid * 4] = s0;
    red[wid * 4 + 1] = c0;
    red[wid * 4 + 2] = s1;
    red[wid * 4 + 3] = c1;
  }
  __syncthreads();
  double ss0 = red[0], cc0 = red[1], ss1 = red[2], cc1 = red[3];
  for (int w = 1; w < NW; ++w) {
    double t, e;
    two_sum(ss0, red[w * 4], t, e);
    ss0 = t;
    cc0 = cc0 + red[w * 4 + 1] + e;
    two_sum(ss1, red[w * 4 + 2], t, e);
    ss1 = t;
    cc1 = cc1 + red[w * 4 + 3] + e;
  }
  out0 = ss0 + cc0;
  out1 = ss1 + cc1;
  if constexpr (TAIL) __syncthreads();
}

// min and max of N u64 values over the block (all threads receive them)
template <int TPC, int N, bool G = false>
__device__ __forceinline__ void block_minmax_u64(uint64_t lo[N], uint64_t hi[N], uint64_t *red) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = threadIdx.x / WAVE;
  constexpr int NW = TPC / WAVE;
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const uint64_t a = __shfl_xor(lo[i], off);
      const uint64_t b = __shfl_xor(hi[i], off);
      lo[i] = a < lo[i] ? a : lo[i];
      hi[i] = b > hi[i] ? b : hi[i];
    }
  }
  if (NW == 1) {
    __syncthreads();
    return;
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      red[(wid * N + i) * 2] = lo[i];
      red[(wid * N + i) * 2 + 1] = hi[i];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    uint64_t a = red[i * 2], b = red[i * 2 + 1];
    for (int w = 1; w < NW; ++w) {
      const uint64_t x = red[(w * N + i) * 2], y = red[(w * N + i) * 2 + 1];
      a = x < a ? x : a;
      b = y > b ? y : b;
    }
    lo[i] = a;
    hi[i] = b;
  }
  __syncthreads();
}

// In-place exclusive scan of a[0..n) (n <= TPC*PPT); a[n] receives the total.
// Thread t owns the chunk [t*PPT, t*PPT + PPT).  wsum: TPC/64 u32 of LDS.
// Ends with a barrier.
template <int TPC, int PPT, bool G = false>
__device__ __forceinline__ void block_exclusive_scan(uint32_t *a, int n, uint32_t *wsum) {
  const int t = threadIdx.x;
  const int lane = t & (WAVE - 1);
  const int wid = t / WAVE;
  constexpr int NW = TPC / WAVE;
  const int lo = t * PPT, hi = (lo + PPT < n) ? lo + PPT : n;
  uint32_t tot = 0;
  for (int idx = lo; idx < hi; ++idx) tot += a[idx];
  const uint32_t incl = wave_incl_scan(tot);
  if (lane == WAVE - 1) wsum[wid] = incl;
  __syncthreads();
  uint32_t woff = 0, total = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const uint32_t x = wsum[w];
    if (w < wid) woff += x;
    total += x;
  }
  uint32_t ex = woff + incl - tot;
  for (int idx = lo; idx < hi; ++idx) {
    const uint32_t x = a[idx];
    a[idx] = ex;
    ex += x;
  }
  if (t == 0) a[n] = total;
  __syncthreads();
}

struct IdentityMap {
  __device__ __forceinline__ int operator()(int i) const { return i; }
};

// Exclusive prefix sum of one value per thread, in thread order; `total`
// receives the sum (all threads).  wsum: TPC/64 u32.  Ends with a barrier.
template <int TPC, bool G>
__device__ __forceinline__ uint32_t block_excl_scan1(uint32_t x, uint32_t *wsum,
                                                     uint32_t &total) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = threadIdx.x / WAVE;
  constexpr int NW = TPC / WAVE;
  const uint32_t incl = wave_incl_scan(x);
  if (lane == WAVE - 1) wsum[wid] = incl;
  __syncthreads();
  uint32_t woff = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const uint32_t v = wsum[w];
    if (w < wid) woff += v;
    tot += v;
  }
  total = tot;
  __syncthreads();
  return woff + incl - x;
}

// ---------------------------------------------------------------------------
// Bucket-rank sort in LDS.  Items 0..n-1 (n <= CAP) with a bucket function
// that is non-decreasing in the sort order and a strict total order `less`.
// out[pos] = map(item) (map: identity unless given).  The result equals a full sort by `less`; the bucket only
// decides how much comparing is needed (about one item per bucket for
// uniform keys).  cnt: u32[CAP+1]; mem: u16[CAP]; wsum: TPC/64 u32.
// occ_limit: a bucket fuller than this ends the sort right after the
// counting (out unset): the caller orders such inputs another way, since
// ranking within a bucket costs its occupancy squared.
// ZEROED: the caller has set cnt[0..n) and *maxocc to zero before a barrier
// (saving the sort's own clearing pass and its barrier).
// Returns the largest bucket occupancy (all threads).
// ---------------------------------------------------------------------------
template <int TPC, int PPT, bool G, bool ZEROED = false, class BucketF, class LessF,
          class MapF = IdentityMap>
__device__ __forceinline__ uint32_t bucket_rank_sort(int n, uint32_t *cnt, uint16_t *mem,
                                                    uint16_t *out, uint32_t *wsum,
                                                    uint32_t *maxocc, BucketF bucket,
                                                    LessF less, uint32_t *slotbuf = nullptr,
                                                    MapF map = MapF(),
                                                    uint32_t occ_limit = 0xFFFFFFFFu) {
  // G: many items per thread; the per-item slot goes to slotbuf[] (memory
  // private to the item's thread) instead of registers, and the bucket is
  // recomputed instead of kept
  const int t = threadIdx.x;
  constexpr int R = G ? 1 : PPT;
  if constexpr (!ZEROED) {
    for (int i = t; i < n; i += TPC) cnt[i] = 0u;
    if (t == 0) *maxocc = 0u;
    __syncthreads();
  }
  uint32_t bk[R], slot[R];
  uint32_t mo = 0;
  if constexpr (G) {
    for (int i = t; i < n; i += TPC) {
      const uint32_t s0 = atomicAdd(&cnt[bucket(i)], 1u);
      slotbuf[i] = s0;
      mo = s0 + 1 > mo ? s0 + 1 : mo;
    }
  } else {
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int i = t + j * TPC;
      if (i < n) {
        bk[j] = bucket(i);
        slot[j] = atomicAdd(&cnt[bk[j]], 1u);
        mo = slot[j] + 1 > mo ? slot[j] + 1 : mo;
      }
    }
  }
  __syncthreads();
  if (mo > 1) atomicMax(maxocc, mo);
  block_exclusive_scan<TPC, PPT, G>(cnt, n, wsum);
  // read here, between barriers: the next call resets *maxocc only after this
  // call's last barrier, so every thread returns the same value
  const uint32_t occ = *maxocc;
  if (occ > occ_limit) return occ;  // (uniform: read between barriers)
  if constexpr (G) {
    for (int i = t; i < n; i += TPC) mem[cnt[bucket(i)] + slotbuf[i]] = (uint16_t)i;
  } else {
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int i = t + j * TPC;
      if (i < n) mem[cnt[bk[j]] + slot[j]] = (uint16_t)i;
    }
  }
  __syncthreads();
  auto place = [&](int i, uint32_t b) {
    const uint32_t s0 = cnt[b], s1 = cnt[b + 1];
    uint32_t r = 0;
    for (uint32_t m = s0; m < s1; ++m) {
      const int o = mem[m];
      if (o != i && less(o, i)) ++r;
    }
    out[s0 + r] = (uint16_t)map(i);
  };
  if constexpr (G) {
    for (int i = t; i < n; i += TPC) place(i, bucket(i));
  } else {
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int i = t + j * TPC;
      if (i < n) place(i, bk[j]);
    }
  }
  __syncthreads();
  return occ;
}

// The bucket-rank sort of the shuffles: items 0..n-1 ordered by (key[i], i)
// ascending, out[pos] = map(item).  As bucket_rank_sort with ZEROED (cnt[0..n)
// zero before a barrier), at most PPT items per thread.  Each thread keeps its
// items' keys in registers; once they are counted, the keys are moved into
// bucket order over the key array itself (it is not read again), so ranking
// inside a bucket reads an entry's key and index with two independent loads
// instead of the index and then its key.
template <int TPC, int PPT, class BucketF, class MapF>
__device__ __forceinline__ void key_rank_sort(int n, uint32_t *key, uint32_t *cnt, uint16_t *mem,
                                              uint16_t *out, uint32_t *wsum, BucketF bucket,
                                              MapF map) {
  const int t = threadIdx.x;
  uint32_t bk[PPT], slot[PPT], kv[PPT];
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int i = t + j * TPC;
    if (i < n) {
      kv[j] = key[i];
      bk[j] = bucket(i, kv[j]);
      slot[j] = atomicAdd(&cnt[bk[j]], 1u);
    }
  }
  __syncthreads();
  block_exclusive_scan<TPC, PPT, false>(cnt, n, wsum);
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int i = t + j * TPC;
    if (i < n) {
      const uint32_t pos = cnt[bk[j]] + slot[j];
      mem[pos] = (uint16_t)i;
      key[pos] = kv[j];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int i = t + j * TPC;
    if (i < n) {
      const uint32_t s0 = cnt[bk[j]], s1 = cnt[bk[j] + 1];
      uint32_t r = 0;
      for (uint32_t m = s0; m < s1; ++m) {
        const uint32_t ko = key[m];
        const int o = mem[m];
        r += (ko < kv[j] || (ko == kv[j] && o < i)) ? 1u : 0u;
      }
      out[s0 + r] = (uint16_t)map(i);
    }
  }
  __syncthreads();
}

// Bitonic sort of P = 2^k item ids in LDS under a strict total order
// `less(a, b)`; padding entries hold 0xFFFF and sort last.
template <int TPC, class LessF>
__device__ __forceinline__ void bitonic_sort_ids(uint16_t *val, int P, LessF less) {
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += TPC) {
        const int p = i ^ j;
        if (p > i) {
          const bool up = (i & k) == 0;
          const uint16_t vi = val[i], vp = val[p];
          // greater(vi, vp): padding is the largest
          const bool gt = (vi == 0xFFFF) ? (vp != 0xFFFF) : (vp != 0xFFFF && less(vp, vi));
          if (gt == up) {
            val[i] = vp;
            val[p] = vi;
          }
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Scalar math of the pair scatter, templated on the kinematics type.
// ---------------------------------------------------------------------------
template <typename T>
struct KMath;

template <>
struct KMath<double> {
  static __device__ __forceinline__ double u(uint32_t a) { return unif64(a); }
  static __device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
  static __device__ __forceinline__ double div(double a, double b) { return a / b; }
  static __device__ __forceinline__ double log_(double x) { return log(x); }
  static __device__ __forceinline__ double exp_(double x) { return exp(x); }
  static __device__ __forceinline__ double expm1_(double x) { return expm1(x); }
  static __device__ __forceinline__ double log1p_(double x) { return log1p(x); }
  static __device__ __forceinline__ double sinh_(double x) { return sinh(x); }
  // sin and cos of 2 pi x
  static __device__ __forceinline__ void sincos2pi(double x, double &s, double &c) {
    sincospi(2.0 * x, &s, &c);
  }
  static __device__ __forceinline__ double cos2pi(double x) { return cospi(2.0 * x); }
  static constexpr int NEWTON_MAX = 60;
  static constexpr double EPS = 2.220446049250313e-16;
  static constexpr double S_ISO = 50.0;
};

template <>
struct KMath<float> {
  static __device__ __forceinline__ float u(uint32_t a) { return unif32(a); }
  // FP32 kinematics: the hardware square root and reciprocal (about 1 ulp)
  static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
  static __device__ __forceinline__ float div(float a, float b) {
    return a * __builtin_amdgcn_rcpf(b);
  }
  static __device__ __forceinline__ float log_(float x) {
    return __builtin_amdgcn_logf(x) * 0.69314718055994531f;
  }
  static __device__ __forceinline__ float exp_(float x) {
    return __builtin_amdgcn_exp2f(x * 1.4426950408889634f);
  }
  static __device__ __forceinline__ float expm1_(float x) { return expm1f(x); }
  static __device__ __forceinline__ float log1p_(float x) { return log1pf(x); }
  static __device__ __forceinline__ float sinh_(float x) { return sinhf(x); }
  // v_sin_f32 / v_cos_f32 take their argument in revolutions
  static __device__ __forceinline__ void sincos2pi(float x, float &s, float &c) {
    s = __builtin_amdgcn_sinf(x);
    c = __builtin_amdgcn_cosf(x);
  }
  static __device__ __forceinline__ float cos2pi(float x) { return __builtin_amdgcn_cosf(x); }
  static constexpr int NEWTON_MAX = 12;
  static constexpr float EPS = 1.1920929e-7f;
  static constexpr float S_ISO = 24.0f;
};

// coth A - 1/A for A < 1/2 by its continued fraction
// x/(3 + x^2/(5 + x^2/(7 + ...))), depth chosen for the type
template <typename T>
__device__ __forceinline__ T langevin_small(T A) {
  const T x2 = A * A;
  constexpr int D = sizeof(T) == 8 ? 12 : 6;
  T d = T(2 * D + 3);
#pragma unroll
  for (int k = D; k >= 1; --k) d = T(2 * k + 1) + x2 / d;
  return A / d;
}

template <typename T>
__device__ __forceinline__ T langevin_deriv(T A) {
  using M = KMath<T>;
  if (A < T(0.5)) {
    const T x2 = A * A;
    return T(1) / T(3) - x2 / T(15) + T(2) * x2 * x2 / T(189) - x2 * x2 * x2 / T(675);
  }
  const T sh = M::sinh_(A);
  return T(1) / (A * A) - T(1) / (sh * sh);
}

// Nanbu's A(s): coth A - 1/A = exp(-s).  For s <= ln 2 the equation is
// solved for 1 - L(A) = -expm1(-s); otherwise for L(A) = exp(-s).  Newton
// inside a bracket.  Returns +inf for s == 0 and 0 when exp(-s) underflows.
template <typename T>
__device__ T n97_A(T s) {
  using M = KMath<T>;
  if (!(s > T(0))) return T(__builtin_inf());
  // large s: A = 3 e^{-s} is below the type's resolution relative to 1 and
  // the sampled angle is isotropic to rounding; avoids subnormal A
  if (s > M::S_ISO) return T(0);
  const bool useM = s <= T(0.69314718055994531);
  T target, lo = T(0), hi, A;
  if (useM) {
    target = -M::expm1_(-s);
    hi = T(1) / target;
    A = hi;
  } else {
    target = M::exp_(-s);
    if (target == T(0)) return T(0);
    hi = T(1) / (T(1) - target);
    A = T(3) * target;
    if (A >= hi) A = T(0.5) * hi;
  }
  for (int it = 0; it < M::NEWTON_MAX; ++it) {
    T g;
    if (useM) {
      const T m = A < T(0.5) ? T(1) - langevin_small(A) : T(1) / A - T(2) / M::expm1_(T(2) * A);
      g = target - m;
    } else {
      const T l = A < T(0.5) ? langevin_small(A) : T(1) + T(2) / M::expm1_(T(2) * A) - T(1) / A;
      g = l - target;
    }
    if (g == T(0)) break;
    if (g < T(0))
      lo = A;
    else
      hi = A;
    if (hi - lo <= T(4) * M::EPS * hi) break;
    T An = A - g / langevin_deriv(A);
    if (!(An > lo && An < hi)) An = T(0.5) * (lo + hi);
    if (fabs(An - A) <= T(0.5) * M::EPS * A) {
      A = An;
      break;
    }
    A = An;
  }
  return A;
}

// ---------------------------------------------------------------------------
// Fast A(s) for the collision step.  Nanbu's equation L(A) = coth A - 1/A =
// exp(-s) has closed-form solutions to rounding at both ends; in between A
// is interpolated (cubic Hermite in t = ln s on a table of A and dA/dt
// computed once per context by n97_A above) and, in FP64, polished by one
// Newton step on the equation itself (the interpolant is good to ~1e-9, so
// one step reaches rounding).
// ---------------------------------------------------------------------------
constexpr int N97_TN = N97_TABLE_SIZE;
constexpr double N97_T0 = -3.25;
constexpr double N97_T1 = 3.0;
constexpr double N97_H = (N97_T1 - N97_T0) / (N97_TN - 1);
// below: 1 - L(A) = 1/A to 1e-20 relative (A > 24); above: L(A) = A/3 to
// 1e-17 relative (A < 7e-9)
constexpr double N97_S_LO = 0.04;
constexpr double N97_S_HI = 20.0;

// coth A - 1/A = sum_n c_n A^(2n-1) with c_n = 2^(2n) B_(2n) / (2n)!
// (Bernoulli numbers B), convergent for |A| < pi; for A < 1/2 twelve terms
// are below FP64 rounding.  Also returns the derivative.
__device__ __forceinline__ void langevin_series(double A, double &L, double &dL) {
  constexpr double c[12] = {
      1.0 / 3.0,       -1.0 / 45.0,      2.0 / 945.0,         -1.0 / 4725.0,
      2.0 / 93555.0,   -1382.0 / 638512875.0, 4.0 / 18243225.0, -3617.0 / 162820783125.0,
      87734.0 / 38979295480125.0, -349222.0 / 1531329465290625.0,
      310732.0 / 13447856940643125.0, -472728182.0 / 201919571963756521875.0};
  const double x2 = A * A;
  double p = c[11], q = 23.0 * c[11];
#pragma unroll
  for (int k = 10; k >= 0; --k) {
    p = fma(p, x2, c[k]);
    q = fma(q, x2, (2.0 * k + 1.0) * c[k]);
  }
  L = A * p;
  dL = q;
}

// one Newton step on Nanbu's equation from A (FP64): the 1 - L form against
// -expm1(-s) for s <= ln 2 (there A > 1.6), else the L form against exp(-s)
__device__ __forceinline__ double n97_newton(double s, double A) {
  double L, M, dL;
  if (A < 0.5) {
    langevin_series(A, L, dL);
    M = 1.0 - L;
  } else {
    const double em1 = expm1(2.0 * A);
    const double r1 = 1.0 / em1, ra = 1.0 / A;
    M = ra - 2.0 * r1;
    L = 1.0 - M;
    dL = ra * ra - 4.0 * (em1 + 1.0) * r1 * r1;  // 1/A^2 - 1/sinh^2 A
  }
  double g;
  if (s <= 0.69314718055994531)
    g = -expm1(-s) - M;  // = L(A) - exp(-s), formed without cancellation
  else
    g = L - exp(-s);
  return A - g / dL;
}

// (tab: double2 in HBM, or float2 holding the same entries rounded to FP32,
// which is what the FP32 form takes of them)
template <typename T, class Tab>
__device__ __forceinline__ T n97_A_fast(T s, const Tab *tab) {
  using M = KMath<T>;
  if (!(s > T(0))) return T(__builtin_inf());
  if (s > M::S_ISO) return T(0);
  if (s >= T(N97_S_HI)) return T(3) * M::exp_(-s);
  if (s <= T(N97_S_LO)) return M::div(T(1), -M::expm1_(-s));
  const T x = (M::log_(s) - T(N97_T0)) * T(1.0 / N97_H);
  int i = (int)x;
  i = i < 0 ? 0 : (i > N97_TN - 2 ? N97_TN - 2 : i);
  const T f = x - T(i);
  const Tab k0 = tab[i], k1 = tab[i + 1];
  const T f2 = f * f, f3 = f2 * f;
  // Hermite basis; the table holds A and h dA/dt at the knots
  const T A = (T(2) * f3 - T(3) * f2 + T(1)) * T(k0.x) + (f3 - T(2) * f2 + f) * T(k0.y) +
              (T(3) * f2 - T(2) * f3) * T(k1.x) + (f3 - f2) * T(k1.y);
  if constexpr (sizeof(T) == 8)
    return n97_newton(s, A);
  else
    return A;
}

// Sampled polar angle: oc = 1 - cos(theta), st = sin(theta).
template <typename T, class Tab>
__device__ __forceinline__ void sample_angle(int method, T s, uint32_t a0, uint32_t a1, T &oc,
                                             T &st, const Tab *n97tab) {
  using M = KMath<T>;
  const T u0 = M::u(a0);
  if (method == 0) {  // TA77: tan(theta/2) ~ N(0, s/2)
    const T z = M::sqrt_(T(-2) * M::log_(u0)) * M::cos2pi(M::u(a1));
    const T delta = M::sqrt_(T(0.5) * s) * z;
    const T d2 = delta * delta;
    if (__builtin_isinf(d2)) {
      oc = T(2);
      st = T(0);
    } else {
      const T q = M::div(T(1), T(1) + d2);
      st = T(2) * delta * q;
      oc = T(2) * d2 * q;
    }
  } else {  // N97
    const T A = n97_A_fast<T>(s, n97tab);
    if (__builtin_isinf(A))
      oc = T(0);
    else if (A == T(0))
      oc = T(2) * u0;
    else
      oc = M::div(-M::log1p_(u0 * M::expm1_(T(-2) * A)), A);
    oc = oc < T(0) ? T(0) : (oc > T(2) ? T(2) : oc);
    st = M::sqrt_(oc * (T(2) - oc));
  }
}

// change of u under rotation by theta about u, azimuth phi (TA77 form)
template <typename T>
__device__ __forceinline__ void rotate_delta(T ux, T uy, T uz, T st, T oc, T sp, T cp, T &dx,
                                             T &dy, T &dz) {
  using M = KMath<T>;
  const T up2 = ux * ux + uy * uy;
  const T up = M::sqrt_(up2);
  const T um = M::sqrt_(up2 + uz * uz);
  if (up > T(0)) {
    const T ax = M::div(ux, up), ay = M::div(uy, up);
    dx = ax * uz * st * cp - ay * um * st * sp - ux * oc;
    dy = ay * uz * st * cp + ax * um * st * sp - uy * oc;
    dz = -up * st * cp - uz * oc;
  } else {
    dx = um * st * cp;
    dy = um * st * sp;
    dz = -uz * oc;
  }
}

}  // namespace mcc
