// mcc_rebin.hip -- incremental re-grouping of a grouped population whose
// particles moved to new cells (the step between two collision steps of a
// particle push).  The result is the stable grouping by the new
// (cell, species) keys: ascending current position inside every new group,
// the same as binning from scratch.  Most particles keep their group, so
// the work is two streaming passes over the particles plus the sorted
// arrival list of each group:
//   - a stayer's rank in its group is its rank among the group's stayers
//     (its old in-group rank less the movers before it in the group) plus
//     the arrivals with a smaller position;
//   - an arrival's rank is the stayers of its new group with a smaller
//     position (the group's old segment lies wholly before or after it)
//     plus its rank in the group's sorted arrival list.
// Arrivals never come from inside a group's old segment, so all stayers of
// a group have the same number of arrivals before them: the arrival lists
// are needed only to place the arrivals themselves.
// Positions are taken in chunks of RB_CH (2048).  A chunk's workgroup finds the
// group of each of its positions from the group starts inside the chunk
// (marked in LDS, then carried forward by a max-scan), and counts the movers
// before a position as the movers of the earlier chunks (one scan over the
// per-chunk counts) plus those before it in the chunk (a scan inside the
// workgroup).  Nothing per particle is kept between the passes but the
// movers themselves.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mcc.h"

namespace mcc {

namespace {

constexpr int RB_TPB = 256, RB_PPT = 8, RB_CH = RB_TPB * RB_PPT, RB_NW = RB_TPB / 64;

// Per group, before the passes: its counters to zero, its offsets checked
// (inconsistent ones are reported), and the chunks whose first position lies
// in its segment claimed (their first group).  With consistent offsets every
// chunk is claimed once; otherwise a chunk may keep an earlier value, which
// the passes clamp into [0, m).
__global__ void k_rebin_prep(int64_t m, int64_t n, const int64_t *off, int64_t nch,
                             uint32_t *leave, uint32_t *arrive, uint32_t *acur, uint32_t *gstart,
                             int32_t *chunk_g0, int32_t *err) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < m;
       g += (int64_t)gridDim.x * blockDim.x) {
    leave[g] = 0u;
    arrive[g] = 0u;
    acur[g] = 0u;
    gstart[g] = 0u;
    const int64_t o0 = off[g], o1 = off[g + 1];
    const bool bad = o1 < o0 || (g == 0 && o0 != 0) || (g == m - 1 && o1 != n);
    if (bad) atomicCAS(err, 0, 1);
    if (!(o0 >= 0 && o1 > o0 && o1 <= n)) continue;
    for (int64_t c = (o0 + RB_CH - 1) / RB_CH; c < nch && c * RB_CH < o1; ++c)
      chunk_g0[c] = (int32_t)g;
  }
}

struct ChunkLds {
  int32_t gs[RB_CH];  // group starting at each position of the chunk (-1: none)
  int32_t wmax[RB_NW];
  uint32_t wsum[RB_NW];
};

__device__ __forceinline__ int32_t wave_incl_max(int32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t y = __shfl_up(x, d);
    if (lane >= d) x = x > y ? x : y;
  }
  return x;
}

__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  return x;
}

// exclusive sum over the workgroup's threads in thread order; total to all
__device__ __forceinline__ uint32_t block_excl_sum(uint32_t x, ChunkLds &L, uint32_t &total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t incl = wave_incl_sum(x);
  if (lane == 63) L.wsum[w] = incl;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < RB_NW; ++k) {
    const uint32_t v = L.wsum[k];
    if (k < w) before += v;
    tot += v;
  }
  total = tot;
  return before + incl - x;
}

// The group of each of the thread's positions c0 + RB_PPT*t + j (j < RB_PPT)
// of chunk [c0, c1), and which of them starts a non-empty group.  g0 is the
// group holding c0.  Groups stay in [0, m) whatever the offsets hold.
__device__ __forceinline__ void chunk_groups(int64_t c0, int64_t c1, int64_t m, int64_t n,
                                             const int64_t *off, int32_t g0, ChunkLds &L,
                                             int32_t (&g)[RB_PPT], uint32_t &starts) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
  for (int j = 0; j < RB_PPT; ++j) L.gs[RB_PPT * t + j] = -1;
  __syncthreads();
  // a group that starts inside the chunk marks its first position; the
  // batches go on while the last group of a batch still starts before c1
  for (int64_t gb = (int64_t)g0 + 1;; gb += RB_TPB) {
    const int64_t gg = gb + t;
    int64_t o = n;
    if (gg < m) {
      o = off[gg];
      if (o >= c0 && o < c1 && off[gg + 1] > o) L.gs[o - c0] = (int32_t)gg;
    }
    if (!__syncthreads_or(t == RB_TPB - 1 && gg < m && o < c1)) break;
  }
  int32_t v[RB_PPT];
  int32_t mx = -1;
  starts = 0u;
#pragma unroll
  for (int j = 0; j < RB_PPT; ++j) {
    v[j] = L.gs[RB_PPT * t + j];
    if (v[j] >= 0) starts |= 1u << j;
    mx = v[j] > mx ? v[j] : mx;
  }
  if (t == 0) {
    // the chunk's first position belongs to g0; it starts g0 only if g0's
    // segment begins there
    v[0] = g0;
    starts = (starts & ~1u) | (off[g0] == c0 ? 1u : 0u);
    mx = mx > g0 ? mx : g0;
  }
  // carry: the largest group starting at an earlier position (groups start
  // in ascending order)
  const int32_t incl = wave_incl_max(mx);
  if (lane == 63) L.wmax[w] = incl;
  __syncthreads();
  int32_t carry = __shfl_up(incl, 1);
  if (lane == 0) carry = -1;
#pragma unroll
  for (int k = 0; k < RB_NW; ++k)
    if (k < w) carry = L.wmax[k] > carry ? L.wmax[k] : carry;
#pragma unroll
  for (int j = 0; j < RB_PPT; ++j) {
    carry = v[j] > carry ? v[j] : carry;
    g[j] = carry < 0 ? 0 : (carry >= m ? (int32_t)(m - 1) : carry);
  }
}

// the new group of the particle at p (group g); a cell id out of range is
// reported and the particle kept where it is
__device__ __forceinline__ int32_t new_group(int32_t g, int32_t c, int32_t S, int32_t n_cells,
                                             int32_t *err) {
  const int32_t s = g % S;
  if (c < 0 || c >= n_cells) {
    atomicCAS(err, 0, 3);
    return g;
  }
  return c * S + s;
}

__device__ __forceinline__ void load_cells(const int32_t *cells_new, int64_t p0, int64_t c1,
                                           int32_t (&c)[RB_PPT]) {
  // (vector loads when the array is 16-byte aligned; p0 is a multiple of RB_PPT)
  if (p0 + RB_PPT <= c1 && ((uintptr_t)cells_new & 15) == 0) {
#pragma unroll
    for (int q = 0; q < RB_PPT / 4; ++q) {
      const int4 a = *reinterpret_cast<const int4 *>(cells_new + p0 + 4 * q);
      c[4 * q] = a.x;
      c[4 * q + 1] = a.y;
      c[4 * q + 2] = a.z;
      c[4 * q + 3] = a.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < RB_PPT; ++j) c[j] = p0 + j < c1 ? cells_new[p0 + j] : 0;
  }
}

// Pass 1, one workgroup per chunk: the movers of the chunk in position order
// into its slice of the mover queue (position, new group), the per-group
// counts of leavers and arrivals, the chunk's mover count, and for each
// group that starts in the chunk the chunk's movers before its start.
__global__ void __launch_bounds__(RB_TPB)
    k_rebin_mark(int64_t n, int64_t m, int32_t S, int32_t n_cells, const int64_t *off,
                 const int32_t *cells_new, const int32_t *chunk_g0, int32_t *mq_p,
                 int32_t *mq_g, uint32_t *chunk_cnt, uint32_t *gstart, uint32_t *leave,
                 uint32_t *arrive, int32_t *err) {
  __shared__ ChunkLds L;
  const int64_t c = blockIdx.x, c0 = c * RB_CH, c1 = c0 + RB_CH < n ? c0 + RB_CH : n;
  const int64_t p0 = c0 + (int64_t)RB_PPT * threadIdx.x;
  int32_t cn[RB_PPT], g2[RB_PPT];
  load_cells(cells_new, p0, c1, cn);
  int32_t g0 = chunk_g0[c];
  g0 = g0 < 0 ? 0 : (g0 >= m ? (int32_t)(m - 1) : g0);
  int32_t g[RB_PPT];
  uint32_t starts;
  chunk_groups(c0, c1, m, n, off, g0, L, g, starts);
  uint32_t mv = 0u;
#pragma unroll
  for (int j = 0; j < RB_PPT; ++j) {
    if (p0 + j >= c1) continue;
    g2[j] = new_group(g[j], cn[j], S, n_cells, err);
    if (g2[j] != g[j]) mv |= 1u << j;
  }
  uint32_t total;
  const uint32_t base = block_excl_sum((uint32_t)__popc(mv), L, total);
  uint32_t r = base;
#pragma unroll
  for (int j = 0; j < RB_PPT; ++j) {
    if (starts & (1u << j)) gstart[g[j]] = r;
    if (mv & (1u << j)) {
      atomicAdd(&leave[g[j]], 1u);
      atomicAdd(&arrive[g2[j]], 1u);
      mq_p[c0 + r] = (int32_t)(p0 + j);
      mq_g[c0 + r] = g2[j];
      ++r;
    }
  }
  if (threadIdx.x == 0) chunk_cnt[c] = total;
}

// The three exclusive scans after the first pass, in one set of launches:
// array 0 the new group sizes (size - leavers + arrivals, computed on the
// fly) into off_new, array 1 the arrival counts into aoff, array 2 the
// chunks' mover counts into chunk_pre; each output gets its total at the
// end.  Tiles of RB_CH entries; the tiles of the three arrays follow one
// another in the grid.
struct Scan3 {
  const int64_t *off;
  const uint32_t *leave, *arrive, *chunk_cnt;
  int64_t m, nch, nt0, nt1, nt2;
  int64_t *off_new, *aoff, *chunk_pre;
};

__device__ __forceinline__ uint32_t scan3_in(const Scan3 &S3, int a, int64_t i) {
  if (a == 0)
    return (uint32_t)(S3.off[i + 1] - S3.off[i]) - S3.leave[i] + S3.arrive[i];
  return a == 1 ? S3.arrive[i] : S3.chunk_cnt[i];
}

// which array the tile b belongs to, its first entry and the array's length
__device__ __forceinline__ int scan3_tile(const Scan3 &S3, int64_t b, int64_t &t0, int64_t &len) {
  if (b < S3.nt0) {
    t0 = b;
    len = S3.m;
    return 0;
  }
  if (b < S3.nt0 + S3.nt1) {
    t0 = b - S3.nt0;
    len = S3.m;
    return 1;
  }
  t0 = b - S3.nt0 - S3.nt1;
  len = S3.nch;
  return 2;
}

__global__ void __launch_bounds__(RB_TPB) k_rebin_scan_tiles(Scan3 S3, int64_t *tiles) {
  __shared__ ChunkLds L;
  int64_t t0, len;
  const int a = scan3_tile(S3, blockIdx.x, t0, len);
  const int64_t base = t0 * RB_CH + (int64_t)RB_PPT * threadIdx.x;
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < RB_PPT; ++j)
    if (base + j < len) sum += scan3_in(S3, a, base + j);
  uint32_t total;
  block_excl_sum(sum, L, total);
  if (threadIdx.x == 0) tiles[blockIdx.x] = total;
}

// one workgroup: each array's tile sums into exclusive tile offsets
__global__ void __launch_bounds__(RB_TPB) k_rebin_scan_sums(Scan3 S3, int64_t *tiles) {
  __shared__ int64_t wtot[RB_NW];
  const int t = threadIdx.x;
  const int64_t seg0[3] = {0, S3.nt0, S3.nt0 + S3.nt1};
  const int64_t segn[3] = {S3.nt0, S3.nt1, S3.nt2};
  for (int a = 0; a < 3; ++a) {
    int64_t *ts = tiles + seg0[a];
    const int64_t nt = segn[a];
    const int64_t per = (nt + RB_TPB - 1) / RB_TPB;
    const int64_t lo = t * per, hi = lo + per < nt ? lo + per : nt;
    int64_t acc = 0;
    for (int64_t i = lo; i < hi; ++i) acc += ts[i];
    // exclusive scan of the threads' sums: in each wave by shuffles, then
    // across the waves
    int64_t incl = acc;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int64_t y = __shfl_up(incl, d);
      if ((t & 63) >= d) incl += y;
    }
    if ((t & 63) == 63) wtot[t >> 6] = incl;
    __syncthreads();
    int64_t run = incl - acc;
#pragma unroll
    for (int k = 0; k < RB_NW; ++k)
      if (k < (t >> 6)) run += wtot[k];
    for (int64_t i = lo; i < hi; ++i) {
      const int64_t x = ts[i];
      ts[i] = run;
      run += x;
    }
    __syncthreads();  // (wtot is reused by the next array)
  }
}

__global__ void __launch_bounds__(RB_TPB) k_rebin_scan_apply(Scan3 S3, const int64_t *tiles) {
  __shared__ ChunkLds L;
  int64_t t0, len;
  const int a = scan3_tile(S3, blockIdx.x, t0, len);
  int64_t *out = a == 0 ? S3.off_new : (a == 1 ? S3.aoff : S3.chunk_pre);
  const int64_t base = t0 * RB_CH + (int64_t)RB_PPT * threadIdx.x;
  uint32_t v[RB_PPT];
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < RB_PPT; ++j) {
    v[j] = base + j < len ? scan3_in(S3, a, base + j) : 0u;
    sum += v[j];
  }
  uint32_t total;
  int64_t run = tiles[blockIdx.x] + (int64_t)block_excl_sum(sum, L, total);
#pragma unroll
  for (int j = 0; j < RB_PPT; ++j) {
    if (base + j < len) out[base + j] = run;
    run += v[j];
  }
  if (base <= len - 1 && len - 1 < base + RB_PPT) out[len] = run;  // the total
}

// the movers of each chunk into their new group's arrival list (unordered:
// atomic slots)
__global__ void k_rebin_lists(const uint32_t *chunk_cnt, const int32_t *mq_p,
                              const int32_t *mq_g, const int64_t *aoff, uint32_t *acur,
                              int32_t *alist) {
  const int64_t c0 = (int64_t)blockIdx.x * RB_CH;
  const uint32_t k = chunk_cnt[blockIdx.x];
  for (uint32_t i = threadIdx.x; i < k && i < (uint32_t)RB_CH; i += blockDim.x) {
    const int32_t g2 = mq_g[c0 + i];
    const uint32_t slot = atomicAdd(&acur[g2], 1u);
    const int64_t at = aoff[g2] + slot;
    if (at < aoff[g2 + 1]) alist[at] = mq_p[c0 + i];
  }
}

// Per group, once the scans are done: its arrivals go to their new
// positions and the group's stayer base is recorded.  With the group's
// arrivals in ascending position, the one of rank i goes to
// off_new + i + (its position before the old segment ? 0 : the stayers).
// Arrivals never come from inside the old segment, so every stayer has the
// same count `below` of arrivals before it, and a stayer at p goes to
//   sbase + p - (movers before p),
//   sbase = off_new - o0 + (movers before o0) + below.
// A group whose offsets are inconsistent (reported by k_rebin_prep) places
// nobody: sbase = kNoGroup.
constexpr int64_t kNoGroup = INT64_MIN;

struct GroupView {
  int64_t o0, o1, nbase, stay;
  bool ok;
};

__device__ __forceinline__ GroupView group_view(int64_t g, int64_t n, const int64_t *off,
                                                const int64_t *off_new, const uint32_t *leave) {
  GroupView v;
  const int64_t o0 = off[g], o1 = off[g + 1];
  v.ok = o0 >= 0 && o1 >= o0 && o1 <= n;
  v.o0 = v.ok ? o0 : 0;
  v.o1 = v.ok ? o1 : 0;
  v.nbase = off_new[g];
  v.stay = v.ok ? (o1 - o0) - (int64_t)leave[g] : 0;
  return v;
}

__device__ __forceinline__ int64_t group_sbase(const GroupView &v, int64_t g,
                                               const int64_t *chunk_pre, const uint32_t *gstart,
                                               int64_t below) {
  if (!v.ok) return kNoGroup;
  if (v.o1 <= v.o0) return 0;  // (no stayers)
  return v.nbase - v.o0 + chunk_pre[v.o0 / RB_CH] + (int64_t)gstart[g] + below;
}

__device__ __forceinline__ void place_arrival(const GroupView &v, int64_t i, int32_t p, int64_t n,
                                              int32_t *perm, int32_t *err) {
  if (!v.ok) return;
  const int64_t pos = v.nbase + i + (p < v.o0 ? 0 : v.stay);
  if (pos < 0 || pos >= n)
    atomicCAS(err, 0, 1);
  else
    perm[pos] = p;
}

__device__ __forceinline__ void cx(int32_t &a, int32_t &b) {
  const int32_t lo = a < b ? a : b, hi = a < b ? b : a;
  a = lo;
  b = hi;
}

// The ascending bitonic network on N values (N a power of two): stage s
// compares each element of a block of s with its mirror in the block, then
// half-cleaners at s/4, s/8, ..., 1 (element i with i + j).  Every
// compare-exchange leaves the smaller value at the lower index, so padding
// taken as +infinity stays at the top.  Fully unrolled: the indices are
// constants and v stays in registers.
template <int N>
__device__ __forceinline__ void sort_net(int32_t (&v)[N]) {
#pragma unroll
  for (int s = 2; s <= N; s <<= 1) {
#pragma unroll
    for (int j = s >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int l = j == (s >> 1) ? (i ^ (s - 1)) : (i ^ j);
        if (l > i) cx(v[i], v[l]);
      }
    }
  }
}

// a list of at most N arrivals: sorted in registers, placed; returns how
// many lie before the old segment
template <int N>
__device__ __forceinline__ int64_t place_list_regs(const int32_t *a, int64_t k,
                                                   const GroupView &gv, int64_t n,
                                                   int32_t *perm, int32_t *err) {
  int32_t v[N];
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = i < k ? a[i] : INT32_MAX;
  if (N > 1) sort_net<N>(v);
  int64_t below = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    if (i < k) {
      below += v[i] < gv.o0 ? 1 : 0;
      place_arrival(gv, i, v[i], n, perm, err);
    }
  }
  return below;
}

// Groups with at most 32 arrivals (nearly all of them when a few per cent of
// the particles move): one thread each.
__global__ void k_rebin_place_arrivals(int64_t m, int64_t n, const int64_t *off,
                                       const int64_t *off_new, const uint32_t *leave,
                                       const int64_t *aoff, const int32_t *alist,
                                       const int64_t *chunk_pre, const uint32_t *gstart,
                                       int64_t *sbase, int32_t *perm, int32_t *err) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < m;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a0 = aoff[g], k = aoff[g + 1] - a0;
    if (k > 32) continue;  // (k_rebin_place_arrivals_long)
    const GroupView gv = group_view(g, n, off, off_new, leave);
    const int32_t *a = alist + a0;
    int64_t below = 0;
    if (k == 0)
      below = 0;
    else if (k == 1)
      below = place_list_regs<1>(a, k, gv, n, perm, err);
    else if (k == 2)
      below = place_list_regs<2>(a, k, gv, n, perm, err);
    else if (k <= 8)
      below = place_list_regs<8>(a, k, gv, n, perm, err);
    else if (k <= 16)
      below = place_list_regs<16>(a, k, gv, n, perm, err);
    else
      below = place_list_regs<32>(a, k, gv, n, perm, err);
    sbase[g] = group_sbase(gv, g, chunk_pre, gstart, below);
  }
}

// Groups with more than 32 arrivals: a wave per block of 64 groups finds
// them (one load of the block's offsets and a ballot) and takes them one
// after the other: the same network over the wave's lanes with shuffles up
// to 64 arrivals, in LDS up to LONG_LDS, in place in the list beyond; then
// every arrival to its position.
constexpr int LONG_LDS = 4096;
__global__ void __launch_bounds__(64)
    k_rebin_place_arrivals_long(int64_t m, int64_t n, const int64_t *off, const int64_t *off_new,
                                const uint32_t *leave, const int64_t *aoff, int32_t *alist,
                                const int64_t *chunk_pre, const uint32_t *gstart,
                                int64_t *sbase, int32_t *perm, int32_t *err) {
  __shared__ int32_t buf[LONG_LDS];
  const int lane = threadIdx.x;
  for (int64_t gb = (int64_t)blockIdx.x * 64; gb < m; gb += (int64_t)gridDim.x * 64) {
    const int64_t gl = gb + lane;
    const int64_t a0l = gl < m ? aoff[gl] : 0, kl = gl < m ? aoff[gl + 1] - a0l : 0;
    uint64_t todo = __ballot(kl > 32);
    while (todo) {
      const int b = __ffsll((unsigned long long)todo) - 1;
      todo &= todo - 1;
      const int64_t g = gb + b;
      const int64_t a0 = __shfl(a0l, b), k = __shfl(kl, b);
      const GroupView gv = group_view(g, n, off, off_new, leave);
      int32_t *a = alist + a0;
      uint32_t below = 0;
      if (k <= 64) {
        int32_t v = lane < k ? a[lane] : INT32_MAX;
#pragma unroll
        for (int s = 2; s <= 64; s <<= 1) {
#pragma unroll
          for (int j = s >> 1; j > 0; j >>= 1) {
            const int l = j == (s >> 1) ? (lane ^ (s - 1)) : (lane ^ j);
            const int32_t u = __shfl(v, l);
            v = (lane < l) == (u > v) ? v : u;  // lower index keeps the smaller
          }
        }
        if (lane < k) place_arrival(gv, lane, v, n, perm, err);
        below = (uint32_t)__popcll(__ballot(lane < k && v < gv.o0));
      } else {
        const bool in_lds = k <= LONG_LDS;
        int32_t *d = in_lds ? buf : a;
        if (in_lds) {
          for (int64_t i = lane; i < k; i += 64) buf[i] = a[i];
          __syncthreads();
        }
        int64_t P = 1;
        while (P < k) P <<= 1;
        for (int64_t sz = 2; sz <= P; sz <<= 1) {
          for (int64_t j = sz >> 1; j > 0; j >>= 1) {
            for (int64_t x = lane; x < (P >> 1); x += 64) {
              const int64_t blk = x / j, r = x - blk * j;
              int64_t i, l;
              if (j == (sz >> 1)) {  // mirror within the block of sz
                i = blk * sz + r;
                l = blk * sz + sz - 1 - r;
              } else {  // half-cleaner of stride j
                i = blk * 2 * j + r;
                l = i + j;
              }
              if (l < k) {
                const int32_t u = d[i], w = d[l];
                if (w < u) {
                  d[i] = w;
                  d[l] = u;
                }
              }
            }
            __syncthreads();
          }
        }
        for (int64_t i0 = 0; i0 < k; i0 += 64) {
          const int64_t i = i0 + lane;
          const int32_t p = i < k ? d[i] : INT32_MAX;
          if (i < k) place_arrival(gv, i, p, n, perm, err);
          below += (uint32_t)__popcll(__ballot(i < k && p < gv.o0));
        }
        __syncthreads();  // (before the next list reuses buf)
      }
      if (lane == 0) sbase[g] = group_sbase(gv, g, chunk_pre, gstart, below);
    }
  }
}

// Pass 2, one workgroup per chunk: every stayer to its new position.
__global__ void __launch_bounds__(RB_TPB)
    k_rebin_place(int64_t n, int64_t m, int32_t S, int32_t n_cells, const int64_t *off,
                  const int32_t *cells_new, const int32_t *chunk_g0, const int64_t *chunk_pre,
                  const int64_t *sbase, int32_t *perm, int32_t *err) {
  __shared__ ChunkLds L;
  const int64_t c = blockIdx.x, c0 = c * RB_CH, c1 = c0 + RB_CH < n ? c0 + RB_CH : n;
  const int64_t p0 = c0 + (int64_t)RB_PPT * threadIdx.x;
  int32_t cn[RB_PPT];
  load_cells(cells_new, p0, c1, cn);
  int32_t g0 = chunk_g0[c];
  g0 = g0 < 0 ? 0 : (g0 >= m ? (int32_t)(m - 1) : g0);
  int32_t g[RB_PPT];
  uint32_t starts;
  chunk_groups(c0, c1, m, n, off, g0, L, g, starts);
  uint32_t mv = 0u;
#pragma unroll
  for (int j = 0; j < RB_PPT; ++j) {
    if (p0 + j >= c1) continue;
    // (a cell id out of range was reported by the first pass: the particle stays)
    const int32_t g2 = (cn[j] < 0 || cn[j] >= n_cells) ? g[j] : cn[j] * S + g[j] % S;
    if (g2 != g[j]) mv |= 1u << j;
  }
  uint32_t total;
  int64_t before = chunk_pre[c] + block_excl_sum((uint32_t)__popc(mv), L, total);
#pragma unroll
  for (int j = 0; j < RB_PPT; ++j) {
    const int64_t p = p0 + j;
    if (p >= c1) continue;
    if (mv & (1u << j)) {
      ++before;
      continue;
    }
    const int64_t sb = sbase[g[j]];
    if (sb == kNoGroup) continue;
    const int64_t pos = sb + p - before;
    if (pos < 0 || pos >= n)
      atomicCAS(err, 0, 1);
    else
      perm[pos] = (int32_t)p;
  }
}

inline int grid_of(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return (int)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

// scratch of launch_rebin: the mover queue (position, new group) and the
// arrival lists, int32[n] each; per chunk of RB_CH positions its first
// group, mover count and the scan of the counts; per group the leaver,
// arrival, slot and start counters, the arrival offsets and the stayer base.
// `tiles` holds rebin_tiles_needed(n, m) entries.
size_t rebin_scratch_bytes(int64_t n, int64_t m) {
  const size_t nn = (size_t)(n > 0 ? n : 1), mm = (size_t)(m > 0 ? m : 1);
  const size_t nch = (nn + RB_CH - 1) / RB_CH;
  return 3 * align256(4 * nn) + 2 * align256(4 * nch) + align256(8 * (nch + 1)) +
         4 * align256(4 * mm) + align256(8 * (mm + 1)) + align256(8 * mm);
}

int64_t rebin_tiles_needed(int64_t n, int64_t m) {
  const int64_t nch = (n + RB_CH - 1) / RB_CH;
  return 2 * ((m + RB_CH - 1) / RB_CH) + (nch + RB_CH - 1) / RB_CH + 1;
}

hipError_t launch_rebin(int64_t n, int64_t m, int32_t S, int32_t n_cells, const int64_t *off,
                        const int32_t *cells_new, int64_t *off_new, int32_t *perm,
                        void *scratch, int64_t *tiles, int32_t *err, hipStream_t s) {
  const size_t nn = (size_t)(n > 0 ? n : 1), mm = (size_t)(m > 0 ? m : 1);
  const int64_t nch = (n + RB_CH - 1) / RB_CH;
  const size_t nchs = (nn + RB_CH - 1) / RB_CH;
  char *p = static_cast<char *>(scratch);
  auto take = [&](size_t bytes) {
    char *q = p;
    p += align256(bytes);
    return q;
  };
  int32_t *mq_p = reinterpret_cast<int32_t *>(take(4 * nn));
  int32_t *mq_g = reinterpret_cast<int32_t *>(take(4 * nn));
  int32_t *alist = reinterpret_cast<int32_t *>(take(4 * nn));
  int32_t *chunk_g0 = reinterpret_cast<int32_t *>(take(4 * nchs));
  uint32_t *chunk_cnt = reinterpret_cast<uint32_t *>(take(4 * nchs));
  int64_t *chunk_pre = reinterpret_cast<int64_t *>(take(8 * (nchs + 1)));
  uint32_t *leave = reinterpret_cast<uint32_t *>(take(4 * mm));
  uint32_t *arrive = reinterpret_cast<uint32_t *>(take(4 * mm));
  uint32_t *acur = reinterpret_cast<uint32_t *>(take(4 * mm));
  uint32_t *gstart = reinterpret_cast<uint32_t *>(take(4 * mm));
  int64_t *aoff = reinterpret_cast<int64_t *>(take(8 * (mm + 1)));
  int64_t *sbase = reinterpret_cast<int64_t *>(take(8 * mm));

  const int64_t nt0 = (m + RB_CH - 1) / RB_CH, nt2 = (nch + RB_CH - 1) / RB_CH;
  const Scan3 S3{off, leave, arrive, chunk_cnt, m, nch, nt0, n > 0 ? nt0 : 0, n > 0 ? nt2 : 0,
                 off_new, aoff, chunk_pre};
  hipLaunchKernelGGL(k_rebin_prep, dim3(grid_of(m)), dim3(256), 0, s, m, n, off, nch, leave,
                     arrive, acur, gstart, chunk_g0, err);
  if (n > 0)
    hipLaunchKernelGGL(k_rebin_mark, dim3((unsigned)nch), dim3(RB_TPB), 0, s, n, m, S, n_cells,
                       off, cells_new, chunk_g0, mq_p, mq_g, chunk_cnt, gstart, leave, arrive,
                       err);
  const int64_t ntt = S3.nt0 + S3.nt1 + S3.nt2;
  hipLaunchKernelGGL(k_rebin_scan_tiles, dim3((unsigned)ntt), dim3(RB_TPB), 0, s, S3, tiles);
  hipLaunchKernelGGL(k_rebin_scan_sums, dim3(1), dim3(RB_TPB), 0, s, S3, tiles);
  hipLaunchKernelGGL(k_rebin_scan_apply, dim3((unsigned)ntt), dim3(RB_TPB), 0, s, S3, tiles);
  if (n > 0) {
    hipLaunchKernelGGL(k_rebin_lists, dim3((unsigned)nch), dim3(256), 0, s, chunk_cnt, mq_p, mq_g,
                       aoff, acur, alist);
    hipLaunchKernelGGL(k_rebin_place_arrivals, dim3(grid_of(m)), dim3(256), 0, s, m, n, off,
                       off_new, leave, aoff, alist, chunk_pre, gstart, sbase, perm, err);
    const int64_t wb = (m + 63) / 64;
    hipLaunchKernelGGL(k_rebin_place_arrivals_long, dim3((unsigned)(wb < 8192 ? wb : 8192)),
                       dim3(64), 0, s, m, n, off, off_new, leave, aoff, alist, chunk_pre, gstart,
                       sbase, perm, err);
    hipLaunchKernelGGL(k_rebin_place, dim3((unsigned)nch), dim3(RB_TPB), 0, s, n, m, S, n_cells,
                       off, cells_new, chunk_g0, chunk_pre, sbase, perm, err);
  }
  return hipGetLastError();
}

}  // namespace mcc
