// mcc_rebin.hip -- incremental re-grouping of a grouped population whose
// particles moved to new cells (the step between two collision steps of a
// particle push).  The result is the stable grouping by the new
// (cell, species) keys: ascending current position inside every new group,
// the same as binning from scratch.  Most particles keep their group, so
// the work is a few streaming passes over the particles plus the sorted
// arrival list of each group:
//   - a stayer's rank in its group is its rank among the group's stayers
//     (its old in-group rank less the movers before it: a prefix count of
//     the mover flags) plus the arrivals with a smaller position;
//   - an arrival's rank is the stayers of its new group with a smaller
//     position (the group's old segment lies wholly before or after it)
//     plus its rank in the group's sorted arrival list.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mcc.h"

namespace mcc {

namespace {

// the group whose segment holds grouped position p (offsets[g] <= p <
// offsets[g + 1]); with empty groups, the last g with offsets[g] <= p
__device__ __forceinline__ int64_t group_of(const int64_t *off, int64_t m, int64_t p) {
  int64_t lo = 0, hi = m;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (off[mid] <= p)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// number of entries of the sorted list a[0, k) below x
__device__ __forceinline__ int64_t count_below(const int32_t *a, int64_t k, int32_t x) {
  int64_t lo = 0, hi = k;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__global__ void k_rebin_check(const int64_t *off, int64_t m, int64_t n, int32_t *err) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < m;
       g += (int64_t)gridDim.x * blockDim.x) {
    const bool bad = off[g + 1] < off[g] || (g == 0 && off[0] != 0) ||
                     (g == m - 1 && off[m] != n);
    if (bad) atomicCAS(err, 0, 1);
  }
}

// old and new group of every position, the mover flags, and the per-group
// counts of leavers and arrivals.  A cell id out of range is reported and
// the particle kept where it is.  A block takes a chunk of MARK_CHUNK
// positions: one search in HBM finds the chunk's first group, the next
// MARK_WIN offsets go to LDS, and each position's group is searched there
// (in HBM only when the chunk runs past the window, as across a long run of
// empty groups).
constexpr int MARK_TPB = 256, MARK_CHUNK = 2048, MARK_WIN = 2048;
__global__ void __launch_bounds__(MARK_TPB)
    k_rebin_mark(int64_t n, int64_t m, int32_t S, int32_t n_cells, const int64_t *off,
                 const int32_t *cells_new, int32_t *gold, int32_t *gnew, uint32_t *flag,
                 uint32_t *leave, uint32_t *arrive, int32_t *err) {
  __shared__ int64_t win[MARK_WIN + 1];
  __shared__ int64_t s_g0;
  for (int64_t c0 = (int64_t)blockIdx.x * MARK_CHUNK; c0 < n;
       c0 += (int64_t)gridDim.x * MARK_CHUNK) {
    if (threadIdx.x == 0) s_g0 = group_of(off, m, c0);
    __syncthreads();
    const int64_t g0 = s_g0;
    const int nw = (int)(m + 1 - g0 < MARK_WIN + 1 ? m + 1 - g0 : MARK_WIN + 1);
    for (int i = threadIdx.x; i < nw; i += MARK_TPB) win[i] = off[g0 + i];
    __syncthreads();
    const int64_t c1 = c0 + MARK_CHUNK < n ? c0 + MARK_CHUNK : n;
    for (int64_t p = c0 + threadIdx.x; p < c1; p += MARK_TPB) {
      int64_t g;
      if (win[nw - 1] <= p) {
        g = group_of(off, m, p);  // past the window (win[nw - 1] = n when it reaches the end)
      } else {
        int lo = 0, hi = nw - 1;  // win[lo] <= p < win[hi]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (win[mid] <= p)
            lo = mid;
          else
            hi = mid;
        }
        g = g0 + lo;
      }
      const int32_t s = (int32_t)(g % S);
      int32_t c = cells_new[p];
      if (c < 0 || c >= n_cells) {
        atomicCAS(err, 0, 3);
        c = (int32_t)(g / S);
      }
      const int64_t g2 = (int64_t)c * S + s;
      gold[p] = (int32_t)g;
      gnew[p] = (int32_t)g2;
      const bool mv = g2 != g;
      flag[p] = mv ? 1u : 0u;
      if (mv) {
        atomicAdd(&leave[g], 1u);
        atomicAdd(&arrive[g2], 1u);
      }
    }
    __syncthreads();
  }
}

__global__ void k_rebin_counts(int64_t m, const int64_t *off, const uint32_t *leave,
                               const uint32_t *arrive, uint32_t *cnt) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < m;
       g += (int64_t)gridDim.x * blockDim.x)
    cnt[g] = (uint32_t)(off[g + 1] - off[g]) - leave[g] + arrive[g];
}

// movers into their new group's arrival list (unordered: atomic slots)
__global__ void k_rebin_lists(int64_t n, const int32_t *gnew, const uint32_t *flag,
                              const int64_t *aoff, uint32_t *acur, int32_t *alist) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x) {
    if (!flag[p]) continue;
    const int32_t g2 = gnew[p];
    const uint32_t slot = atomicAdd(&acur[g2], 1u);
    const int64_t at = aoff[g2] + slot;
    if (at < aoff[g2 + 1]) alist[at] = (int32_t)p;
  }
}

// each group's arrivals into ascending position: up to 8 in registers
// (Batcher's odd-even merge network, 19 compare-exchanges), longer lists by a
// wave each (k_rebin_sort_long)
__device__ __forceinline__ void cx(int32_t &a, int32_t &b) {
  const int32_t lo = a < b ? a : b, hi = a < b ? b : a;
  a = lo;
  b = hi;
}
// Lists of 2 to 8 entries (nearly all of them when a few per cent of the
// particles move): one thread each.
__global__ void k_rebin_sort(int64_t m, const int64_t *aoff, int32_t *alist) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < m;
       g += (int64_t)gridDim.x * blockDim.x) {
    int32_t *a = alist + aoff[g];
    const int64_t k = aoff[g + 1] - aoff[g];
    if (k < 2 || k > 8) continue;
    if (k == 2) {
      const int32_t x = a[0], y = a[1];
      if (y < x) {
        a[0] = y;
        a[1] = x;
      }
      continue;
    }
    {
      int32_t v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = i < k ? a[i] : INT32_MAX;
      cx(v[0], v[1]); cx(v[2], v[3]); cx(v[4], v[5]); cx(v[6], v[7]);
      cx(v[0], v[2]); cx(v[1], v[3]); cx(v[4], v[6]); cx(v[5], v[7]);
      cx(v[1], v[2]); cx(v[5], v[6]);
      cx(v[0], v[4]); cx(v[1], v[5]); cx(v[2], v[6]); cx(v[3], v[7]);
      cx(v[2], v[4]); cx(v[3], v[5]);
      cx(v[1], v[2]); cx(v[3], v[4]); cx(v[5], v[6]);
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (i < k) a[i] = v[i];
    }
  }
}
// Lists longer than 8: one wave per list, sorted by the ascending bitonic
// network on the list padded to a power of two P (stage s: each element of a
// block of s against its mirror in the block, then half-cleaners at s/4,
// s/8, ..., 1; every compare-exchange leaves the smaller value at the lower
// index, so padding entries, taken as +infinity, never move and pairs that
// reach past the list are skipped).  Lists up to LONG_LDS entries are sorted
// in LDS, longer ones in place.  An insertion sort by one thread, as before,
// took O(k^2) dependent loads for the few lists of some tens of arrivals that
// a push leaves in the largest cells, and held the whole kernel on them.
constexpr int LONG_TPB = 64, LONG_LDS = 4096;
__global__ void __launch_bounds__(LONG_TPB)
    k_rebin_sort_long(int64_t m, const int64_t *aoff, int32_t *alist) {
  __shared__ int32_t buf[LONG_LDS];
  const int lane = threadIdx.x;
  for (int64_t g = blockIdx.x; g < m; g += gridDim.x) {
    const int64_t k = aoff[g + 1] - aoff[g];  // (the same in every lane)
    if (k <= 8) continue;
    int32_t *a = alist + aoff[g];
    const bool in_lds = k <= LONG_LDS;
    int32_t *d = in_lds ? buf : a;
    if (in_lds) {
      for (int64_t i = lane; i < k; i += LONG_TPB) buf[i] = a[i];
      __syncthreads();
    }
    int64_t P = 1;
    while (P < k) P <<= 1;
    for (int64_t sz = 2; sz <= P; sz <<= 1) {
      for (int64_t j = sz >> 1; j > 0; j >>= 1) {
        for (int64_t x = lane; x < (P >> 1); x += LONG_TPB) {
          int64_t i, l;
          if (j == (sz >> 1)) {  // mirror within the block of sz
            const int64_t blk = x / j, r = x - blk * j;
            i = blk * sz + r;
            l = blk * sz + sz - 1 - r;
          } else {  // half-cleaner of stride j
            const int64_t blk = x / j, r = x - blk * j;
            i = blk * 2 * j + r;
            l = i + j;
          }
          if (l < k) {
            const int32_t u = d[i], v = d[l];
            if (v < u) {
              d[i] = v;
              d[l] = u;
            }
          }
        }
        __syncthreads();
      }
    }
    if (in_lds) {
      for (int64_t i = lane; i < k; i += LONG_TPB) a[i] = buf[i];
      __syncthreads();  // (before the next list reuses buf)
    }
  }
}

// Per group, once the scans are done, everything a particle of it needs:
//   sbase  new position of a stayer at p is sbase + p - mpre[p] + (arrivals
//          below p): off_new - off + (movers before the old segment)
//   nbase  new offset; o0 old segment start; stay its stayers (for arrivals)
//   a0, k  the group's sorted arrival list
struct GroupRec {
  int64_t sbase, nbase, o0, a0;
  int32_t stay, k, ok, pad;
};
static_assert(sizeof(GroupRec) == 48, "the API allocates 48 bytes per group");
__global__ void k_rebin_groups(int64_t m, int64_t n, const int64_t *off, const int64_t *mpre,
                               const int64_t *aoff, const uint32_t *leave,
                               const int64_t *off_new, GroupRec *rec) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < m;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o0 = off[g], o1 = off[g + 1];
    GroupRec r;
    r.ok = (o0 >= 0 && o1 >= o0 && o1 <= n) ? 1 : 0;  // inconsistent offsets (reported)
    const int64_t c0 = r.ok ? o0 : 0;
    r.sbase = off_new[g] - c0 + mpre[c0];
    r.nbase = off_new[g];
    r.o0 = c0;
    r.stay = r.ok ? (int32_t)((o1 - o0) - (int64_t)leave[g]) : 0;
    r.a0 = aoff[g];
    r.k = (int32_t)(aoff[g + 1] - aoff[g]);
    r.pad = 0;
    rec[g] = r;
  }
}

__global__ void k_rebin_place(int64_t n, const int32_t *gold, const int32_t *gnew,
                              const int64_t *mpre, const GroupRec *rec, const int32_t *alist,
                              int32_t *perm, int32_t *err) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t go = gold[p], gn = gnew[p];
    const bool stayer = go == gn;
    const int64_t mp = stayer ? mpre[p] : 0;
    const GroupRec r = rec[gn];
    if (!r.ok) continue;
    const int64_t below = r.k ? count_below(alist + r.a0, r.k, (int32_t)p) : 0;
    const int64_t pos = stayer ? r.sbase + p - mp + below
                               : r.nbase + (p < r.o0 ? 0 : (int64_t)r.stay) + below;
    if (pos < 0 || pos >= n) {
      atomicCAS(err, 0, 1);
      continue;
    }
    perm[pos] = (int32_t)p;
  }
}

inline int grid_of(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return (int)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

}  // namespace

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_scan(const uint32_t *counts, int64_t m, int64_t *tiles, int64_t *offsets,
                       hipStream_t s);

// scratch: gold, gnew, alist int32[n]; flag uint32[n]; mpre int64[n + 1];
// leave, arrive, acur, cnt uint32[m]; aoff int64[m + 1]; rec GroupRec[m];
// tiles of the scans
hipError_t launch_rebin(int64_t n, int64_t m, int32_t S, int32_t n_cells, const int64_t *off,
                        const int32_t *cells_new, int64_t *off_new, int32_t *perm,
                        int32_t *gold, int32_t *gnew, int32_t *alist, uint32_t *flag,
                        int64_t *mpre, uint32_t *leave, uint32_t *arrive, uint32_t *acur,
                        uint32_t *cnt, int64_t *aoff, void *rec, int64_t *tiles, int32_t *err,
                        hipStream_t s) {
  hipError_t e;
  for (uint32_t *b : {leave, arrive, acur})
    if ((e = launch_fill_u32(b, 0u, m, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_rebin_check, dim3(grid_of(m)), dim3(256), 0, s, off, m, n, err);
  if (n > 0) {
    const int64_t chunks = (n + MARK_CHUNK - 1) / MARK_CHUNK;
    hipLaunchKernelGGL(k_rebin_mark, dim3((unsigned)(chunks < 8192 ? chunks : 8192)),
                       dim3(MARK_TPB), 0, s, n, m, S, n_cells, off, cells_new, gold, gnew, flag,
                       leave, arrive, err);
  }
  hipLaunchKernelGGL(k_rebin_counts, dim3(grid_of(m)), dim3(256), 0, s, m, off, leave, arrive,
                     cnt);
  if ((e = launch_scan(cnt, m, tiles, off_new, s)) != hipSuccess) return e;
  if ((e = launch_scan(arrive, m, tiles, aoff, s)) != hipSuccess) return e;
  if ((e = launch_scan(flag, n, tiles, mpre, s)) != hipSuccess) return e;
  if (n > 0) {
    hipLaunchKernelGGL(k_rebin_lists, dim3(grid_of(n)), dim3(256), 0, s, n, gnew, flag, aoff,
                       acur, alist);
    hipLaunchKernelGGL(k_rebin_sort, dim3(grid_of(m)), dim3(256), 0, s, m, aoff, alist);
    hipLaunchKernelGGL(k_rebin_sort_long, dim3((unsigned)(m < 4096 ? (m > 0 ? m : 1) : 4096)),
                       dim3(LONG_TPB), 0, s, m, aoff, alist);
    hipLaunchKernelGGL(k_rebin_groups, dim3(grid_of(m)), dim3(256), 0, s, m, n, off, mpre, aoff,
                       leave, off_new, reinterpret_cast<GroupRec *>(rec));
    hipLaunchKernelGGL(k_rebin_place, dim3(grid_of(n)), dim3(256), 0, s, n, gold, gnew, mpre,
                       reinterpret_cast<const GroupRec *>(rec), alist, perm, err);
  }
  return hipGetLastError();
}

}  // namespace mcc
