// mcc_aux.hip -- small kernels around the collide kernels: cell-size
// bucketing of the work list, cell binning for the unsorted entry (count,
// scan, scatter, per-group canonical order, gather/scatter of the payload),
// and counter resets.  Every kernel bounds-checks its indices.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mcc.h"
#include "mcc_device.hpp"
#include "mcc_variants.hpp"

namespace mcc {

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// weights must be positive and finite (a species' density is sum w / dV)
__global__ void k_check_weights(int64_t n, const double *w, int32_t *err) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double x = w[i];
    if (!(x > 0.0) || x == __builtin_inf()) {
      atomicCAS(err, 0, 4);
      return;
    }
  }
}

__global__ void k_zero_stats(mcc_stats *s) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    s->pairs = s->corr_pairs = s->failed = s->collisions = 0ull;
    s->max_rel_dP = 0.0;
    s->max_rel_dE = 0.0;
  }
}

__global__ void k_set_u64(uint64_t *p, uint64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void k_inc_u64(uint64_t *p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p += 1ull;
}

// Work lists: cell c of size n goes to the first bucket whose capacity holds
// it.  lists[b * n_cells + i], counts[b].  Empty cells get cell_corr = 0.
__global__ void k_bucket_cells(const int64_t *offsets, int32_t n_cells, int32_t S, int64_t n,
                               int32_t *lists, uint32_t *counts, int32_t *cell_corr,
                               int32_t *err) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n_cells;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b0 = offsets[c * S], b1 = offsets[(c + 1) * S];
    if (b0 < 0 || b1 < b0 || b1 > n) {
      atomicCAS(err, 0, 1);
      continue;
    }
    const int64_t sz = b1 - b0;
    if (sz == 0) {
      if (cell_corr) cell_corr[c] = 0;
      continue;
    }
    int b = 0;
    while (b < NBUCKET && sz > kBucketCap[b]) ++b;
    if (b == NBUCKET) {
      atomicCAS(err, 0, 2);
      if (cell_corr) cell_corr[c] = 0;
      continue;
    }
    const uint32_t pos = atomicAdd(&counts[b], 1u);
    lists[(int64_t)b * n_cells + pos] = (int32_t)c;
  }
}

// ----------------------------------------------------------------------------
// Binning (unsorted entry)
// ----------------------------------------------------------------------------
__global__ void k_bin_count(int64_t n, const int32_t *cells, const int32_t *species,
                            int32_t n_cells, int32_t S, uint32_t *counts, int32_t *err) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = cells[i], s = species[i];
    if (c < 0 || c >= n_cells || s < 0 || s >= S) {
      atomicCAS(err, 0, 3);
      continue;
    }
    atomicAdd(&counts[(int64_t)c * S + s], 1u);
  }
}

// three-phase scan of u32 counts into int64 offsets (offsets[m] = total)
constexpr int SCAN_TPB = 256, SCAN_PPT = 8, SCAN_TILE = SCAN_TPB * SCAN_PPT;

__global__ void k_scan_tiles(const uint32_t *in, int64_t m, int64_t *tile_sums) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  int64_t acc = 0;
  for (int j = threadIdx.x; j < SCAN_TILE; j += SCAN_TPB)
    if (base + j < m) acc += in[base + j];
  __shared__ int64_t red[SCAN_TPB];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = SCAN_TPB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = red[0];
}

// exclusive scan of the tile sums in one workgroup (serial chunks per thread)
__global__ void k_scan_tile_sums(int64_t *tile_sums, int64_t ntiles) {
  __shared__ int64_t part[SCAN_TPB];
  const int64_t per = (ntiles + SCAN_TPB - 1) / SCAN_TPB;
  const int64_t lo = threadIdx.x * per, hi = lo + per < ntiles ? lo + per : ntiles;
  int64_t acc = 0;
  for (int64_t i = lo; i < hi; ++i) acc += tile_sums[i];
  part[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int i = 0; i < SCAN_TPB; ++i) {
      const int64_t x = part[i];
      part[i] = run;
      run += x;
    }
  }
  __syncthreads();
  int64_t run = part[threadIdx.x];
  for (int64_t i = lo; i < hi; ++i) {
    const int64_t x = tile_sums[i];
    tile_sums[i] = run;
    run += x;
  }
}

// a tile's prefix sums: each thread sums its SCAN_PPT consecutive entries,
// the thread sums are scanned in LDS (log2 SCAN_TPB doubling steps), and
// each thread writes its entries' offsets
__global__ void k_scan_apply(const uint32_t *in, int64_t m, const int64_t *tile_off,
                             int64_t *out) {
  __shared__ int64_t part[SCAN_TPB];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)t * SCAN_PPT;
  uint32_t v[SCAN_PPT];
  int64_t sum = 0;
#pragma unroll
  for (int j = 0; j < SCAN_PPT; ++j) {
    v[j] = base + j < m ? in[base + j] : 0u;
    sum += v[j];
  }
  part[t] = sum;
  __syncthreads();
  for (int d = 1; d < SCAN_TPB; d <<= 1) {
    const int64_t x = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += x;
    __syncthreads();
  }
  int64_t run = tile_off[blockIdx.x] + part[t] - sum;
#pragma unroll
  for (int j = 0; j < SCAN_PPT; ++j) {
    if (base + j < m) out[base + j] = run;
    run += v[j];
  }
  if (base <= m - 1 && m - 1 < base + SCAN_PPT) out[m] = run;  // the total
}

// unstable placement of original indices; cursor starts as a copy of offsets
__global__ void k_bin_place(int64_t n, const int32_t *cells, const int32_t *species,
                            int32_t n_cells, int32_t S, unsigned long long *cursor,
                            int32_t *perm) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = cells[i], s = species[i];
    if (c < 0 || c >= n_cells || s < 0 || s >= S) continue;
    const unsigned long long pos = atomicAdd(&cursor[(int64_t)c * S + s], 1ull);
    if ((int64_t)pos < n) perm[pos] = (int32_t)i;
  }
}

__global__ void k_copy_i64_u64(const int64_t *in, unsigned long long *out, int64_t m) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (unsigned long long)in[i];
}

// Canonical (ascending original index) order inside every (cell, species)
// group: a bucket-rank sort of the group's indices.  Groups larger than CAP
// are appended to a list for the large-group form, which runs one wave per
// group on global scratch (one wave keeps every exchange in program order).
template <int TPC, int CAP, bool G>
__global__ void __launch_bounds__(TPC) k_bin_canon(const int64_t *offsets, int64_t m,
                                                   int32_t *perm, int32_t *big_list,
                                                   uint32_t *big_count, const int32_t *list,
                                                   const uint32_t *list_count, uint32_t *gscr,
                                                   uint64_t gstride) {
  constexpr int PPT = CAP / TPC;
  static_assert(!G || TPC == WAVE, "the global form runs one wave per group");
  __shared__ uint32_t wsum[TPC / WAVE];
  __shared__ uint32_t maxocc;
  __shared__ uint64_t mm[2 * 2 * (TPC / WAVE)];
  // the bucket counters are LDS in both forms (global atomics complete in L2
  // and later plain loads could hit stale L1 lines)
  __shared__ uint32_t cnt[CAP + 1];
  uint32_t *vals, *slot = nullptr;
  uint16_t *mem, *out;
  if constexpr (!G) {
    __shared__ uint32_t lv[CAP];
    __shared__ uint16_t lm[CAP], lo[CAP];
    vals = lv;
    mem = lm;
    out = lo;
  } else {
    uint32_t *g = gscr + (uint64_t)blockIdx.x * gstride;
    vals = g;
    slot = g + CAP;
    mem = reinterpret_cast<uint16_t *>(g + 2 * CAP);
    out = mem + CAP;
  }
  const int64_t ngroups = G ? (int64_t)*list_count : m;
  for (int64_t gi = blockIdx.x; gi < ngroups; gi += gridDim.x) {
    const int64_t g = G ? (int64_t)list[gi] : gi;
    const int64_t b0 = offsets[g], b1 = offsets[g + 1];
    const int64_t len = b1 - b0;
    if (len <= 1) continue;
    if (len > CAP) {
      if (!G && threadIdx.x == 0) {
        const uint32_t p = atomicAdd(big_count, 1u);
        big_list[p] = (int32_t)g;
      }
      continue;
    }
    const int n = (int)len;
    uint64_t lo[1] = {~0ull}, hi[1] = {0ull};
    for (int i = threadIdx.x; i < n; i += TPC) {
      const uint32_t v = (uint32_t)perm[b0 + i];
      vals[i] = v;
      lo[0] = v < lo[0] ? v : lo[0];
      hi[0] = v > hi[0] ? v : hi[0];
    }
    block_minmax_u64<TPC, 1>(lo, hi, mm);
    __syncthreads();
    const double scale = (double)n / ((double)(hi[0] - lo[0]) + 1.0);
    const uint64_t vlo = lo[0];
    bucket_rank_sort<TPC, PPT, G>(
        n, cnt, mem, out, wsum, &maxocc,
        [&](int i) -> uint32_t {
          const uint32_t k = (uint32_t)((double)(vals[i] - vlo) * scale);
          return k < (uint32_t)n ? k : (uint32_t)(n - 1);
        },
        [&](int o, int i) -> bool { return vals[o] < vals[i]; }, slot);
    for (int i = threadIdx.x; i < n; i += TPC) perm[b0 + i] = (int32_t)vals[out[i]];
    __syncthreads();
  }
}

template __global__ void k_bin_canon<256, 4096, false>(const int64_t *, int64_t, int32_t *,
                                                       int32_t *, uint32_t *, const int32_t *,
                                                       const uint32_t *, uint32_t *, uint64_t);
template __global__ void k_bin_canon<64, MCC_MAX_CELL, true>(const int64_t *, int64_t,
                                                             int32_t *, int32_t *, uint32_t *,
                                                             const int32_t *, const uint32_t *,
                                                             uint32_t *, uint64_t);

__global__ void k_gather(int64_t n, const int32_t *perm, const double *w, const double *vx,
                         const double *vy, const double *vz, double *gw, double *gx, double *gy,
                         double *gz) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = perm[j];
    if (i < 0 || i >= n) continue;
    gw[j] = w[i];
    gx[j] = vx[i];
    gy[j] = vy[i];
    gz[j] = vz[i];
  }
}

__global__ void k_scatter_back(int64_t n, const int32_t *perm, const double *gx,
                               const double *gy, const double *gz, double *vx, double *vy,
                               double *vz) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = perm[j];
    if (i < 0 || i >= n) continue;
    vx[i] = gx[j];
    vy[i] = gy[j];
    vz[i] = gz[j];
  }
}

}  // namespace mcc

namespace mcc {
// the angle sampler of the collision step, evaluated alone
template <typename T>
__global__ void k_sample_angles(int method, int64_t n, const double *s, const uint32_t *a0,
                                const uint32_t *a1, double *oc, double *st, double *A,
                                const double2 *tab) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    T o, t;
    sample_angle<T>(method, (T)s[i], a0[i], a1[i], o, t, tab);
    oc[i] = (double)o;
    st[i] = (double)t;
    if (A) A[i] = method == 1 ? (double)n97_A_fast<T>((T)s[i], tab) : 0.0;
  }
}

// the N97 table: A at the knots t_i = T0 + i h (s = e^t) from the bracketed
// solver, and h dA/dt = -h s exp(-s) / L'(A) from differentiating L(A) = exp(-s)
__global__ void k_n97_table(double2 *tab) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N97_TN) return;
  const double s = exp(N97_T0 + i * N97_H);
  const double A = n97_A<double>(s);
  const double dAdt = -s * exp(-s) / langevin_deriv<double>(A);
  tab[i] = make_double2(A, N97_H * dAdt);
}
}  // namespace mcc

// ----------------------------------------------------------------------------
// Host-side launchers (called by the runtime in mcc_api.hip)
// ----------------------------------------------------------------------------
namespace mcc {

static inline int grid_for(int64_t n, int tpb) {
  int64_t g = (n + tpb - 1) / tpb;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (int)g;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_check_weights(int64_t n, const double *w, int32_t *err, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_weights, dim3(grid_for(n, 256)), dim3(256), 0, s, n, w, err);
  return hipGetLastError();
}

hipError_t launch_zero_stats(mcc_stats *st, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_stats, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_set_u64(uint64_t *p, uint64_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

hipError_t launch_inc_u64(uint64_t *p, hipStream_t s) {
  hipLaunchKernelGGL(k_inc_u64, dim3(1), dim3(64), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_bucket_cells(const int64_t *offsets, int32_t n_cells, int32_t S, int64_t n,
                               int32_t *lists, uint32_t *counts, int32_t *cell_corr, int32_t *err,
                               hipStream_t s) {
  if (n_cells <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bucket_cells, dim3(grid_for(n_cells, 256)), dim3(256), 0, s, offsets,
                     n_cells, S, n, lists, counts, cell_corr, err);
  return hipGetLastError();
}

// offsets[m+1] from counts[m]; tiles: scratch of ceil(m / SCAN_TILE) int64
hipError_t launch_scan(const uint32_t *counts, int64_t m, int64_t *tiles, int64_t *offsets,
                       hipStream_t s) {
  const int64_t nt = (m + SCAN_TILE - 1) / SCAN_TILE;
  if (nt == 0) {
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(64), 0, s, reinterpret_cast<uint64_t *>(offsets),
                       0ull);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(SCAN_TPB), 0, s, counts, m, tiles);
  hipLaunchKernelGGL(k_scan_tile_sums, dim3(1), dim3(SCAN_TPB), 0, s, tiles, nt);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nt), dim3(SCAN_TPB), 0, s, counts, m, tiles,
                     offsets);
  return hipGetLastError();
}

int64_t scan_tiles_needed(int64_t m) { return (m + SCAN_TILE - 1) / SCAN_TILE + 1; }

hipError_t launch_bin(int64_t n, const int32_t *cells, const int32_t *species, int32_t n_cells,
                      int32_t S, uint32_t *counts, int64_t *tiles, int64_t *offsets,
                      unsigned long long *cursor, int32_t *perm, int32_t *big_list,
                      uint32_t *big_count, uint32_t *canon_scr, int canon_big_grid, int32_t *err,
                      hipStream_t s) {
  const int64_t m = (int64_t)n_cells * S;
  hipError_t e = launch_fill_u32(counts, 0u, m, s);
  if (e != hipSuccess) return e;
  if (n > 0)
    hipLaunchKernelGGL(k_bin_count, dim3(grid_for(n, 256)), dim3(256), 0, s, n, cells, species,
                       n_cells, S, counts, err);
  e = launch_scan(counts, m, tiles, offsets, s);
  if (e != hipSuccess) return e;
  if (m > 0)
    hipLaunchKernelGGL(k_copy_i64_u64, dim3(grid_for(m, 256)), dim3(256), 0, s, offsets, cursor,
                       m);
  if (n > 0)
    hipLaunchKernelGGL(k_bin_place, dim3(grid_for(n, 256)), dim3(256), 0, s, n, cells, species,
                       n_cells, S, cursor, perm);
  e = launch_fill_u32(big_count, 0u, 1, s);
  if (e != hipSuccess) return e;
  if (m > 0) {
    const int g = m < 65536 ? (int)m : 65536;
    hipLaunchKernelGGL((k_bin_canon<256, 4096, false>), dim3(g), dim3(256), 0, s, offsets, m,
                       perm, big_list, big_count, (const int32_t *)nullptr,
                       (const uint32_t *)nullptr, (uint32_t *)nullptr, (uint64_t)0);
    hipLaunchKernelGGL((k_bin_canon<64, MCC_MAX_CELL, true>), dim3(canon_big_grid), dim3(64),
                       0, s, offsets, m, perm, big_list, big_count, (const int32_t *)big_list,
                       (const uint32_t *)big_count, canon_scr, (uint64_t)(3 * MCC_MAX_CELL));
  }
  return hipGetLastError();
}

hipError_t launch_n97_table(double2 *tab, hipStream_t s) {
  hipLaunchKernelGGL(k_n97_table, dim3((N97_TN + 63) / 64), dim3(64), 0, s, tab);
  return hipGetLastError();
}

hipError_t launch_sample_angles(int method, int precision, int64_t n, const double *s,
                                const uint32_t *a0, const uint32_t *a1, double *oc, double *st,
                                double *A, const double2 *tab, hipStream_t st_) {
  if (n <= 0) return hipSuccess;
  if (precision == 1)
    hipLaunchKernelGGL(k_sample_angles<float>, dim3(grid_for(n, 256)), dim3(256), 0, st_, method,
                       n, s, a0, a1, oc, st, A, tab);
  else
    hipLaunchKernelGGL(k_sample_angles<double>, dim3(grid_for(n, 256)), dim3(256), 0, st_,
                       method, n, s, a0, a1, oc, st, A, tab);
  return hipGetLastError();
}

uint64_t canon_scratch_words() { return 3ull * MCC_MAX_CELL; }

hipError_t launch_gather(int64_t n, const int32_t *perm, const double *w, const double *vx,
                         const double *vy, const double *vz, double *gw, double *gx, double *gy,
                         double *gz, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather, dim3(grid_for(n, 256)), dim3(256), 0, s, n, perm, w, vx, vy, vz,
                     gw, gx, gy, gz);
  return hipGetLastError();
}

hipError_t launch_scatter_back(int64_t n, const int32_t *perm, const double *gx,
                               const double *gy, const double *gz, double *vx, double *vy,
                               double *vz, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_back, dim3(grid_for(n, 256)), dim3(256), 0, s, n, perm, gx, gy,
                     gz, vx, vy, vz);
  return hipGetLastError();
}

}  // namespace mcc
