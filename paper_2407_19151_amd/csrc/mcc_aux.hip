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

// data error `code` when the count of a size bucket is not zero (cells the
// caller's entry point does not step)
__global__ void k_flag_nonzero(const uint32_t *count, int32_t code, int32_t *err) {
  if (threadIdx.x == 0 && *count != 0u) atomicCAS(err, 0, code);
}

__global__ void k_inc_u64(uint64_t *p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p += 1ull;
}

// Work lists: cell c of size n goes to the first bucket whose capacity holds
// it.  lists[b * n_cells + i], counts[b].  Empty cells get cell_corr = 0.
// A workgroup counts its cells per bucket in LDS (one LDS atomic per wave and
// bucket), reserves its slots with one global atomic per bucket, and each
// wave writes its cells after its own slots: per-wave global atomics on the
// seven counters would serialize the grid on them.
__global__ void __launch_bounds__(256)
    k_bucket_cells(const int64_t *offsets, int32_t n_cells, int32_t S, int64_t n,
                   int32_t *lists, uint32_t *counts, int32_t *cell_corr, int32_t *err) {
  __shared__ uint32_t lcount[NBUCKET], lbase[NBUCKET];
  const int lane = threadIdx.x & (WAVE - 1);
  const uint64_t below = (1ull << lane) - 1ull;
  for (int64_t c0 = blockIdx.x * (int64_t)blockDim.x; c0 < n_cells;
       c0 += (int64_t)gridDim.x * blockDim.x) {
    if (threadIdx.x < NBUCKET) lcount[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t c = c0 + threadIdx.x;
    int b = -1;  // this lane's bucket, or -1: no list entry
    if (c < n_cells) {
      const int64_t b0 = offsets[c * S], b1 = offsets[(c + 1) * S];
      const int64_t sz = b1 - b0;
      if (b0 < 0 || b1 < b0 || b1 > n) {
        atomicCAS(err, 0, 1);
      } else if (sz == 0) {
        if (cell_corr) cell_corr[c] = 0;
      } else {
        b = 0;
        while (b < NBUCKET && sz > kBucketCap[b]) ++b;
        if (b == NBUCKET) {
          atomicCAS(err, 0, 2);
          if (cell_corr) cell_corr[c] = 0;
          b = -1;
        }
      }
    }
    uint32_t slot = 0;  // the lane's slot among the workgroup's cells of bucket b
    for (int k = 0; k < NBUCKET; ++k) {
      const uint64_t m = __ballot(b == k);
      if (m == 0) continue;  // (uniform over the wave)
      const int leader = __ffsll((unsigned long long)m) - 1;
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(&lcount[k], (uint32_t)__popcll(m));
      base = __shfl(base, leader);
      if (b == k) slot = base + (uint32_t)__popcll(m & below);
    }
    __syncthreads();
    if (threadIdx.x < NBUCKET)
      lbase[threadIdx.x] =
          lcount[threadIdx.x] ? atomicAdd(&counts[threadIdx.x], lcount[threadIdx.x]) : 0u;
    __syncthreads();
    if (b >= 0) lists[(int64_t)b * n_cells + lbase[b] + slot] = (int32_t)c;
    __syncthreads();  // (lcount and lbase are reused by the next chunk)
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

// exclusive scan of the tile sums in one workgroup: serial chunks per
// thread, the chunk sums scanned by shuffles in each wave and across waves
__global__ void k_scan_tile_sums(int64_t *tile_sums, int64_t ntiles) {
  __shared__ int64_t wtot[SCAN_TPB / WAVE];
  const int t = threadIdx.x;
  const int64_t per = (ntiles + SCAN_TPB - 1) / SCAN_TPB;
  const int64_t lo = t * per, hi = lo + per < ntiles ? lo + per : ntiles;
  int64_t acc = 0;
  for (int64_t i = lo; i < hi; ++i) acc += tile_sums[i];
  int64_t incl = acc;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const int64_t y = __shfl_up(incl, d);
    if ((t & (WAVE - 1)) >= d) incl += y;
  }
  if ((t & (WAVE - 1)) == WAVE - 1) wtot[t / WAVE] = incl;
  __syncthreads();
  int64_t run = incl - acc;
#pragma unroll
  for (int k = 0; k < SCAN_TPB / WAVE; ++k)
    if (k < t / WAVE) run += wtot[k];
  for (int64_t i = lo; i < hi; ++i) {
    const int64_t x = tile_sums[i];
    tile_sums[i] = run;
    run += x;
  }
}

// a tile's prefix sums: each thread sums its SCAN_PPT consecutive entries,
// the thread sums are scanned by shuffles in each wave and across waves, and
// each thread writes its entries' offsets
__global__ void k_scan_apply(const uint32_t *in, int64_t m, const int64_t *tile_off,
                             int64_t *out) {
  __shared__ int64_t wtot[SCAN_TPB / WAVE];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)t * SCAN_PPT;
  uint32_t v[SCAN_PPT];
  int64_t sum = 0;
#pragma unroll
  for (int j = 0; j < SCAN_PPT; ++j) {
    v[j] = base + j < m ? in[base + j] : 0u;
    sum += v[j];
  }
  int64_t incl = sum;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const int64_t y = __shfl_up(incl, d);
    if ((t & (WAVE - 1)) >= d) incl += y;
  }
  if ((t & (WAVE - 1)) == WAVE - 1) wtot[t / WAVE] = incl;
  __syncthreads();
  int64_t run = tile_off[blockIdx.x] + incl - sum;
#pragma unroll
  for (int k = 0; k < SCAN_TPB / WAVE; ++k)
    if (k < t / WAVE) run += wtot[k];
#pragma unroll
  for (int j = 0; j < SCAN_PPT; ++j) {
    if (base + j < m) out[base + j] = run;
    run += v[j];
  }
  if (base <= m - 1 && m - 1 < base + SCAN_PPT) out[m] = run;  // the total
}

// ----------------------------------------------------------------------------
// Binning (unsorted entry): a stable LSD radix sort of the group keys
// g = cell * S + species, 9 bits per pass (two passes up to 2^18 groups).  Each wave owns a tile of
// RADIX_ROWS rows of 64 consecutive particles.  Per pass: the tiles' digit
// histograms (digit-major, so one scan gives every (digit, tile) its first
// output position), the scan, and a scatter in which a particle's rank
// among the equal digits of its row comes from ballots over the digit bits,
// rows taken in order: the pass is stable, and no global atomics are used.
// A particle with an id out of range takes the key m (after every group),
// so it sorts to the end; the group offsets then come from the boundaries
// of the sorted keys.
// ----------------------------------------------------------------------------
constexpr int RADIX_BITS = 9, RADIX_BINS = 1 << RADIX_BITS;
constexpr int RADIX_WPB = 4;                      // waves per workgroup (one tile)
constexpr int RADIX_ROWS = 16;                    // rows of 64 particles per wave
constexpr int RADIX_TILE = RADIX_WPB * RADIX_ROWS * WAVE;  // 4096 particles
static_assert(RADIX_BINS % (RADIX_WPB * WAVE) == 0, "digits per thread");

__device__ __forceinline__ uint32_t bin_key(const int32_t *cells, const int32_t *species,
                                            int64_t i, int32_t n_cells, int32_t S,
                                            uint32_t m) {
  const int32_t c = cells[i], sp = species[i];
  return (c < 0 || c >= n_cells || sp < 0 || sp >= S) ? m
                                                       : (uint32_t)c * (uint32_t)S + (uint32_t)sp;
}

// digit histogram of every tile: hist[d * T + tile]
template <bool FIRST>
__global__ void __launch_bounds__(RADIX_WPB * WAVE)
    k_radix_hist(int64_t n, const int32_t *cells, const int32_t *species, int32_t n_cells,
                 int32_t S, uint32_t m, const uint32_t *keys, int shift, int64_t T,
                 uint32_t *hist, int32_t *err) {
  constexpr int TPB = RADIX_WPB * WAVE, DPT = RADIX_BINS / TPB;  // digits per thread
  __shared__ uint32_t h[RADIX_BINS];
  const int t = threadIdx.x;
  const int64_t tile = blockIdx.x;
#pragma unroll
  for (int j = 0; j < DPT; ++j) h[t + j * TPB] = 0u;
  __syncthreads();
  const int64_t base = tile * RADIX_TILE;
  int bad = 0;
  auto add = [&](uint32_t k) {
    if (FIRST && k == m) bad = 1;
    atomicAdd(&h[(k >> shift) & (RADIX_BINS - 1)], 1u);
  };
  if (!FIRST && base + RADIX_TILE <= n) {
    // a whole tile: four keys per load (order does not matter here)
    const uint4 *k4 = reinterpret_cast<const uint4 *>(keys + base);
    for (int j = t; j < RADIX_TILE / 4; j += TPB) {
      const uint4 q = k4[j];
      add(q.x);
      add(q.y);
      add(q.z);
      add(q.w);
    }
  } else {
    for (int j = t; j < RADIX_TILE; j += TPB) {
      const int64_t i = base + j;
      if (i < n) add(FIRST ? bin_key(cells, species, i, n_cells, S, m) : keys[i]);
    }
  }
  if (FIRST && bad) atomicCAS(err, 0, 3);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < DPT; ++j) hist[(int64_t)(t + j * TPB) * T + tile] = h[t + j * TPB];
}

// Stable scatter of (key, value) by the digit; pos[d * T + tile] is the
// first output position of the tile's digit d (scan of the histograms).
// The tile is first sorted by digit in LDS -- wave w ranks its 16 rows in
// order (ballots over the digit bits give a particle's rank among the
// equal digits of its row), the per-(digit, wave) counts are scanned --
// then written out along the sorted order, so every digit's run of the
// tile goes to consecutive addresses.
template <bool FIRST>
__global__ void __launch_bounds__(RADIX_WPB * WAVE)
    k_radix_scatter(int64_t n, const int32_t *cells, const int32_t *species, int32_t n_cells,
                    int32_t S, uint32_t m, const uint32_t *keys_in, const int32_t *vals_in,
                    int shift, int64_t T, const int64_t *pos, uint32_t *keys_out,
                    int32_t *vals_out) {
  __shared__ uint32_t cnt[RADIX_WPB][RADIX_BINS];  // per wave: its digit counts
  __shared__ uint32_t lbase[RADIX_BINS];           // first local slot of each digit
  __shared__ uint32_t gsum[RADIX_WPB];
  __shared__ uint32_t lk[RADIX_TILE];
  __shared__ int32_t lv[RADIX_TILE];
  const int t = threadIdx.x, wv = t / WAVE, lane = t & (WAVE - 1);
  const int64_t tile = blockIdx.x;
  const int64_t base = tile * RADIX_TILE;
  const uint64_t lt = (1ull << lane) - 1ull;
  for (int d = lane; d < RADIX_BINS; d += WAVE) cnt[wv][d] = 0u;
  __builtin_amdgcn_wave_barrier();
  uint32_t rk[RADIX_ROWS];  // rank of the lane's particle among its wave's equal digits
  uint32_t ky[RADIX_ROWS];
  int32_t vl[RADIX_ROWS];
#pragma unroll
  for (int r = 0; r < RADIX_ROWS; ++r) {
    const int64_t i = base + (int64_t)(wv * RADIX_ROWS + r) * WAVE + lane;
    const bool act = i < n;
    uint32_t k = 0u;
    int32_t v = 0;
    if (act) {
      if constexpr (FIRST) {
        k = bin_key(cells, species, i, n_cells, S, m);
        v = (int32_t)i;
      } else {
        k = keys_in[i];
        v = vals_in[i];
      }
    }
    const uint32_t d = (k >> shift) & (RADIX_BINS - 1);
    uint64_t eq = __ballot(act);
#pragma unroll
    for (int b = 0; b < RADIX_BITS; ++b) {
      const uint64_t bb = __ballot((d >> b) & 1u);
      eq &= ((d >> b) & 1u) ? bb : ~bb;
    }
    rk[r] = act ? cnt[wv][d] + (uint32_t)__popcll(eq & lt) : 0u;
    ky[r] = k;
    vl[r] = v;
    // (every lane has read the count before the leader of its digit advances it)
    __builtin_amdgcn_wave_barrier();
    if (act && (eq & lt) == 0ull) cnt[wv][d] += (uint32_t)__popcll(eq);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // digit totals of the tile and their exclusive scan (thread t owns the
  // DPT consecutive digits from DPT t)
  constexpr int TPB = RADIX_WPB * WAVE, DPT = RADIX_BINS / TPB;
  uint32_t tot[DPT], sum = 0;
#pragma unroll
  for (int j = 0; j < DPT; ++j) {
    tot[j] = 0;
#pragma unroll
    for (int w = 0; w < RADIX_WPB; ++w) tot[j] += cnt[w][DPT * t + j];
    sum += tot[j];
  }
  uint32_t gt;
  uint32_t run = block_excl_scan1<TPB, false>(sum, gsum, gt);
#pragma unroll
  for (int j = 0; j < DPT; ++j) {
    const int d = DPT * t + j;
    lbase[d] = run;
    // each wave's first slot within the digit
#pragma unroll
    for (int w = 0; w < RADIX_WPB; ++w) {
      const uint32_t c = cnt[w][d];
      cnt[w][d] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RADIX_ROWS; ++r) {
    const int64_t i = base + (int64_t)(wv * RADIX_ROWS + r) * WAVE + lane;
    if (i < n) {
      const uint32_t d = (ky[r] >> shift) & (RADIX_BINS - 1);
      const uint32_t slot = cnt[wv][d] + rk[r];
      lk[slot] = ky[r];
      lv[slot] = vl[r];
    }
  }
  __syncthreads();
  const int64_t tn = n - base < RADIX_TILE ? n - base : RADIX_TILE;
  for (int j = t; j < tn; j += RADIX_WPB * WAVE) {
    const uint32_t k = lk[j];
    const uint32_t d = (k >> shift) & (RADIX_BINS - 1);
    const int64_t g = pos[(int64_t)d * T + tile] + (j - (int64_t)lbase[d]);
    keys_out[g] = k;
    vals_out[g] = lv[j];
  }
}

// group offsets from the sorted keys: offsets[g] = first position whose key
// is >= g (keys above m - 1 mark particles with bad ids, at the end)
__global__ void k_bin_bounds(int64_t n, const uint32_t *keys, uint32_t m, int64_t *offsets) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t kp = i == 0 ? -1 : (int64_t)keys[i - 1];
    const int64_t k = i == n ? (int64_t)m : ((int64_t)keys[i] < (int64_t)m ? keys[i] : m);
    for (int64_t g = kp + 1; g <= k; ++g) offsets[g] = i;
  }
}

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

// The unsorted entry's payload moves through 32-byte records (w, vx, vy, vz)
// of a context-owned array in the caller's order: a particle's random access
// is then one aligned 32-byte record, one memory segment, instead of an 8-byte
// word in each of four arrays.  Packing and unpacking stream.
struct alignas(32) Rec4 {
  double w, x, y, z;
};

__global__ void k_pack_rec(int64_t n, const double *w, const double *vx, const double *vy,
                           const double *vz, Rec4 *rec) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    rec[i] = Rec4{w[i], vx[i], vy[i], vz[i]};
}

__global__ void k_gather_rec(int64_t n, const int32_t *perm, const Rec4 *rec, double *gw,
                             double *gx, double *gy, double *gz) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = perm[j];
    if (i < 0 || i >= n) continue;
    const Rec4 r = rec[i];
    gw[j] = r.w;
    gx[j] = r.x;
    gy[j] = r.y;
    gz[j] = r.z;
  }
}

// whole records back (the weight unchanged), then the velocities out
__global__ void k_scatter_rec(int64_t n, const int32_t *perm, const double *gw, const double *gx,
                              const double *gy, const double *gz, Rec4 *rec) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = perm[j];
    if (i < 0 || i >= n) continue;
    rec[i] = Rec4{gw[j], gx[j], gy[j], gz[j]};
  }
}

__global__ void k_unpack_v(int64_t n, const Rec4 *rec, double *vx, double *vy, double *vz) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const Rec4 r = rec[i];
    vx[i] = r.x;
    vy[i] = r.y;
    vz[i] = r.z;
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

hipError_t launch_flag_nonzero(const uint32_t *count, int32_t code, int32_t *err,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_flag_nonzero, dim3(1), dim3(64), 0, s, count, code, err);
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

// scratch of launch_bin: two key and two value buffers of n u32, the tiles'
// digit histograms and their scanned positions
int64_t bin_tiles(int64_t n) { return (n + RADIX_TILE - 1) / RADIX_TILE; }
// entries of the digit histograms (and of their scanned positions, + 1)
int64_t bin_hist_entries(int64_t n) {
  const int64_t T = bin_tiles(n);
  return (int64_t)RADIX_BINS * (T > 0 ? T : 1);
}

hipError_t launch_bin(int64_t n, const int32_t *cells, const int32_t *species, int32_t n_cells,
                      int32_t S, uint32_t *keys0, uint32_t *keys1, int32_t *vals0,
                      int32_t *vals1, uint32_t *hist, int64_t *pos, int64_t *tiles,
                      int64_t *offsets, int32_t *perm, int32_t *err, hipStream_t s) {
  const uint32_t m = (uint32_t)((int64_t)n_cells * S);
  int bits = 1;
  while (bits < 32 && (m >> bits) != 0u) ++bits;  // keys run up to m (the bad-id key)
  const int passes = (bits + RADIX_BITS - 1) / RADIX_BITS;
  const int64_t T = bin_tiles(n);
  uint32_t *kb[2] = {keys0, keys1};
  int32_t *vb[2] = {vals0, vals1};
  if (n > 0) {
    const int grid = (int)T;
    for (int p = 0; p < passes; ++p) {
      const int shift = p * RADIX_BITS;
      const uint32_t *kin = p ? kb[(p - 1) & 1] : nullptr;
      const int32_t *vin = p ? vb[(p - 1) & 1] : nullptr;
      uint32_t *kout = kb[p & 1];
      int32_t *vout = p == passes - 1 ? perm : vb[p & 1];
      if (p == 0)
        hipLaunchKernelGGL(k_radix_hist<true>, dim3(grid), dim3(RADIX_WPB * WAVE), 0, s, n,
                           cells, species, n_cells, S, m, kin, shift, T, hist, err);
      else
        hipLaunchKernelGGL(k_radix_hist<false>, dim3(grid), dim3(RADIX_WPB * WAVE), 0, s, n,
                           cells, species, n_cells, S, m, kin, shift, T, hist, err);
      hipError_t e = launch_scan(hist, (int64_t)RADIX_BINS * T, tiles, pos, s);
      if (e != hipSuccess) return e;
      if (p == 0)
        hipLaunchKernelGGL(k_radix_scatter<true>, dim3(grid), dim3(RADIX_WPB * WAVE), 0, s, n,
                           cells, species, n_cells, S, m, kin, vin, shift, T, pos, kout, vout);
      else
        hipLaunchKernelGGL(k_radix_scatter<false>, dim3(grid), dim3(RADIX_WPB * WAVE), 0, s, n,
                           cells, species, n_cells, S, m, kin, vin, shift, T, pos, kout, vout);
    }
  }
  hipLaunchKernelGGL(k_bin_bounds, dim3(grid_for(n + 1, 256)), dim3(256), 0, s, n,
                     kb[(passes - 1) & 1], m, offsets);
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

hipError_t launch_gather(int64_t n, const int32_t *perm, const double *w, const double *vx,
                         const double *vy, const double *vz, double *gw, double *gx, double *gy,
                         double *gz, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather, dim3(grid_for(n, 256)), dim3(256), 0, s, n, perm, w, vx, vy, vz,
                     gw, gx, gy, gz);
  return hipGetLastError();
}

// gather through records: rec (32 * n bytes, 32-byte aligned) is scratch
hipError_t launch_gather_rec(int64_t n, const int32_t *perm, const double *w, const double *vx,
                             const double *vy, const double *vz, void *rec, double *gw,
                             double *gx, double *gy, double *gz, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  Rec4 *r = static_cast<Rec4 *>(rec);
  hipLaunchKernelGGL(k_pack_rec, dim3(grid_for(n, 256)), dim3(256), 0, s, n, w, vx, vy, vz, r);
  hipLaunchKernelGGL(k_gather_rec, dim3(grid_for(n, 256)), dim3(256), 0, s, n, perm, r, gw, gx,
                     gy, gz);
  return hipGetLastError();
}

hipError_t launch_scatter_back_rec(int64_t n, const int32_t *perm, const double *gw,
                                   const double *gx, const double *gy, const double *gz,
                                   void *rec, double *vx, double *vy, double *vz,
                                   hipStream_t s) {
  if (n <= 0) return hipSuccess;
  Rec4 *r = static_cast<Rec4 *>(rec);
  hipLaunchKernelGGL(k_scatter_rec, dim3(grid_for(n, 256)), dim3(256), 0, s, n, perm, gw, gx, gy,
                     gz, r);
  hipLaunchKernelGGL(k_unpack_v, dim3(grid_for(n, 256)), dim3(256), 0, s, n, r, vx, vy, vz);
  return hipGetLastError();
}


}  // namespace mcc
