// mcc_api.hip -- host runtime behind include/mcc.h: context and workspace,
// argument checks, per-collision constants, size-bucketed launches of the
// collide kernel variants, the unsorted entry (binning + gather/scatter),
// and the batched plan (device work lists, autotuned variants, HIP graph).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mcc.h"
#include "mcc_kernel_args.hpp"
#include "mcc_variants.hpp"

const void *const *mcc_kernel_table_fp64();
const void *const *mcc_kernel_table_fp32();
const void *const *mcc_kernel_table_rel();
const void *const *mcc_kernel_table_tan();
const void *const *mcc_kernel_table_fp64_diag();
const void *const *mcc_kernel_table_fp32_diag();
const void *const *mcc_kernel_table_rel_diag();
const void *const *mcc_kernel_table_fp64_nxn();
const void *const *mcc_kernel_table_fp32_nxn();
const void *const *mcc_kernel_table_rel_nxn();
const void *const *mcc_kernel_table_fp64_dup();
const void *const *mcc_kernel_table_fp32_dup();
const void *const *mcc_kernel_table_rel_dup();

namespace mcc {
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_zero_stats(mcc_stats *st, hipStream_t s);
hipError_t launch_check_weights(int64_t n, const double *w, int32_t *err, hipStream_t s);
hipError_t launch_set_u64(uint64_t *p, uint64_t v, hipStream_t s);
hipError_t launch_inc_u64(uint64_t *p, hipStream_t s);
hipError_t launch_flag_nonzero(const uint32_t *count, int32_t code, int32_t *err,
                               hipStream_t s);
hipError_t launch_bucket_cells(const int64_t *offsets, int32_t n_cells, int32_t S, int64_t n,
                               int32_t *lists, uint32_t *counts, int32_t *cell_corr, int32_t *err,
                               hipStream_t s);
int64_t scan_tiles_needed(int64_t m);
int64_t bin_tiles(int64_t n);
int64_t bin_hist_entries(int64_t n);
hipError_t launch_bin(int64_t n, const int32_t *cells, const int32_t *species, int32_t n_cells,
                      int32_t S, uint32_t *keys0, uint32_t *keys1, int32_t *vals0,
                      int32_t *vals1, uint32_t *hist, int64_t *pos, int64_t *tiles,
                      int64_t *offsets, int32_t *perm, int32_t *err, hipStream_t s);
hipError_t launch_sample_angles(int method, int precision, int64_t n, const double *s,
                                const uint32_t *a0, const uint32_t *a1, double *oc, double *st,
                                double *A, const double2 *tab, hipStream_t st_);
hipError_t launch_n97_table(double2 *tab, hipStream_t s);
size_t rebin_scratch_bytes(int64_t n, int64_t m);
int64_t rebin_tiles_needed(int64_t n, int64_t m);
hipError_t launch_rebin(int64_t n, int64_t m, int32_t S, int32_t n_cells, const int64_t *off,
                        const int32_t *cells_new, int64_t *off_new, int32_t *perm,
                        void *scratch, int64_t *tiles, int32_t *err, hipStream_t s);
hipError_t launch_gather_rec(int64_t n, const int32_t *perm, const double *w, const double *vx,
                             const double *vy, const double *vz, void *rec, double *gw,
                             double *gx, double *gy, double *gz, hipStream_t s);
hipError_t launch_scatter_back_rec(int64_t n, const int32_t *perm, const double *gw,
                                   const double *gx, const double *gy, const double *gz,
                                   void *rec, double *vx, double *vy, double *vz,
                                   hipStream_t s);
hipError_t launch_gather(int64_t n, const int32_t *perm, const double *w, const double *vx,
                         const double *vy, const double *vz, double *gw, double *gx, double *gy,
                         double *gz, hipStream_t s);
struct AdjointArgs;
hipError_t launch_adjoint(const AdjointArgs &base, bool fp32, const int32_t *lists,
                          const uint32_t *counts, int32_t n_cells, int b, int tpc, int cap,
                          int grid, hipStream_t s);
hipError_t launch_sum_f64(const double *x, int64_t n, double *out, hipStream_t s);
}  // namespace mcc
#include "mcc_adjoint_args.hpp"

using namespace mcc;

namespace {

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  bool ensure(size_t want) {
    if (want <= bytes) return true;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    if (hipMalloc(&p, want) != hipSuccess) {
      p = nullptr;
      return false;
    }
    bytes = want;
    return true;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T *as() const {
    return reinterpret_cast<T *>(p);
  }
};

// global scratch of the large-cell (GLOBAL layout) variants.  A context
// owns one for its direct calls and every plan owns its own: a plan's graph
// holds the scratch address, so a buffer the context later grows (and
// reallocates) must never be the one a plan replays against.
struct BigScratch {
  DevBuf big4k, big32k;
  void release() {
    big4k.release();
    big32k.release();
  }
};

const void *const *kernel_table(int mode) {
  switch (mode) {
    case MODE_FP64: return mcc_kernel_table_fp64();
    case MODE_FP32: return mcc_kernel_table_fp32();
    case MODE_TAN: return mcc_kernel_table_tan();
    case MODE_FP64_DIAG: return mcc_kernel_table_fp64_diag();
    case MODE_FP32_DIAG: return mcc_kernel_table_fp32_diag();
    case MODE_REL_DIAG: return mcc_kernel_table_rel_diag();
    case MODE_FP64_NXN: return mcc_kernel_table_fp64_nxn();
    case MODE_FP32_NXN: return mcc_kernel_table_fp32_nxn();
    case MODE_REL_NXN: return mcc_kernel_table_rel_nxn();
    case MODE_FP64_DUP: return mcc_kernel_table_fp64_dup();
    case MODE_FP32_DUP: return mcc_kernel_table_fp32_dup();
    case MODE_REL_DUP: return mcc_kernel_table_rel_dup();
    default: return mcc_kernel_table_rel();
  }
}

}  // namespace

// A side stream and two events (default priority, created once) that let the
// 4096 bucket run on a branch beside the 2048 bucket: its cells take a whole
// CU's LDS each and drain unevenly, and the 2048 cells fill the CUs it leaves.
// Every other bucket runs alone: cells of different sizes sharing CUs slowed
// the step (2-7 %).
struct Branch {
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

struct mcc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  Branch branch;  // the per-call steps' branch (launch_buckets)
  int n_cu = 0;
  bool validate = false;
  int32_t *err = nullptr;  // device error word
  DevBuf lists, counts;
  BigScratch big;  // large-cell scratch of the direct (non-plan) calls
  DevBuf n97;  // N97 A(s) table (built once)
  // per size bucket: the collide kernels' cell-claim and finished-workgroup
  // counters (zero between launches: each launch resets them at its end, so
  // launches of one context must not overlap)
  DevBuf work;
  // unsorted entry
  DevBuf tiles, off, perm, gw, gx, gy, gz, rec;
  DevBuf bin_k0, bin_k1, bin_v0, bin_v1, bin_hist, bin_pos;  // radix-sort scratch
  // reverse-mode form: per-workgroup scratch (cells up to 4096 particles,
  // and above), per-cell lnL adjoints
  DevBuf adj_small, adj_big, adj_part;
  // incremental re-binning
  DevBuf rb;
  int grid[NMODE][NVARIANT] = {};
  int variant[NBUCKET] = {};
};

struct mcc_plan {
  mcc_ctx *ctx = nullptr;
  CollideArgs args{};
  int mode = 0;
  int32_t n_cells = 0;
  int variant[NBUCKET] = {};
  uint32_t hcount[NBUCKET] = {};  // cells per bucket (fixed for the plan)
  DevBuf lists, counts, step;
  BigScratch big;          // large-cell scratch of this plan's kernels (its graph holds it)
  DevBuf prep, prep_word;  // weight data of the bound population (PREP_READ)
  mcc_stats *stats = nullptr;
  int32_t *cell_corr = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  double tuned_ms[NBUCKET][NVARIANT] = {};
};

namespace {

mcc_status from_hip(hipError_t e) {
  if (e == hipSuccess) return MCC_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return MCC_ERR_OOM;
  return MCC_ERR_DEVICE;
}

#define HIP_TRY(expr)                         \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return from_hip(e_); \
  } while (0)

// kernel family of a step: precision / physics, and whether diagnostics are
// measured (A.diag, set by fill_args)
int mode_of(const mcc_params *p, const CollideArgs &A) {
  if (p->pairing == MCC_PAIRING_NXN)
    return p->relativistic ? MODE_REL_NXN
           : p->precision == MCC_FP32_KINEMATICS ? MODE_FP32_NXN : MODE_FP64_NXN;
  if (p->pairing == MCC_PAIRING_DUPLICITY)
    return p->relativistic ? MODE_REL_DUP
           : p->precision == MCC_FP32_KINEMATICS ? MODE_FP32_DUP : MODE_FP64_DUP;
  if (p->relativistic) return A.diag ? MODE_REL_DIAG : MODE_REL;
  if (p->precision == MCC_FP32_KINEMATICS) return A.diag ? MODE_FP32_DIAG : MODE_FP32;
  return A.diag ? MODE_FP64_DIAG : MODE_FP64;
}

// host checks of the step arguments shared by every entry point
mcc_status check_step(int64_t n, int32_t n_cells, int32_t n_species, const double *w,
                      const double *vx, const double *vy, const double *vz,
                      const double *cell_volume, double dVs, const mcc_species *sp,
                      int32_t n_coll, const mcc_collision *coll, double dt, double lnL,
                      const mcc_params *p) {
  if (n < 0 || n_cells < 0 || n_species < 1 || n_species > MCC_MAX_SPECIES) return MCC_ERR_INVALID;
  if (n_coll < 0 || n_coll > MCC_MAX_COLLISIONS) return MCC_ERR_INVALID;
  if (n > 0 && (!w || !vx || !vy || !vz)) return MCC_ERR_INVALID;
  if (n > (int64_t)INT32_MAX) return MCC_ERR_UNSUPPORTED;
  if (!sp || (n_coll > 0 && !coll) || !p) return MCC_ERR_INVALID;
  for (int s = 0; s < n_species; ++s)
    if (!(sp[s].mass > 0.0) || !std::isfinite(sp[s].mass) || !std::isfinite(sp[s].charge))
      return MCC_ERR_INVALID;
  for (int k = 0; k < n_coll; ++k)
    if (coll[k].a < 0 || coll[k].a >= n_species || coll[k].b < 0 || coll[k].b >= n_species)
      return MCC_ERR_INVALID;
  if (!std::isfinite(dt) || dt < 0.0 || !std::isfinite(lnL) || lnL < 0.0) return MCC_ERR_INVALID;
  if (p->method != MCC_TA77 && p->method != MCC_N97 && p->method != MCC_HARD_SPHERE)
    return MCC_ERR_INVALID;
  if (p->method == MCC_HARD_SPHERE)
    for (int k = 0; k < n_coll; ++k)
      if (!(coll[k].cross_section >= 0.0) || !std::isfinite(coll[k].cross_section))
        return MCC_ERR_INVALID;
  if (p->precision != MCC_FP64 && p->precision != MCC_FP32_KINEMATICS) return MCC_ERR_INVALID;
  if (p->on_failure != MCC_FAIL_RESET && p->on_failure != MCC_FAIL_KEEP) return MCC_ERR_INVALID;
  if (p->max_passes < 1) return MCC_ERR_INVALID;
  if (p->pairing != MCC_PAIRING_ORDER_N && p->pairing != MCC_PAIRING_NXN &&
      p->pairing != MCC_PAIRING_DUPLICITY)
    return MCC_ERR_INVALID;
  if (p->pairing != MCC_PAIRING_ORDER_N && p->diagnostics) return MCC_ERR_UNSUPPORTED;
  if (!(p->f_E > 0.0 && p->f_E < 1.0)) return MCC_ERR_INVALID;
  if (!(p->eps0 > 0.0) || !std::isfinite(p->eps0)) return MCC_ERR_INVALID;
  if (p->relativistic && !(p->c > 0.0 && std::isfinite(p->c))) return MCC_ERR_INVALID;
  if (p->relativistic && p->precision != MCC_FP64) return MCC_ERR_UNSUPPORTED;
  if (p->method == MCC_HARD_SPHERE && (p->relativistic || p->precision != MCC_FP64))
    return MCC_ERR_UNSUPPORTED;
  if (!cell_volume && !(dVs > 0.0 && std::isfinite(dVs))) return MCC_ERR_INVALID;
  return MCC_OK;
}

void fill_args(CollideArgs &A, int64_t n, int32_t n_cells, int32_t S, const int64_t *offsets,
               const double *w, double *vx, double *vy, double *vz, const double *cell_volume,
               double dVs, const mcc_species *sp, int32_t n_coll, const mcc_collision *coll,
               double dt, double lnL, uint64_t seed, uint64_t step, const mcc_params *p,
               mcc_stats *stats, int32_t *cell_corr, int32_t *err, const double2 *n97) {
  std::memset(&A, 0, sizeof(A));
  A.offsets = offsets;
  A.w = w;
  A.vx = vx;
  A.vy = vy;
  A.vz = vz;
  A.cell_volume = cell_volume;
  A.dV = dVs;
  A.n = n;
  A.n_cells = n_cells;
  A.S = S;
  A.n_coll = n_coll;
  A.method = p->method;
  A.corr = p->moment_correction ? 1 : 0;
  A.sortw = p->sort_by_weight ? 1 : 0;
  A.max_passes = p->max_passes;
  A.keep = p->on_failure == MCC_FAIL_KEEP ? 1 : 0;
  A.diag = (p->diagnostics && stats) ? 1 : 0;
  A.fE = p->f_E;
  A.c = p->relativistic ? p->c : 1.0;
  A.seed = seed;
  A.step = step;
  A.step_dev = nullptr;
  for (int s = 0; s < S; ++s) A.mass[s] = sp[s].mass;
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < n_coll; ++k) {
    const int a = coll[k].a, b = coll[k].b;
    const double ma = sp[a].mass, mb = sp[b].mass, qa = sp[a].charge, qb = sp[b].charge;
    const double mu = ma * mb / (ma + mb);
    CollConst &C = A.coll[k];
    C.a = a;
    C.b = b;
    // Eq. (12) without the per-pair factors f, w_max, N_min, dV and |u|^3;
    // for hard spheres s = sigma n_eff |u| dt without f, w_max, N_min, dV, |u|
    const double base = qa * qa * qb * qb * lnL * dt / (4.0 * pi * p->eps0 * p->eps0);
    C.coef = p->method == MCC_HARD_SPHERE ? coll[k].cross_section * dt
             : p->relativistic            ? base
                                          : base / (mu * mu);
    C.fa = mb / (ma + mb);
    C.fb = ma / (ma + mb);
  }
  A.stats = stats;
  A.cell_corr = cell_corr;
  A.err = err;
  A.n97 = n97;
}

bool ensure_lists(mcc_ctx *ctx, DevBuf &lists, DevBuf &counts, int32_t n_cells) {
  return lists.ensure(sizeof(int32_t) * (size_t)NBUCKET * (size_t)std::max(n_cells, 1)) &&
         counts.ensure(sizeof(uint32_t) * 16);
}

// global-layout variants: persistent grid and per-workgroup scratch
int grid_of(mcc_ctx *ctx, int mode, int v) {
  const Variant V = variant_of(mode, v);
  if (V.layout == 2) return ctx->n_cu;
  return ctx->grid[mode][v];
}

bool ensure_big(mcc_ctx *ctx, BigScratch &B, int mode, int v) {
  const Variant V = variant_of(mode, v);
  if (V.layout != 2) return true;
  const uint64_t stride = big_stride_bytes(V.cap, mode == MODE_TAN);
  if (V.cap > 4096) return B.big32k.ensure(stride * (uint64_t)ctx->n_cu);
  return B.big4k.ensure(stride * (uint64_t)ctx->n_cu);
}

void set_big_args(const BigScratch &B, CollideArgs &A, int mode, int v) {
  const Variant V = variant_of(mode, v);
  if (V.layout != 2) return;
  A.big_scratch = V.cap > 4096 ? B.big32k.as<char>() : B.big4k.as<char>();
  A.big_stride = big_stride_bytes(V.cap, mode == MODE_TAN);
}

#ifdef MCC_PHASE_TIMING
// profiling build: clock ticks per kernel phase, 16 counters per size bucket
unsigned long long *g_phase = nullptr;
#endif

// enqueue the collide kernel of one bucket, reading its device work list
mcc_status launch_bucket(mcc_ctx *ctx, BigScratch &big, const CollideArgs &base, int mode,
                         int32_t n_cells, const int32_t *lists, const uint32_t *counts, int b,
                         int v, hipStream_t stream) {
  const void *const *tab = kernel_table(mode);
  if (!ensure_big(ctx, big, mode, v)) return MCC_ERR_OOM;
  CollideArgs A = base;
#ifdef MCC_PHASE_TIMING
  A.phase = g_phase ? g_phase + 16 * b : nullptr;
#endif
  A.cell_list = lists + (int64_t)b * std::max(n_cells, 1);
  A.cell_count = counts + b;
  A.work = ctx->work.as<uint32_t>() + WORK_QUEUES * WORK_STRIDE * b;
  set_big_args(big, A, mode, v);
  void *kargs[] = {&A};
  HIP_TRY(hipLaunchKernel(tab[v], dim3(grid_of(ctx, mode, v)), dim3(variant_of(mode, v).tpc),
                          kargs, 0, stream));
  return MCC_OK;
}

constexpr int kSideBucket = 5, kBesideBucket = 4;
static_assert(kBucketCap[kSideBucket] == 4096 && kBucketCap[kBesideBucket] == 2048,
              "the branch pairs the 4096 and 2048 buckets");

// enqueue the collide kernels of all buckets, largest cells first
// (host_counts: the buckets' cell counts when known on the host; empty
// buckets are then not launched).  With br, the 4096 bucket runs on the
// branch, unless both kernels use global scratch (they would share the
// large-cell buffer).
mcc_status launch_buckets(mcc_ctx *ctx, BigScratch &big, const CollideArgs &base, int mode,
                          int32_t n_cells, const int32_t *lists, const uint32_t *counts,
                          const int *variant, hipStream_t stream,
                          const uint32_t *host_counts = nullptr, const Branch *br = nullptr) {
  auto pick = [&](int b) { return variant[b] >= 0 ? variant[b] : default_variant(mode, b); };
  const bool branch =
      br && (!host_counts || (host_counts[kSideBucket] > 0 && host_counts[kBesideBucket] > 0)) &&
      !(variant_of(mode, pick(kSideBucket)).layout == 2 &&
        variant_of(mode, pick(kBesideBucket)).layout == 2);
  if (branch) {
    HIP_TRY(hipEventRecord(br->fork, stream));
    HIP_TRY(hipStreamWaitEvent(br->side, br->fork, 0));
  }
  for (int b = NBUCKET - 1; b >= 0; --b) {
    if (host_counts && host_counts[b] == 0) continue;
    const mcc_status st = launch_bucket(ctx, big, base, mode, n_cells, lists, counts, b, pick(b),
                                        (branch && b == kSideBucket) ? br->side : stream);
    if (st != MCC_OK) return st;
    if (branch && b == kBesideBucket) {
      HIP_TRY(hipEventRecord(br->join, br->side));
      HIP_TRY(hipStreamWaitEvent(stream, br->join, 0));
    }
  }
  return MCC_OK;
}

mcc_status finish(mcc_ctx *ctx) {
  if (!ctx->validate) return MCC_OK;
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  int32_t code = 0;
  HIP_TRY(hipMemcpy(&code, ctx->err, sizeof(code), hipMemcpyDeviceToHost));
  return code ? MCC_ERR_DATA : MCC_OK;
}

}  // namespace

extern "C" {

#ifdef MCC_PHASE_TIMING
// profiling build only (not part of the public header): copy out and
// optionally clear the per-bucket phase counters
int mcc_debug_phase_read(unsigned long long *out, int reset) {
  if (!g_phase) return -1;
  if (hipDeviceSynchronize() != hipSuccess) return -3;
  const size_t bytes = sizeof(unsigned long long) * 16 * NBUCKET;
  if (hipMemcpy(out, g_phase, bytes, hipMemcpyDeviceToHost) != hipSuccess) return -3;
  if (reset && hipMemset(g_phase, 0, bytes) != hipSuccess) return -3;
  return 0;
}
#endif

void mcc_default_params(mcc_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->method = MCC_N97;
  p->precision = MCC_FP64;
  p->relativistic = 0;
  p->moment_correction = 1;
  p->sort_by_weight = 1;
  p->max_passes = 1;
  p->on_failure = MCC_FAIL_RESET;
  p->diagnostics = 0;
  p->pairing = MCC_PAIRING_ORDER_N;
  p->f_E = 0.05;
  p->eps0 = 1.0;
  p->c = 0.0;
}

const char *mcc_status_string(mcc_status s) {
  switch (s) {
    case MCC_OK: return "ok";
    case MCC_ERR_INVALID: return "invalid argument";
    case MCC_ERR_OOM: return "device out of memory";
    case MCC_ERR_DEVICE: return "HIP runtime error";
    case MCC_ERR_UNSUPPORTED: return "unsupported combination";
    case MCC_ERR_DATA: return "device-side data check failed";
  }
  return "unknown status";
}

// ---------------------------------------------------------------------------
// Fixed device scratch of the allocation-free step: the size-bucket counters
// (256 B) and the cell work lists of up to NOALLOC_MAX_CELLS cells.  Each
// device holds its own copy at its own address; host code reaches it only
// through the address hipGetSymbolAddress returns for that device.
// ---------------------------------------------------------------------------
constexpr int32_t NOALLOC_MAX_CELLS = 1 << 18;
constexpr size_t NOALLOC_BYTES = 256 + sizeof(int32_t) * (size_t)NBUCKET * NOALLOC_MAX_CELLS;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};
hipError_t g_noalloc_rc[NOALLOC_MAX_DEVICES] = {};
bool g_noalloc_done[NOALLOC_MAX_DEVICES] = {};

// once per device, with that device current
void noalloc_setup(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (g_noalloc_done[device]) return;
  void *p = nullptr;
  g_noalloc_rc[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_noalloc_ptr[device] = g_noalloc_rc[device] == hipSuccess ? p : nullptr;
  g_noalloc_done[device] = true;
}

void *noalloc_ptr(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  return g_noalloc_done[device] ? g_noalloc_ptr[device] : nullptr;
}
}  // namespace

mcc_status mcc_create(mcc_ctx **out, int device, void *hip_stream) {
  if (!out) return MCC_ERR_INVALID;
  *out = nullptr;
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return MCC_ERR_INVALID;
  HIP_TRY(hipSetDevice(device));
  mcc_ctx *ctx = new mcc_ctx();
  ctx->device = device;
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) {
    delete ctx;
    return from_hip(e);
  }
  ctx->n_cu = prop.multiProcessorCount;
  noalloc_setup(device);  // (the device is current)
  for (int b = 0; b < NBUCKET; ++b) ctx->variant[b] = -1;  // the mode's default
  const char *val = std::getenv("MCC_VALIDATE");
  ctx->validate = val && val[0] == '1';
  e = hipMalloc(&ctx->err, sizeof(int32_t));
  if (e == hipSuccess) e = hipMemset(ctx->err, 0, sizeof(int32_t));
  if (e == hipSuccess)
    e = ctx->n97.ensure(sizeof(double2) * N97_TABLE_SIZE) ? hipSuccess : hipErrorOutOfMemory;
  if (e == hipSuccess) e = launch_n97_table(ctx->n97.as<double2>(), nullptr);
  if (e == hipSuccess)
    e = ctx->work.ensure(sizeof(uint32_t) * WORK_QUEUES * WORK_STRIDE * NBUCKET)
            ? hipSuccess
            : hipErrorOutOfMemory;
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->branch.side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->branch.fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->branch.join, hipEventDisableTiming);
  if (e == hipSuccess)
    e = hipMemset(ctx->work.p, 0, sizeof(uint32_t) * WORK_QUEUES * WORK_STRIDE * NBUCKET);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    mcc_destroy(ctx);  // (releases what was created)
    return from_hip(e);
  }
#ifdef MCC_PHASE_TIMING
  if (!g_phase && hipMalloc(&g_phase, sizeof(unsigned long long) * 16 * NBUCKET) == hipSuccess)
    (void)hipMemset(g_phase, 0, sizeof(unsigned long long) * 16 * NBUCKET);
#endif
  for (int m = 0; m < NMODE; ++m) {
    const void *const *tab = kernel_table(m);
    for (int v = 0; v < NVARIANT; ++v) {
      int nb = 0;
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, tab[v], variant_of(m, v).tpc, 0);
      if (e != hipSuccess || nb < 1) nb = 1;
      ctx->grid[m][v] = nb * ctx->n_cu;
    }
  }
  *out = ctx;
  return MCC_OK;
}

mcc_status mcc_set_stream(mcc_ctx *ctx, void *hip_stream) {
  if (!ctx) return MCC_ERR_INVALID;
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return MCC_OK;
}

void mcc_destroy(mcc_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->big.release();
  for (DevBuf *b : {&ctx->lists, &ctx->counts, &ctx->tiles, &ctx->off, &ctx->perm,
                    &ctx->bin_k0, &ctx->bin_k1, &ctx->bin_v0, &ctx->bin_v1, &ctx->bin_hist,
                    &ctx->bin_pos, &ctx->gw, &ctx->gx, &ctx->gy, &ctx->gz, &ctx->rec, &ctx->n97,
                    &ctx->work, &ctx->rb, &ctx->adj_small, &ctx->adj_big,
                    &ctx->adj_part})
    b->release();
  if (ctx->err) (void)hipFree(ctx->err);
  if (ctx->branch.side) (void)hipStreamSynchronize(ctx->branch.side);
  if (ctx->branch.join) (void)hipEventDestroy(ctx->branch.join);
  if (ctx->branch.fork) (void)hipEventDestroy(ctx->branch.fork);
  if (ctx->branch.side) (void)hipStreamDestroy(ctx->branch.side);
  delete ctx;
}

mcc_status mcc_set_variant(mcc_ctx *ctx, int32_t bucket, int32_t variant) {
  if (!ctx || bucket < 0 || bucket >= NBUCKET || variant < -1 || variant >= NVARIANT)
    return MCC_ERR_INVALID;
  if (variant == -1) {
    ctx->variant[bucket] = -1;
    return MCC_OK;
  }
  if (kVariants[variant].cap < kBucketCap[bucket]) return MCC_ERR_INVALID;
  ctx->variant[bucket] = variant;
  return MCC_OK;
}

mcc_status mcc_sample_angles(mcc_ctx *ctx, int32_t method, int32_t precision, int64_t n,
                             const double *s, const uint32_t *a0, const uint32_t *a1, double *oc,
                             double *st, double *A) {
  if (!ctx || n < 0 || (method != MCC_TA77 && method != MCC_N97) ||
      (precision != MCC_FP64 && precision != MCC_FP32_KINEMATICS))
    return MCC_ERR_INVALID;
  if (n > 0 && (!s || !a0 || !a1 || !oc || !st)) return MCC_ERR_INVALID;
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(launch_sample_angles(method, precision, n, s, a0, a1, oc, st, A,
                               ctx->n97.as<double2>(), ctx->stream));
  return finish(ctx);
}

mcc_status mcc_device_error(mcc_ctx *ctx, int32_t *code) {
  if (!ctx || !code) return MCC_ERR_INVALID;
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  HIP_TRY(hipMemcpy(code, ctx->err, sizeof(int32_t), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemset(ctx->err, 0, sizeof(int32_t)));
  return MCC_OK;
}

mcc_status mcc_collide_sorted(mcc_ctx *ctx, int64_t n, int32_t n_cells, int32_t n_species,
                              const int64_t *offsets, const double *weights, double *vx,
                              double *vy, double *vz, const double *cell_volume,
                              double cell_volume_scalar, const mcc_species *species,
                              int32_t n_coll, const mcc_collision *coll, double dt,
                              double coulomb_log, uint64_t seed, uint64_t step,
                              const mcc_params *p, mcc_stats *stats, int32_t *cell_corr_pairs) {
  if (!ctx || !offsets) return MCC_ERR_INVALID;
  mcc_status st = check_step(n, n_cells, n_species, weights, vx, vy, vz, cell_volume,
                             cell_volume_scalar, species, n_coll, coll, dt, coulomb_log, p);
  if (st != MCC_OK) return st;
  HIP_TRY(hipSetDevice(ctx->device));
  if (!ensure_lists(ctx, ctx->lists, ctx->counts, n_cells)) return MCC_ERR_OOM;
  CollideArgs A;
  fill_args(A, n, n_cells, n_species, offsets, weights, vx, vy, vz, cell_volume,
            cell_volume_scalar, species, n_coll, coll, dt, coulomb_log, seed, step, p, stats,
            cell_corr_pairs, ctx->err, ctx->n97.as<double2>());
  hipStream_t s = ctx->stream;
  HIP_TRY(launch_fill_u32(ctx->counts.as<uint32_t>(), 0u, NBUCKET, s));
  if (stats) HIP_TRY(launch_zero_stats(stats, s));
  if (n_cells == 0) return finish(ctx);
  HIP_TRY(launch_check_weights(n, weights, ctx->err, s));
  HIP_TRY(launch_bucket_cells(offsets, n_cells, n_species, n, ctx->lists.as<int32_t>(),
                              ctx->counts.as<uint32_t>(), cell_corr_pairs, ctx->err, s));
  st = launch_buckets(ctx, ctx->big, A, mode_of(p, A), n_cells, ctx->lists.as<int32_t>(),
                      ctx->counts.as<uint32_t>(), ctx->variant, s, nullptr, &ctx->branch);
  if (st != MCC_OK) return st;
  return finish(ctx);
}

mcc_status mcc_collide_sorted_noalloc(mcc_ctx *ctx, int64_t n, int32_t n_cells,
                                      int32_t n_species, const int64_t *offsets,
                                      const double *weights, double *vx, double *vy, double *vz,
                                      const double *cell_volume, double cell_volume_scalar,
                                      const mcc_species *species, int32_t n_coll,
                                      const mcc_collision *coll, double dt, double coulomb_log,
                                      uint64_t seed, uint64_t step, const mcc_params *p,
                                      mcc_stats *stats, int32_t *cell_corr_pairs) {
  if (!ctx || !offsets) return MCC_ERR_INVALID;
  mcc_status st = check_step(n, n_cells, n_species, weights, vx, vy, vz, cell_volume,
                             cell_volume_scalar, species, n_coll, coll, dt, coulomb_log, p);
  if (st != MCC_OK) return st;
  if (n_cells > NOALLOC_MAX_CELLS) return MCC_ERR_INVALID;
  if (p->relativistic) return MCC_ERR_UNSUPPORTED;
  HIP_TRY(hipSetDevice(ctx->device));
  char *base = static_cast<char *>(noalloc_ptr(ctx->device));
  if (!base) return MCC_ERR_DEVICE;
  uint32_t *counts = reinterpret_cast<uint32_t *>(base);
  int32_t *lists = reinterpret_cast<int32_t *>(base + 256);
  CollideArgs A;
  fill_args(A, n, n_cells, n_species, offsets, weights, vx, vy, vz, cell_volume,
            cell_volume_scalar, species, n_coll, coll, dt, coulomb_log, seed, step, p, stats,
            cell_corr_pairs, ctx->err, ctx->n97.as<double2>());
  const int mode = mode_of(p, A);
  hipStream_t s = ctx->stream;
  HIP_TRY(launch_fill_u32(counts, 0u, NBUCKET, s));
  if (stats) HIP_TRY(launch_zero_stats(stats, s));
  if (n_cells == 0) return finish(ctx);
  HIP_TRY(launch_check_weights(n, weights, ctx->err, s));
  HIP_TRY(launch_bucket_cells(offsets, n_cells, n_species, n, lists, counts, cell_corr_pairs,
                              ctx->err, s));
  // cells above 4096 particles need the global-scratch kernels: not stepped
  HIP_TRY(launch_flag_nonzero(counts + (NBUCKET - 1), 2, ctx->err, s));
  BigScratch none;  // (the variants below never use it)
  for (int b = NBUCKET - 2; b >= 0; --b) {
    int v = ctx->variant[b] >= 0 ? ctx->variant[b] : default_variant(mode, b);
    if (variant_of(mode, v).layout == 2) v = default_variant(mode, b);
    if (variant_of(mode, v).layout == 2) return MCC_ERR_UNSUPPORTED;
    st = launch_bucket(ctx, none, A, mode, n_cells, lists, counts, b, v, s);
    if (st != MCC_OK) return st;
  }
  return finish(ctx);
}

mcc_status mcc_collide_sorted_jvp(mcc_ctx *ctx, int64_t n, int32_t n_cells, int32_t n_species,
                                  const int64_t *offsets, const double *weights, double *vx,
                                  double *vy, double *vz, double *tx, double *ty, double *tz,
                                  const double *cell_volume, double cell_volume_scalar,
                                  const mcc_species *species, int32_t n_coll,
                                  const mcc_collision *coll, double dt, double coulomb_log,
                                  double coulomb_log_tangent, uint64_t seed, uint64_t step,
                                  const mcc_params *p, int32_t update_primal,
                                  mcc_stats *stats) {
  if (!ctx || !offsets) return MCC_ERR_INVALID;
  mcc_status st = check_step(n, n_cells, n_species, weights, vx, vy, vz, cell_volume,
                             cell_volume_scalar, species, n_coll, coll, dt, coulomb_log, p);
  if (st != MCC_OK) return st;
  if (n > 0 && (!tx || !ty || !tz)) return MCC_ERR_INVALID;
  if (!std::isfinite(coulomb_log_tangent)) return MCC_ERR_INVALID;
  if (coulomb_log_tangent != 0.0 && !(coulomb_log > 0.0)) return MCC_ERR_INVALID;
  if (p->relativistic || p->precision != MCC_FP64 || p->pairing != MCC_PAIRING_ORDER_N ||
      p->method == MCC_HARD_SPHERE)
    return MCC_ERR_UNSUPPORTED;
  HIP_TRY(hipSetDevice(ctx->device));
  if (!ensure_lists(ctx, ctx->lists, ctx->counts, n_cells)) return MCC_ERR_OOM;
  CollideArgs A;
  mcc_params q = *p;
  q.diagnostics = 0;
  fill_args(A, n, n_cells, n_species, offsets, weights, vx, vy, vz, cell_volume,
            cell_volume_scalar, species, n_coll, coll, dt, coulomb_log, seed, step, &q, stats,
            nullptr, ctx->err, ctx->n97.as<double2>());
  A.tx = tx;
  A.ty = ty;
  A.tz = tz;
  A.dlnl = coulomb_log_tangent != 0.0 ? coulomb_log_tangent / coulomb_log : 0.0;
  A.write_primal = update_primal ? 1 : 0;
  hipStream_t s = ctx->stream;
  HIP_TRY(launch_check_weights(n, weights, ctx->err, s));
  HIP_TRY(launch_fill_u32(ctx->counts.as<uint32_t>(), 0u, NBUCKET, s));
  if (stats) HIP_TRY(launch_zero_stats(stats, s));
  if (n_cells == 0) return finish(ctx);
  HIP_TRY(launch_bucket_cells(offsets, n_cells, n_species, n, ctx->lists.as<int32_t>(),
                              ctx->counts.as<uint32_t>(), nullptr, ctx->err, s));
  st = launch_buckets(ctx, ctx->big, A, MODE_TAN, n_cells, ctx->lists.as<int32_t>(),
                      ctx->counts.as<uint32_t>(), ctx->variant, s);
  if (st != MCC_OK) return st;
  return finish(ctx);
}

mcc_status mcc_collide_adjoint(mcc_ctx *ctx, int64_t n, int32_t n_cells, int32_t n_species,
                               const int64_t *offsets, const double *weights, const double *vx,
                               const double *vy, const double *vz, double *gx, double *gy,
                               double *gz, const double *cell_volume,
                               double cell_volume_scalar, const mcc_species *species,
                               int32_t n_coll, const mcc_collision *coll, double dt,
                               double coulomb_log, uint64_t seed, uint64_t step,
                               const mcc_params *p, double *g_coulomb_log) {
  if (!ctx || !offsets) return MCC_ERR_INVALID;
  mcc_status st = check_step(n, n_cells, n_species, weights, vx, vy, vz, cell_volume,
                             cell_volume_scalar, species, n_coll, coll, dt, coulomb_log, p);
  if (st != MCC_OK) return st;
  if (n > 0 && (!gx || !gy || !gz)) return MCC_ERR_INVALID;
  if (p->relativistic || p->pairing != MCC_PAIRING_ORDER_N || p->method == MCC_HARD_SPHERE ||
      p->max_passes != 1)
    return MCC_ERR_UNSUPPORTED;
  HIP_TRY(hipSetDevice(ctx->device));
  if (!ensure_lists(ctx, ctx->lists, ctx->counts, n_cells) ||
      !ctx->adj_part.ensure(sizeof(double) * (size_t)std::max(n_cells, 1)))
    return MCC_ERR_OOM;
  CollideArgs F;
  fill_args(F, n, n_cells, n_species, offsets, weights, const_cast<double *>(vx),
            const_cast<double *>(vy), const_cast<double *>(vz), cell_volume, cell_volume_scalar,
            species, n_coll, coll, dt, coulomb_log, seed, step, p, nullptr, nullptr, ctx->err,
            ctx->n97.as<double2>());
  AdjointArgs A;
  std::memset(&A, 0, sizeof(A));
  A.offsets = offsets;
  A.w = weights;
  A.vx = vx;
  A.vy = vy;
  A.vz = vz;
  A.gx = gx;
  A.gy = gy;
  A.gz = gz;
  A.cell_volume = cell_volume;
  A.dV = cell_volume_scalar;
  A.n = n;
  A.n_cells = n_cells;
  A.S = n_species;
  A.n_coll = n_coll;
  A.method = p->method;
  A.corr = F.corr;
  A.sortw = F.sortw;
  A.keep = F.keep;
  A.fE = F.fE;
  A.inv_lnl = coulomb_log > 0.0 ? 1.0 / coulomb_log : 0.0;
  A.seed = seed;
  A.step = step;
  for (int s = 0; s < n_species; ++s) A.mass[s] = F.mass[s];
  for (int k = 0; k < n_coll; ++k) A.coll[k] = F.coll[k];
  A.lnl_part = ctx->adj_part.as<double>();
  A.err = ctx->err;
  A.n97 = ctx->n97.as<double2>();
  hipStream_t s = ctx->stream;
  HIP_TRY(launch_check_weights(n, weights, ctx->err, s));
  HIP_TRY(launch_fill_u32(ctx->counts.as<uint32_t>(), 0u, NBUCKET, s));
  HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->adj_part.p), 0u,
                          2 * (int64_t)std::max(n_cells, 1), s));
  if (n_cells > 0) {
    HIP_TRY(launch_bucket_cells(offsets, n_cells, n_species, n, ctx->lists.as<int32_t>(),
                                ctx->counts.as<uint32_t>(), nullptr, ctx->err, s));
    // the cell counts per size bucket size the scratch (one wait on the stream)
    uint32_t hc[NBUCKET];
    HIP_TRY(hipMemcpyAsync(hc, ctx->counts.p, sizeof(hc), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int b = 0; b < NBUCKET; ++b) {
      if (hc[b] == 0) continue;
      // threads per cell of the forward-mode variant of the bucket, so the
      // per-cell sums (and the choices they decide) round as there
      const int v = ctx->variant[b] >= 0 ? ctx->variant[b] : default_variant(MODE_TAN, b);
      const Variant V = variant_of(MODE_TAN, v);
      const bool big = kBucketCap[b] > 4096;
      const int tpc = big ? 64 : V.tpc;
      const int cap = big ? MCC_MAX_CELL : 4096;
      const int grid = (int)std::min<uint32_t>(hc[b], (uint32_t)(big ? ctx->n_cu : ctx->n_cu * 2));
      DevBuf &buf = big ? ctx->adj_big : ctx->adj_small;
      A.stride = adj_stride_bytes(cap);
      if (!buf.ensure(A.stride * (uint64_t)grid)) return MCC_ERR_OOM;
      A.scratch = buf.as<char>();
      HIP_TRY(launch_adjoint(A, p->precision == MCC_FP32_KINEMATICS, ctx->lists.as<int32_t>(),
                             ctx->counts.as<uint32_t>(), n_cells, b, tpc, cap, grid, s));
    }
  }
  if (g_coulomb_log)
    HIP_TRY(launch_sum_f64(ctx->adj_part.as<double>(), n_cells, g_coulomb_log, s));
  return finish(ctx);
}

static mcc_status bin_into(mcc_ctx *ctx, int64_t n, const int32_t *cells,
                           const int32_t *species_id, int32_t n_cells, int32_t n_species,
                           int64_t *offsets, int32_t *perm) {
  const size_t nn = (size_t)std::max<int64_t>(n, 1);
  const int64_t hb = bin_hist_entries(n);  // digit histograms of the tiles
  if (!ctx->bin_k0.ensure(4 * nn) || !ctx->bin_k1.ensure(4 * nn) ||
      !ctx->bin_v0.ensure(4 * nn) || !ctx->bin_v1.ensure(4 * nn) ||
      !ctx->bin_hist.ensure(sizeof(uint32_t) * (size_t)hb) ||
      !ctx->bin_pos.ensure(sizeof(int64_t) * (size_t)(hb + 1)) ||
      !ctx->tiles.ensure(sizeof(int64_t) * (size_t)scan_tiles_needed(hb)))
    return MCC_ERR_OOM;
  return from_hip(launch_bin(n, cells, species_id, n_cells, n_species,
                             ctx->bin_k0.as<uint32_t>(), ctx->bin_k1.as<uint32_t>(),
                             ctx->bin_v0.as<int32_t>(), ctx->bin_v1.as<int32_t>(),
                             ctx->bin_hist.as<uint32_t>(), ctx->bin_pos.as<int64_t>(),
                             ctx->tiles.as<int64_t>(), offsets, perm, ctx->err, ctx->stream));
}

mcc_status mcc_bin(mcc_ctx *ctx, int64_t n, const int32_t *cells, const int32_t *species_id,
                   int32_t n_cells, int32_t n_species, int64_t *offsets_out, int32_t *perm_out) {
  if (!ctx || n < 0 || n_cells < 0 || n_species < 1 || n_species > MCC_MAX_SPECIES ||
      !offsets_out || (n > 0 && (!cells || !species_id || !perm_out)))
    return MCC_ERR_INVALID;
  if (n > (int64_t)INT32_MAX || (int64_t)n_cells * n_species > (int64_t)INT32_MAX)
    return MCC_ERR_UNSUPPORTED;
  HIP_TRY(hipSetDevice(ctx->device));
  mcc_status st = bin_into(ctx, n, cells, species_id, n_cells, n_species, offsets_out, perm_out);
  if (st != MCC_OK) return st;
  return finish(ctx);
}

namespace {
// the regrouping of mcc_rebin and mcc_rebin_out: offsets_out and perm_out
mcc_status rebin_keys(mcc_ctx *ctx, int64_t n, int32_t n_cells, int32_t n_species,
                      const int64_t *offsets, const int32_t *cells_new, int64_t *offsets_out,
                      int32_t *perm_out) {
  if (!ctx || n < 0 || n_cells < 0 || n_species < 1 || n_species > MCC_MAX_SPECIES ||
      !offsets || !offsets_out || (n > 0 && (!cells_new || !perm_out)))
    return MCC_ERR_INVALID;
  const int64_t m = (int64_t)n_cells * n_species;
  if (n > (int64_t)INT32_MAX || m > (int64_t)INT32_MAX) return MCC_ERR_UNSUPPORTED;
  if (m == 0 && n > 0) return MCC_ERR_INVALID;
  HIP_TRY(hipSetDevice(ctx->device));
  if (!ctx->rb.ensure(rebin_scratch_bytes(n, m)) ||
      !ctx->tiles.ensure(sizeof(int64_t) * (size_t)rebin_tiles_needed(n, m)))
    return MCC_ERR_OOM;
  if (m == 0) {
    HIP_TRY(launch_set_u64(reinterpret_cast<uint64_t *>(offsets_out), 0ull, ctx->stream));
    return MCC_OK;
  }
  HIP_TRY(launch_rebin(n, m, n_species, n_cells, offsets, cells_new, offsets_out, perm_out,
                       ctx->rb.p, ctx->tiles.as<int64_t>(), ctx->err, ctx->stream));
  return MCC_OK;
}
}  // namespace

mcc_status mcc_rebin(mcc_ctx *ctx, int64_t n, int32_t n_cells, int32_t n_species,
                     const int64_t *offsets, const int32_t *cells_new, int64_t *offsets_out,
                     int32_t *perm_out, double *weights, double *vx, double *vy, double *vz) {
  const int any = (weights != nullptr) + (vx != nullptr) + (vy != nullptr) + (vz != nullptr);
  if (any != 0 && any != 4) return MCC_ERR_INVALID;
  const mcc_status st =
      rebin_keys(ctx, n, n_cells, n_species, offsets, cells_new, offsets_out, perm_out);
  if (st != MCC_OK) return st;
  const size_t nn = (size_t)std::max<int64_t>(n, 1);
  if (any && n > 0 && (int64_t)n_cells * n_species > 0) {
    if (!ctx->gw.ensure(sizeof(double) * nn) || !ctx->gx.ensure(sizeof(double) * nn) ||
        !ctx->gy.ensure(sizeof(double) * nn) || !ctx->gz.ensure(sizeof(double) * nn))
      return MCC_ERR_OOM;
    HIP_TRY(launch_gather(n, perm_out, weights, vx, vy, vz, ctx->gw.as<double>(),
                          ctx->gx.as<double>(), ctx->gy.as<double>(), ctx->gz.as<double>(),
                          ctx->stream));
    const size_t b = sizeof(double) * (size_t)n;
    HIP_TRY(hipMemcpyAsync(weights, ctx->gw.p, b, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(vx, ctx->gx.p, b, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(vy, ctx->gy.p, b, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(vz, ctx->gz.p, b, hipMemcpyDeviceToDevice, ctx->stream));
  }
  return finish(ctx);
}

mcc_status mcc_rebin_out(mcc_ctx *ctx, int64_t n, int32_t n_cells, int32_t n_species,
                         const int64_t *offsets, const int32_t *cells_new, int64_t *offsets_out,
                         int32_t *perm_out, const double *weights, const double *vx,
                         const double *vy, const double *vz, double *weights_out,
                         double *vx_out, double *vy_out, double *vz_out) {
  if (n > 0 && (!weights || !vx || !vy || !vz || !weights_out || !vx_out || !vy_out || !vz_out))
    return MCC_ERR_INVALID;
  const double *in[4] = {weights, vx, vy, vz};
  const double *out[4] = {weights_out, vx_out, vy_out, vz_out};
  for (int i = 0; i < 4 && n > 0; ++i)
    for (int j = 0; j < 4; ++j)
      if (in[i] == out[j]) return MCC_ERR_INVALID;  // a gather cannot run in place
  const mcc_status st =
      rebin_keys(ctx, n, n_cells, n_species, offsets, cells_new, offsets_out, perm_out);
  if (st != MCC_OK) return st;
  if (n > 0 && (int64_t)n_cells * n_species > 0)
    HIP_TRY(launch_gather(n, perm_out, weights, vx, vy, vz, weights_out, vx_out, vy_out, vz_out,
                          ctx->stream));
  return finish(ctx);
}

mcc_status mcc_collide(mcc_ctx *ctx, int64_t n, const int32_t *cells, const int32_t *species_id,
                       int32_t n_cells, int32_t n_species, const double *weights, double *vx,
                       double *vy, double *vz, const double *cell_volume,
                       double cell_volume_scalar, const mcc_species *species, int32_t n_coll,
                       const mcc_collision *coll, double dt, double coulomb_log, uint64_t seed,
                       uint64_t step, const mcc_params *p, mcc_stats *stats,
                       int32_t *cell_corr_pairs) {
  if (!ctx || (n > 0 && (!cells || !species_id))) return MCC_ERR_INVALID;
  mcc_status st = check_step(n, n_cells, n_species, weights, vx, vy, vz, cell_volume,
                             cell_volume_scalar, species, n_coll, coll, dt, coulomb_log, p);
  if (st != MCC_OK) return st;
  HIP_TRY(hipSetDevice(ctx->device));
  const int64_t m = (int64_t)n_cells * n_species;
  if (m > (int64_t)INT32_MAX) return MCC_ERR_UNSUPPORTED;
  const size_t nn = (size_t)std::max<int64_t>(n, 1);
  if (!ctx->off.ensure(sizeof(int64_t) * (size_t)(m + 1)) ||
      !ctx->perm.ensure(sizeof(int32_t) * nn) || !ctx->gw.ensure(sizeof(double) * nn) ||
      !ctx->gx.ensure(sizeof(double) * nn) || !ctx->gy.ensure(sizeof(double) * nn) ||
      !ctx->gz.ensure(sizeof(double) * nn) || !ctx->rec.ensure(32 * nn))
    return MCC_ERR_OOM;
  st = bin_into(ctx, n, cells, species_id, n_cells, n_species, ctx->off.as<int64_t>(),
                ctx->perm.as<int32_t>());
  if (st != MCC_OK) return st;
  HIP_TRY(launch_gather_rec(n, ctx->perm.as<int32_t>(), weights, vx, vy, vz, ctx->rec.p,
                            ctx->gw.as<double>(), ctx->gx.as<double>(), ctx->gy.as<double>(),
                            ctx->gz.as<double>(), ctx->stream));
  const bool v = ctx->validate;
  ctx->validate = false;
  st = mcc_collide_sorted(ctx, n, n_cells, n_species, ctx->off.as<int64_t>(),
                          ctx->gw.as<double>(), ctx->gx.as<double>(), ctx->gy.as<double>(),
                          ctx->gz.as<double>(), cell_volume, cell_volume_scalar, species, n_coll,
                          coll, dt, coulomb_log, seed, step, p, stats, cell_corr_pairs);
  ctx->validate = v;
  if (st != MCC_OK) return st;
  HIP_TRY(launch_scatter_back_rec(n, ctx->perm.as<int32_t>(), ctx->gw.as<double>(),
                                  ctx->gx.as<double>(), ctx->gy.as<double>(),
                                  ctx->gz.as<double>(), ctx->rec.p, vx, vy, vz, ctx->stream));
  return finish(ctx);
}

// ---------------------------------------------------------------------------
// Batched plan
// ---------------------------------------------------------------------------
// One step into the graph being captured on s (the branch of
// launch_buckets on the capture's side stream and events)
static mcc_status plan_enqueue_step(mcc_plan *pl, hipStream_t s, const Branch &br) {
  // counters are reset by kernels (no memset nodes in the graph)
  if (pl->stats) HIP_TRY(launch_zero_stats(pl->stats, s));
  const mcc_status st =
      launch_buckets(pl->ctx, pl->big, pl->args, pl->mode, pl->n_cells, pl->lists.as<int32_t>(),
                     pl->counts.as<uint32_t>(), pl->variant, s, pl->hcount, &br);
  if (st != MCC_OK) return st;
  HIP_TRY(launch_inc_u64(pl->step.as<uint64_t>(), s));
  return MCC_OK;
}

// A plan's bucket work lists, largest cell first (ties by cell index), once
// at plan creation.  A persistent bucket kernel claims its cells in list
// order, so the last cells claimed are then the smallest and the grid drains
// evenly.  Cells are independent (their random numbers are keyed by cell),
// so the order changes no result.
static hipError_t order_largest_first(mcc_plan *pl, const int64_t *offsets, int32_t n_cells,
                                      int32_t S) {
  std::vector<int64_t> off((size_t)n_cells * S + 1);
  hipError_t e = hipMemcpy(off.data(), offsets, sizeof(int64_t) * off.size(),
                           hipMemcpyDeviceToHost);
  std::vector<int32_t> list;
  for (int b = 0; b < NBUCKET && e == hipSuccess; ++b) {
    const uint32_t k = pl->hcount[b];
    if (k < 2) continue;
    int32_t *dl = pl->lists.as<int32_t>() + (int64_t)b * n_cells;
    list.resize(k);
    e = hipMemcpy(list.data(), dl, sizeof(int32_t) * k, hipMemcpyDeviceToHost);
    if (e != hipSuccess) break;
    auto size = [&](int32_t c) {
      return off[(size_t)(c + 1) * S] - off[(size_t)c * S];
    };
    std::sort(list.begin(), list.end(), [&](int32_t x, int32_t y) {
      const int64_t sx = size(x), sy = size(y);
      return sx > sy || (sx == sy && x < y);
    });
    e = hipMemcpy(dl, list.data(), sizeof(int32_t) * k, hipMemcpyHostToDevice);
  }
  return e;
}

mcc_status mcc_plan_create(mcc_ctx *ctx, mcc_plan **plan, int64_t n, int32_t n_cells,
                           int32_t n_species, const int64_t *offsets, const double *weights,
                           double *vx, double *vy, double *vz, const double *cell_volume,
                           double cell_volume_scalar, const mcc_species *species, int32_t n_coll,
                           const mcc_collision *coll, double dt, double coulomb_log, uint64_t seed,
                           const mcc_params *p, mcc_stats *stats, int32_t *cell_corr_pairs,
                           int32_t autotune) {
  if (!ctx || !plan || !offsets) return MCC_ERR_INVALID;
  *plan = nullptr;
  mcc_status st = check_step(n, n_cells, n_species, weights, vx, vy, vz, cell_volume,
                             cell_volume_scalar, species, n_coll, coll, dt, coulomb_log, p);
  if (st != MCC_OK) return st;
  HIP_TRY(hipSetDevice(ctx->device));
  mcc_plan *pl = new mcc_plan();
  pl->ctx = ctx;
  pl->n_cells = n_cells;
  pl->stats = stats;
  pl->cell_corr = cell_corr_pairs;
  for (int b = 0; b < NBUCKET; ++b) pl->variant[b] = -1;
  if (!ensure_lists(ctx, pl->lists, pl->counts, n_cells) || !pl->step.ensure(64)) {
    mcc_plan_destroy(pl);
    return MCC_ERR_OOM;
  }
  fill_args(pl->args, n, n_cells, n_species, offsets, weights, vx, vy, vz, cell_volume,
            cell_volume_scalar, species, n_coll, coll, dt, coulomb_log, seed, 0, p, stats,
            cell_corr_pairs, ctx->err, ctx->n97.as<double2>());
  pl->mode = mode_of(p, pl->args);
  for (int b = 0; b < NBUCKET; ++b) pl->variant[b] = default_variant(pl->mode, b);
  pl->args.step_dev = pl->step.as<uint64_t>();
  hipStream_t s = ctx->stream;
  // device work lists, built once (offsets are fixed for the plan)
  hipError_t e = launch_fill_u32(pl->counts.as<uint32_t>(), 0u, NBUCKET, s);
  if (e == hipSuccess && n_cells > 0)
    e = launch_bucket_cells(offsets, n_cells, n_species, n, pl->lists.as<int32_t>(),
                            pl->counts.as<uint32_t>(), cell_corr_pairs, ctx->err, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess)
    e = hipMemcpy(pl->hcount, pl->counts.p, sizeof(pl->hcount), hipMemcpyDeviceToHost);
  if (e == hipSuccess && n_cells > 0) e = order_largest_first(pl, offsets, n_cells, n_species);
  if (e != hipSuccess) {
    mcc_plan_destroy(pl);
    return from_hip(e);
  }
  if (autotune && n_cells > 0) {
    // time every candidate variant of every non-empty bucket on this
    // population; the trial steps use a scratch copy of the velocities so the
    // caller's state is untouched
    uint32_t hcounts[NBUCKET];
    e = hipMemcpy(hcounts, pl->counts.p, sizeof(hcounts), hipMemcpyDeviceToHost);
    DevBuf tv;
    const size_t nb = sizeof(double) * (size_t)std::max<int64_t>(n, 1);
    if (e != hipSuccess || !tv.ensure(3 * nb)) {
      mcc_plan_destroy(pl);
      return e != hipSuccess ? from_hip(e) : MCC_ERR_OOM;
    }
    CollideArgs T = pl->args;
    T.vx = tv.as<double>();
    T.vy = T.vx + std::max<int64_t>(n, 1);
    T.vz = T.vy + std::max<int64_t>(n, 1);
    T.stats = nullptr;
    T.cell_corr = nullptr;
    T.step_dev = nullptr;
    T.step = 0x7FFFFFFFull;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const void *const *tab = kernel_table(pl->mode);
    for (int b = 0; b < NBUCKET && e == hipSuccess; ++b) {
      if (hcounts[b] == 0) continue;
      double best = 1e300;
      for (int ci = 0; ci < 5 && kCandidates[b][ci] >= 0; ++ci) {
        const int v = kCandidates[b][ci];
        if (!ensure_big(ctx, pl->big, pl->mode, v)) continue;
        CollideArgs A = T;
        A.cell_list = pl->lists.as<int32_t>() + (int64_t)b * std::max(n_cells, 1);
        A.cell_count = pl->counts.as<uint32_t>() + b;
        A.work = ctx->work.as<uint32_t>() + WORK_QUEUES * WORK_STRIDE * b;
        set_big_args(pl->big, A, pl->mode, v);
        void *kargs[] = {&A};
        float ms_best = 1e30f;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
          e = hipMemcpyAsync(T.vx, vx, nb, hipMemcpyDeviceToDevice, s);
          if (e == hipSuccess) e = hipMemcpyAsync(T.vy, vy, nb, hipMemcpyDeviceToDevice, s);
          if (e == hipSuccess) e = hipMemcpyAsync(T.vz, vz, nb, hipMemcpyDeviceToDevice, s);
          if (e == hipSuccess) e = hipEventRecord(e0, s);
          if (e == hipSuccess)
            e = hipLaunchKernel(tab[v], dim3(grid_of(ctx, pl->mode, v)),
                                dim3(variant_of(pl->mode, v).tpc), kargs, 0, s);
          if (e == hipSuccess) e = hipEventRecord(e1, s);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          float ms = 0.f;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
          if (rep > 0) ms_best = std::min(ms_best, ms);  // first run warms up
        }
        pl->tuned_ms[b][v] = ms_best;
        if (ms_best < best) {
          best = ms_best;
          pl->variant[b] = v;
        }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    tv.release();
    if (e != hipSuccess) {
      mcc_plan_destroy(pl);
      return from_hip(e);
    }
  }
  // workspace of every chosen variant exists before capture (no allocation
  // while capturing)
  for (int b = 0; b < NBUCKET; ++b)
    if (!ensure_big(ctx, pl->big, pl->mode, pl->variant[b])) {
      mcc_plan_destroy(pl);
      return MCC_ERR_OOM;
    }
  // the weights are bound to the plan: checked once here (positive and
  // finite; a violation is latched as data error 4) and never again per step
  e = launch_check_weights(n, weights, ctx->err, s);
  if (e != hipSuccess) {
    mcc_plan_destroy(pl);
    return from_hip(e);
  }
  // the weights are bound to the plan: their per-(cell, species) sums, range
  // and class, and the descending-weight order, are computed once here (with
  // the chosen variants, so the sums round as in a step) and read by every
  // step
  if (p->moment_correction && n_cells > 0) {
    if (!pl->prep.ensure(sizeof(SpeciesPrep) * (size_t)n_cells * n_species) ||
        // (+4: the kernel reads a cell's entries in whole dwords)
        !pl->prep_word.ensure(sizeof(uint16_t) * (size_t)(std::max<int64_t>(n, 1) + 4))) {
      mcc_plan_destroy(pl);
      return MCC_ERR_OOM;
    }
    CollideArgs W = pl->args;
    W.prep_mode = PREP_WRITE;
    W.n_coll = 0;  // weight data only: no collision is applied (velocities unchanged)
    W.prep = pl->prep.as<SpeciesPrep>();
    W.prep_word = pl->prep_word.as<uint16_t>();
    W.stats = nullptr;
    W.cell_corr = nullptr;
    st = launch_buckets(ctx, pl->big, W, pl->mode, n_cells, pl->lists.as<int32_t>(),
                        pl->counts.as<uint32_t>(), pl->variant, s, pl->hcount);
    if (st == MCC_OK) st = from_hip(hipStreamSynchronize(s));
    if (st != MCC_OK) {
      mcc_plan_destroy(pl);
      return st;
    }
    pl->args.prep_mode = PREP_READ;
    pl->args.prep = W.prep;
    pl->args.prep_word = W.prep_word;
  }
  // capture one step into a graph: stats reset, bucket kernels, step += 1
  // (default-priority streams; the side stream only carries a branch)
  hipStream_t cs = nullptr;
  Branch br;
  e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&br.side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&br.fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&br.join, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    st = plan_enqueue_step(pl, cs, br);
    hipError_t e2 = hipStreamEndCapture(cs, &pl->graph);
    if (st == MCC_OK && e2 != hipSuccess) st = from_hip(e2);
    if (st == MCC_OK) e = hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0);
  }
  if (br.join) (void)hipEventDestroy(br.join);
  if (br.fork) (void)hipEventDestroy(br.fork);
  if (br.side) (void)hipStreamDestroy(br.side);
  if (cs) (void)hipStreamDestroy(cs);
  if (e != hipSuccess || st != MCC_OK) {
    mcc_plan_destroy(pl);
    return st != MCC_OK ? st : from_hip(e);
  }
  *plan = pl;
  return MCC_OK;
}

mcc_status mcc_plan_run(mcc_plan *pl, uint64_t first_step, int32_t n_steps) {
  if (!pl || n_steps < 0) return MCC_ERR_INVALID;
  HIP_TRY(hipSetDevice(pl->ctx->device));
  hipStream_t s = pl->ctx->stream;
  HIP_TRY(launch_set_u64(pl->step.as<uint64_t>(), first_step, s));
  for (int i = 0; i < n_steps; ++i) HIP_TRY(hipGraphLaunch(pl->exec, s));
  return finish(pl->ctx);
}

mcc_status mcc_plan_run_bucket(mcc_plan *pl, int32_t bucket, uint64_t step) {
  if (!pl || bucket < 0 || bucket >= NBUCKET) return MCC_ERR_INVALID;
  HIP_TRY(hipSetDevice(pl->ctx->device));
  CollideArgs A = pl->args;
  A.step_dev = nullptr;
  A.step = step;
  const mcc_status st = launch_bucket(pl->ctx, pl->big, A, pl->mode, pl->n_cells, pl->lists.as<int32_t>(),
                                      pl->counts.as<uint32_t>(), bucket, pl->variant[bucket],
                                      pl->ctx->stream);
  if (st != MCC_OK) return st;
  return finish(pl->ctx);
}

mcc_status mcc_plan_describe(mcc_plan *pl, char *buf, size_t len) {
  if (!pl || !buf || len == 0) return MCC_ERR_INVALID;
  uint32_t hc[NBUCKET] = {};
  HIP_TRY(hipStreamSynchronize(pl->ctx->stream));
  HIP_TRY(hipMemcpy(hc, pl->counts.p, sizeof(hc), hipMemcpyDeviceToHost));
  std::string out = "{\"buckets\": [";
  for (int b = 0; b < NBUCKET; ++b) {
    const Variant V = variant_of(pl->mode, pl->variant[b]);
    char tmp[512];
    std::snprintf(tmp, sizeof(tmp),
                  "%s{\"max_cell\": %d, \"cells\": %u, \"tpc\": %d, \"cap\": %d, \"layout\": %d, "
                  "\"grid\": %d, \"timed_ms\": {",
                  b ? ", " : "", kBucketCap[b], hc[b], V.tpc, V.cap, V.layout,
                  grid_of(pl->ctx, pl->mode, pl->variant[b]));
    out += tmp;
    bool first = true;
    for (int u = 0; u < NVARIANT; ++u) {
      if (pl->tuned_ms[b][u] <= 0.0) continue;
      const Variant U = variant_of(pl->mode, u);
      std::snprintf(tmp, sizeof(tmp), "%s\"%dx%d\": %.4f", first ? "" : ", ", U.tpc, U.cap,
                    pl->tuned_ms[b][u]);
      out += tmp;
      first = false;
    }
    out += "}}";
  }
  out += "]}";
  std::snprintf(buf, len, "%s", out.c_str());
  return MCC_OK;
}

void mcc_plan_destroy(mcc_plan *pl) {
  if (!pl) return;
  (void)hipSetDevice(pl->ctx->device);
  (void)hipStreamSynchronize(pl->ctx->stream);
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  pl->lists.release();
  pl->counts.release();
  pl->step.release();
  pl->prep.release();
  pl->prep_word.release();
  pl->big.release();
  delete pl;
}

}  // extern "C"
