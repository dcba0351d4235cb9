// mcc_variants.hpp -- kernel variants (threads per cell, cell capacity) and
// the cell-size buckets they serve.  Shared by the host runtime and the
// instantiation units.
#pragma once

namespace mcc {

// precision / physics modes compiled
// MODE_TAN: FP64 step carrying the tangent of the velocities (forward mode);
// the *_DIAG modes also measure the residual momentum and energy (separate
// kernels, so the step without diagnostics carries none of their registers)
enum Mode {
  MODE_FP64 = 0,
  MODE_FP32 = 1,
  MODE_REL = 2,
  MODE_TAN = 3,
  MODE_FP64_DIAG = 4,
  MODE_FP32_DIAG = 5,
  MODE_REL_DIAG = 6,
  // N x N pairing (Sec. 3.1) in the FP64, FP32 and relativistic forms
  MODE_FP64_NXN = 7,
  MODE_FP32_NXN = 8,
  MODE_REL_NXN = 9,
  // duplicity pairing (Higginson et al.'s s) in the same three forms
  MODE_FP64_DUP = 10,
  MODE_FP32_DUP = 11,
  MODE_REL_DUP = 12,
  NMODE = 13
};

// the order-N mode whose variants and defaults another pairing's mode shares
inline constexpr int base_mode(int mode) {
  return (mode == MODE_FP64_NXN || mode == MODE_FP64_DUP)   ? MODE_FP64
         : (mode == MODE_FP32_NXN || mode == MODE_FP32_DUP) ? MODE_FP32
         : (mode == MODE_REL_NXN || mode == MODE_REL_DUP)   ? MODE_REL
                                                             : mode;
}

// layout: 0 all in LDS; 1 compact LDS (weights read from the input);
// 2 per-workgroup global scratch (one wave per cell, or several waves for
// the plain FP64 and FP32 modes)
struct Variant {
  int tpc;     // threads per cell (workgroup size)
  int cap;     // largest cell the variant holds
  int layout;  // 0 LDS, 1 compact LDS, 2 global scratch
};

constexpr int NVARIANT = 16;
constexpr Variant kVariants[NVARIANT] = {
    {64, 128, 0},    {64, 256, 0},   {128, 256, 0},  {128, 512, 0},  {256, 512, 0},
    {256, 1024, 0},  {512, 1024, 0}, {512, 2048, 0}, {1024, 2048, 0}, {1024, 4096, 1},
    {64, 32768, 2},  {256, 2048, 0}, {512, 4096, 1}, {256, 4096, 1},
    {256, 32768, 2}, {512, 32768, 2}};
// the one-wave global variant, which the modes without multi-wave global
// kernels use in place of variants 14 and 15
constexpr int kGlobalOneWave = 10;
// the relativistic mode keeps a per-pair h(-mu) buffer, which the compact
// layout has no room for: its 4096-cell variants use global scratch
constexpr Variant kRelVariant4096 = {64, 4096, 2};
// the same with 4 waves per cell, for the relativistic order-N step (8 waves
// would cap the registers at 256 and spill)
constexpr Variant kRelVariant4096Wide = {256, 4096, 2};

// cell-size buckets: bucket b holds cells with kBucketCap[b-1] < n <= kBucketCap[b]
constexpr int NBUCKET = 7;
constexpr int kBucketCap[NBUCKET] = {128, 256, 512, 1024, 2048, 4096, 32768};
// default variant per bucket (the fastest measured on lognormal cell-size
// mixes; the autotuner may pick another candidate).  The FP32 and FP64 modes
// take 256 threads for the 2048 bucket (under the 2-wave register cap the
// FP64 512-thread kernel holds one workgroup per CU: 0.55 against 0.43 ms on
// the 65,536-cell mix); the relativistic and tangent modes, whose cells keep
// the full LDS layout, 512.  Cells above 4096 particles take 8 waves in
// global scratch (measured on cells of 4 400 to 8 200 particles: 5.1-5.3x the
// one-wave variant, 1.5x the 4-wave)
constexpr int kDefaultVariant[NBUCKET] = {0, 1, 3, 5, 7, 12, 15};
constexpr int kDefaultVariantFP[NBUCKET] = {0, 1, 3, 5, 11, 12, 15};
// candidates the autotuner times per bucket (-1 terminated)
constexpr int kCandidates[NBUCKET][5] = {
    {0, 1, 2, -1, -1}, {1, 2, 3, 4, -1}, {3, 4, 5, 6, -1}, {5, 6, 7, 11, -1},
    {7, 11, 8, -1, -1}, {12, 13, 9, -1, -1}, {15, 14, 10, -1, -1}};

// the tangent form keeps six more doubles per particle and one per pair: in
// LDS up to 1024 particles, above that in global scratch
constexpr Variant kTanVariantBig = {64, 4096, 2};

// The FP64 and FP32 modes run every LDS variant in the compact layout
// (weights read from HBM, keys and pair energies aliased: 40-42 B of LDS per
// particle of capacity instead of 56, so more cells are resident per CU); the
// relativistic and tangent modes keep the full layout.
inline constexpr Variant compact_of(Variant V) {
  return V.layout == 0 ? Variant{V.tpc, V.cap, 1} : V;
}

inline constexpr int default_variant(int mode, int bucket) {
  return (base_mode(mode) == MODE_FP32 || mode == MODE_FP32_DIAG || base_mode(mode) == MODE_FP64 ||
          mode == MODE_FP64_DIAG)
             ? kDefaultVariantFP[bucket]
             : kDefaultVariant[bucket];
}

// multi-wave global-scratch kernels: the FP64, FP32 and relativistic modes
// of every pairing (the waves of a workgroup share their CU's L1, so the
// barrier orders their scratch accesses as it does for LDS)
inline constexpr bool multiwave_global(int m) {
  return m == MODE_FP64 || m == MODE_FP32 || m == MODE_REL || m == MODE_FP64_NXN ||
         m == MODE_FP32_NXN || m == MODE_REL_NXN || m == MODE_FP64_DUP || m == MODE_FP32_DUP ||
         m == MODE_REL_DUP;
}
inline constexpr Variant variant_of(int m, int v) {
  const int mode = base_mode(m);
  return (kVariants[v].layout == 2 && kVariants[v].tpc > 64 && !multiwave_global(m))
             ? variant_of(m, kGlobalOneWave)
         : ((mode == MODE_REL || mode == MODE_REL_DIAG) && kVariants[v].layout == 1)
             ? (m == MODE_REL ? kRelVariant4096Wide : kRelVariant4096)
         : (mode == MODE_TAN && kVariants[v].cap > 1024 && kVariants[v].layout != 2)
             ? kTanVariantBig
         : (mode == MODE_FP64 || mode == MODE_FP32 || mode == MODE_FP64_DIAG ||
            mode == MODE_FP32_DIAG)
             ? compact_of(kVariants[v])
             : kVariants[v];
}

// Minimum waves per SIMD the compiler must leave room for (it then caps the
// registers, spilling a little): measured on the lognormal cell-size mix,
// where 2 waves per SIMD (the uncapped allocation) left the cell kernels
// waiting on LDS and barriers most of the time.  Cells of 2048 and 4096
// particles, whose LDS use allows at most 8 waves per CU, ask for 2: an
// uncapped allocation that reaches 256 registers leaves room for one.
// 1: no cap (the global-scratch and tangent forms).
constexpr int min_waves(int tpc, int cap, int layout, bool fp64, bool tangent) {
  if (tangent || layout == 2) return 1;
  if (cap >= 2048) return 2;
  if (tpc == 64 && cap == 128) return 4;
  return 3;
}

// global scratch bytes per workgroup of a global-layout variant:
// 8 CAP doubles (v, w, snapshot, pair buffer), 2 CAP u32 (keys, slots),
// 6 CAP u16 (lists, orders, bucket members, weight order)
// (tangent form: 7 more CAP doubles for the tangent, its snapshot and the
// per-pair tangents)
constexpr unsigned long long big_stride_bytes(int cap, bool tan = false) {
  return ((unsigned long long)cap * (8 * 8 + 2 * 4 + 6 * 2 + (tan ? 7 * 8 : 0)) + 255ull) &
         ~255ull;
}

}  // namespace mcc
