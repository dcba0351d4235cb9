// mcc_kernel_args.hpp -- argument block shared by the host launcher and the
// collide kernels (passed by value, one kernel argument).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mcc.h"

namespace mcc {

// knots of the N97 A(s) table (uniform in ln s)
constexpr int N97_TABLE_SIZE = 256;

// Per-collision constants computed on the host in FP64.
struct CollConst {
  int32_t a, b;   // species of the collision (a == b: intra-species)
  double coef;    // NR: qa^2 qb^2 lnL dt / (4 pi eps0^2 mu^2); REL: without mu^2
  double fa, fb;  // m_b/(m_a+m_b), m_a/(m_a+m_b): shares of du (Eq. (8) masses)
};

// Per (cell, species) data that depends on the weights only, computed once
// by a plan and read by every step: sum w, sum w^2, the weight range (bit
// patterns) and the weight class (equal / distinct / ties)
struct SpeciesPrep {
  double sw, sw2;
  uint64_t lo, hi;
  int32_t flag;
  int32_t pad;
};

// prep_mode of CollideArgs
enum : int32_t { PREP_NONE = 0, PREP_WRITE = 1, PREP_READ = 2 };

// the collide kernels hand out cells from up to this many interleaved
// queues, each with a claim and a finished-workgroup counter at the start of
// its own WORK_STRIDE u32 (256 B)
constexpr int WORK_QUEUES = 32;
constexpr int WORK_STRIDE = 64;

struct CollideArgs {
  const int64_t *offsets;  // [n_cells*S + 1]
  const double *w;
  double *vx, *vy, *vz;
  const double *cell_volume;  // nullable
  double dV;
  int64_t n;
  int32_t n_cells, S, n_coll;
  int32_t method, corr, sortw, max_passes, keep, diag;
  double fE, c;
  uint64_t seed, step;
  const uint64_t *step_dev;  // nullable: step read from device memory (graph replay)
  double mass[MCC_MAX_SPECIES];
  CollConst coll[MCC_MAX_COLLISIONS];
  const int32_t *cell_list;     // work list of this size bucket
  const uint32_t *cell_count;   // device count of cell_list
  uint32_t *work;               // [WORK_QUEUES * WORK_STRIDE] queue counters of the launch,
                                // zero at launch and reset to zero by its end
  mcc_stats *stats;             // nullable
  int32_t *cell_corr;           // nullable
  int32_t *err;                 // device error word
  char *big_scratch;            // large-cell variants: per-block global scratch
  uint64_t big_stride;          // bytes per block
  unsigned long long *phase;    // profiling builds (MCC_PHASE_TIMING): clock ticks per phase
  const double2 *n97;           // N97 table: A and h dA/dt at the knots of t = ln s
  // tangent (forward-mode) form only
  double *tx, *ty, *tz;         // tangent of the velocities, in/out
  double dlnl;                  // tangent of ln(Lambda) relative to ln(Lambda)
  int32_t write_primal;         // 0: the velocities are read but not written back
  // weight data of a plan: PREP_WRITE computes and stores it (launched with
  // no collisions), PREP_READ uses it (prep[n_cells*S], prep_word[n]:
  // descending-weight order, cell-local)
  int32_t prep_mode;
  SpeciesPrep *prep;
  uint16_t *prep_word;
};

}  // namespace mcc
