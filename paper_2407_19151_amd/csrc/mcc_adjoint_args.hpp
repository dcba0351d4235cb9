// mcc_adjoint_args.hpp -- argument block of the reverse-mode kernels
// (mcc_collide_adjoint), shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mcc_kernel_args.hpp"

namespace mcc {

struct AdjointArgs {
  const int64_t *offsets;
  const double *w;
  const double *vx, *vy, *vz;  // the step's input (read)
  double *gx, *gy, *gz;        // in: adjoint of the output; out: of the input
  const double *cell_volume;
  double dV;
  int64_t n;
  int32_t n_cells, S, n_coll;
  int32_t method, corr, sortw, keep;
  double fE;
  double inv_lnl;  // 1 / lnL (0 when lnL = 0: no pair scatters)
  uint64_t seed, step;
  double mass[MCC_MAX_SPECIES];
  CollConst coll[MCC_MAX_COLLISIONS];
  const int32_t *cell_list;
  const uint32_t *cell_count;
  double *lnl_part;  // [n_cells]: per-cell adjoint of lnL
  int32_t *err;
  const double2 *n97;
  char *scratch;
  uint64_t stride;
};

// per-workgroup scratch: 26 doubles, 2 u32 and 6 u16 per particle of capacity
constexpr unsigned long long adj_stride_bytes(int cap) {
  return ((unsigned long long)cap * (26 * 8 + 2 * 4 + 6 * 2) + 255ull) & ~255ull;
}

}  // namespace mcc
