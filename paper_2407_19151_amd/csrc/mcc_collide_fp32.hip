// Instantiations of the collide kernel for the FP32 mode.
#include "mcc_collide.hpp"
#include "mcc_variants.hpp"

namespace mcc {
#define V(i)                                                                        \
  ((const void *)&collide_kernel<variant_of(MODE_FP32, i).tpc, variant_of(MODE_FP32, i).cap, \
                                 float, false, variant_of(MODE_FP32, i).layout>)
const void *const kTable_FP32[NVARIANT] = {V(0), V(1), V(2),  V(3),  V(4),  V(5),  V(6),
                                    V(7), V(8), V(9), V(10), V(11), V(12), V(13), V(14), V(15)};
#undef V
}  // namespace mcc

const void *const *mcc_kernel_table_fp32() { return mcc::kTable_FP32; }
