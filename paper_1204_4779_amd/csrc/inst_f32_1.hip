// Kernel instantiations for float, 1D.
#include "euler_kernels.h"
#include "euler_resident1d.h"
#include "kernel_table.h"

namespace paraiso {

#define PARAISO_SET(K) {(const void*)K<float, 1, 0>, (const void*)K<float, 1, 3>, \
                        (const void*)K<float, 1, 4>, (const void*)K<float, 1, 5>}
#define PARAISO_SET_OPT(K, O) {(const void*)K<float, 1, 0, O>, (const void*)K<float, 1, 3, O>, \
                               (const void*)K<float, 1, 4, O>, (const void*)K<float, 1, 5, O>}
#define PARAISO_SET_KEEP(K, KP) {(const void*)K<float, 1, 0, 0, KP>, (const void*)K<float, 1, 3, 0, KP>, \
                                 (const void*)K<float, 1, 4, 0, KP>, (const void*)K<float, 1, 5, 0, KP>}

const KernelTable* table_f32_1() {
  static const KernelTable t = {
      PARAISO_SET(k_stage_direct),
      PARAISO_SET(k_stage_lds),
      {PARAISO_SET_OPT(k_stage_lds, 1), PARAISO_SET_OPT(k_stage_lds, 2), PARAISO_SET_OPT(k_stage_lds, 3)},
      PARAISO_SET(k_fused_lds),
      PARAISO_SET_OPT(k_fused_lds, 2),
      {PARAISO_SET_KEEP(k_stage_lds, 1), PARAISO_SET_KEEP(k_stage_lds, 2)},
      {PARAISO_SET_KEEP(k_fused_lds, 1), PARAISO_SET_KEEP(k_fused_lds, 2)},
      PARAISO_SET(k_fused_direct),
      {nullptr, nullptr, nullptr, nullptr},
      {nullptr, nullptr, nullptr, nullptr},
      {nullptr, nullptr, nullptr, nullptr},
      {nullptr, nullptr, nullptr, nullptr},
      {(const void*)k_resident1d<float, 512>, (const void*)k_resident1d<float, 1024>},
      (const void*)k_cfl<float, 1>,
      (const void*)k_totals_partial<float, 1>,
      (const void*)k_totals_final<1>,
      (const void*)k_exact_state<float, 1>,
      nullptr,
      (int)sizeof(float),
  };
  return &t;
}

}  // namespace paraiso
