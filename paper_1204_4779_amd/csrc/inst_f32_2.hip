// Kernel instantiations for float, 2D.
#include "euler_kernels.h"
#include "euler_march2d.h"
#include "kernel_table.h"

namespace paraiso {

#define PARAISO_SET(K) {(const void*)K<float, 2, 0>, (const void*)K<float, 2, 3>, \
                        (const void*)K<float, 2, 4>, (const void*)K<float, 2, 5>}
#define PARAISO_SET_OPT(K, O) {(const void*)K<float, 2, 0, O>, (const void*)K<float, 2, 3, O>, \
                               (const void*)K<float, 2, 4, O>, (const void*)K<float, 2, 5, O>}
#define PARAISO_SET_KEEP(K, KP) {(const void*)K<float, 2, 0, 0, KP>, (const void*)K<float, 2, 3, 0, KP>, \
                                 (const void*)K<float, 2, 4, 0, KP>, (const void*)K<float, 2, 5, 0, KP>}

const KernelTable* table_f32_2() {
  static const KernelTable t = {
      PARAISO_SET(k_stage_direct),
      PARAISO_SET(k_stage_lds),
      {PARAISO_SET_OPT(k_stage_lds, 1), PARAISO_SET_OPT(k_stage_lds, 2), PARAISO_SET_OPT(k_stage_lds, 3)},
      PARAISO_SET(k_fused_lds),
      PARAISO_SET_OPT(k_fused_lds, 2),
      {PARAISO_SET_KEEP(k_stage_lds, 1), PARAISO_SET_KEEP(k_stage_lds, 2)},
      {PARAISO_SET_KEEP(k_fused_lds, 1), PARAISO_SET_KEEP(k_fused_lds, 2)},
      PARAISO_SET(k_fused_direct),
      {(const void*)k_march2d<float, 0, true>, (const void*)k_march2d<float, 3, true>,
       (const void*)k_march2d<float, 4, true>, (const void*)k_march2d<float, 5, true>},
      {(const void*)k_march2d<float, 0, false>, (const void*)k_march2d<float, 3, false>,
       (const void*)k_march2d<float, 4, false>, (const void*)k_march2d<float, 5, false>},
      {(const void*)k_march2d<float, 0, false, true>, (const void*)k_march2d<float, 3, false, true>,
       (const void*)k_march2d<float, 4, false, true>, (const void*)k_march2d<float, 5, false, true>},
      {nullptr, nullptr, nullptr, nullptr},
      {nullptr, nullptr},
      (const void*)k_cfl<float, 2>,
      (const void*)k_totals_partial<float, 2>,
      (const void*)k_totals_final<2>,
      (const void*)k_exact_state<float, 2>,
      (const void*)k_analytic_ghosts<float>,
      (int)sizeof(float),
  };
  return &t;
}

}  // namespace paraiso
