// Kernel instantiations for float, 3D.
#include "euler_kernels.h"
#include "euler_march3d.h"
#include "kernel_table.h"

namespace paraiso {

#define PARAISO_SET(K) {(const void*)K<float, 3, 0>, (const void*)K<float, 3, 3>, \
                        (const void*)K<float, 3, 4>, (const void*)K<float, 3, 5>}
#define PARAISO_SET_OPT(K, O) {(const void*)K<float, 3, 0, O>, (const void*)K<float, 3, 3, O>, \
                               (const void*)K<float, 3, 4, O>, (const void*)K<float, 3, 5, O>}
#define PARAISO_SET_KEEP(K, KP) {(const void*)K<float, 3, 0, 0, KP>, (const void*)K<float, 3, 3, 0, KP>, \
                                 (const void*)K<float, 3, 4, 0, KP>, (const void*)K<float, 3, 5, 0, KP>}

const KernelTable* table_f32_3() {
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
      {(const void*)k_march3d<float, 0>, (const void*)k_march3d<float, 3>, (const void*)k_march3d<float, 4>,
       (const void*)k_march3d<float, 5>},
      {nullptr, nullptr},
      (const void*)k_cfl<float, 3>,
      (const void*)k_totals_partial<float, 3>,
      (const void*)k_totals_final<3>,
      (const void*)k_exact_state<float, 3>,
      nullptr,
      (int)sizeof(float),
      {(const void*)k_march3d_fused<float, 0>, (const void*)k_march3d_fused<float, 3>,
       (const void*)k_march3d_fused<float, 4>, (const void*)k_march3d_fused<float, 5>},
  };
  return &t;
}

}  // namespace paraiso
