// Table of kernel entry points for one (element type, dimension) pair.
#pragma once

namespace paraiso {

// index of a waves-per-EU hint in the tables: 0 (compiler), 3, 4, 5
inline int waves_slot(int w) { return w == 3 ? 1 : (w == 4 ? 2 : (w == 5 ? 3 : 0)); }

struct KernelTable {
  const void* stage_direct[4];
  const void* stage_lds[4];
  const void* stage_lds_opt[3][4];  // [kOpt* bits - 1]: analytic ghosts, first order, both
  const void* fused_lds[4];
  const void* fused_lds_first[4];  // first-order reconstruction
  const void* stage_lds_keep[2][4];  // [manifest - 1]: face states kept in LDS, without / with face fluxes
  const void* fused_lds_keep[2][4];
  const void* fused_direct[4];
  const void* march_fused[4];  // 2D register march (null for other dimensions)
  const void* march_stage[4];
  const void* march_stage_an[4];  // one stage with analytic ghost cells from the ghost arrays (2D)
  const void* march3d_stage[4];  // 3D register march, one stage (null for other dimensions)
  const void* resident1d[2];     // whole-advance kernel of small 1D meshes, 512 / 1024 threads (null otherwise)
  const void* cfl;
  const void* totals_partial;
  const void* totals_final;
  const void* exact_state;       // exact solution of an analytic problem into a state buffer
  const void* analytic_ghosts;   // the ghost arrays of 2D analytic meshes for one step (2D)
  int elem_bytes;
  const void* march3d_fused[4];  // 3D register march, both stages in one launch (null for other dimensions)
};

const KernelTable* table_f32_1();
const KernelTable* table_f32_2();
const KernelTable* table_f32_3();
const KernelTable* table_f64_1();
const KernelTable* table_f64_2();
const KernelTable* table_f64_3();

}  // namespace paraiso
