// Per-cell (direct) step kernels: each cell computes its own face fluxes.
#pragma once

#include "euler_common.h"

namespace paraiso {

// ---------------------------------------------------------------------------
// direct stage: each cell computes its own 2d face fluxes from global memory
// (nothing shared between neighbours; the untuned baseline)
// ---------------------------------------------------------------------------

template <typename T, int D, int AX>
__device__ __forceinline__ void direct_axis(const MeshDev& M, const Fields<T, D>& Uin, int i, int j,
                                            int k, const T* vc, const Gas<T>& g, T coef, T* acc) {
  T v[5][D + 2];  // cells -2..+2 along AX
  const int c[3] = {i, j, k};
#pragma unroll
  for (int o = -2; o <= 2; ++o) {
    if (o == 0) {
#pragma unroll
      for (int q = 0; q < D + 2; ++q) v[2][q] = vc[q];
      continue;
    }
    int cc[3] = {c[0], c[1], c[2]};
    cc[AX] = map_index(c[AX] + o, M.n[AX], M.bc[AX]);
    const int gi = gidx(M, cc[0], cc[1], cc[2]);
    T u[D + 2];
#pragma unroll
    for (int q = 0; q < D + 2; ++q) u[q] = Uin.f[q][gi];
    prim_of_cons<T, D>(u, v[o + 2], g);
  }
  T vl[D + 2], vr[D + 2], fm[D + 2], fp[D + 2];
#pragma unroll
  for (int q = 0; q < D + 2; ++q) face_states(v[0][q], v[1][q], v[2][q], v[3][q], vl[q], vr[q]);
  hllc<T, D, AX>(vl, vr, fm, g);
#pragma unroll
  for (int q = 0; q < D + 2; ++q) face_states(v[1][q], v[2][q], v[3][q], v[4][q], vl[q], vr[q]);
  hllc<T, D, AX>(vl, vr, fp, g);
#pragma unroll
  for (int q = 0; q < D + 2; ++q) acc[q] += coef * (fm[q] - fp[q]);
}

// acc = sum_a coef_a (F_a[i-1/2] - F_a[i+1/2]) of one cell from state Uin.
template <typename T, int D>
__device__ __forceinline__ void direct_rhs(const MeshDev& M, const Fields<T, D>& Uin, int i, int j,
                                           int k, const Gas<T>& g, const T* coef, T* acc) {
  T u[D + 2], vc[D + 2];
  const int gc = gidx(M, i, j, k);
#pragma unroll
  for (int q = 0; q < D + 2; ++q) {
    u[q] = Uin.f[q][gc];
    acc[q] = T(0);
  }
  prim_of_cons<T, D>(u, vc, g);
  direct_axis<T, D, 0>(M, Uin, i, j, k, vc, g, coef[0], acc);
  if constexpr (D > 1) direct_axis<T, D, 1>(M, Uin, i, j, k, vc, g, coef[1], acc);
  if constexpr (D > 2) direct_axis<T, D, 2>(M, Uin, i, j, k, vc, g, coef[2], acc);
}

template <typename T, int D, int W>
__global__ void __launch_bounds__(512) PARAISO_WAVES_ATTR(W) k_stage_direct(Args a, LdsGeom) {
  __shared__ double s_red[16];
  __shared__ int s_item;
  ItemLoop it{0, 1};
  for (int item; (item = next_item(a, it, &s_item, a.stage - 1)) >= 0;) {
    const Tile t = tile_of(a, item);
    const MeshDev& M = a.meshes[t.m];
    bool active;
    const double dt = step_dt(a, t.m, active);
    if (a.stage == 2 && t.first && threadIdx.x == 0) step_bookkeeping(a, t.m, dt, active);
    const Gas<T> g = gas_of<T>(M);
    const double cdt = (a.stage == 1 ? 0.5 : 1.0) * dt;
    T coef[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) coef[ax] = (T)(cdt * M.inv_dx[ax]);
    const Fields<T, D> U0 = fields<T, D>(M.s[a.src]);
    const Fields<T, D> Uin = a.stage == 1 ? U0 : fields<T, D>(M.w);
    const Fields<T, D> Uout = a.stage == 1 ? fields<T, D>(M.w) : fields<T, D>(M.s[1 - a.src]);
    if (!active && a.stage == 1) continue;
    double qmax = 0.0;
    bool bad = false;
    const int tc = a.tile[0] * a.tile[1] * a.tile[2];
    for (int l = threadIdx.x; l < tc; l += blockDim.x) {
      const int li = l % a.tile[0], r = l / a.tile[0];
      const int lj = r % a.tile[1], lk = r / a.tile[1];
      const int i = t.org[0] + li, j = t.org[1] + lj, k = t.org[2] + lk;
      if (i >= M.n[0] || j >= M.n[1] || k >= M.n[2]) continue;
      const int gc = gidx(M, i, j, k);
      T out[D + 2];
      if (active) {
        T acc[D + 2];
        direct_rhs<T, D>(M, Uin, i, j, k, g, coef, acc);
#pragma unroll
        for (int q = 0; q < D + 2; ++q) out[q] = U0.f[q][gc] + acc[q];
      } else {
#pragma unroll
        for (int q = 0; q < D + 2; ++q) out[q] = U0.f[q][gc];
      }
#pragma unroll
      for (int q = 0; q < D + 2; ++q) Uout.f[q][gc] = out[q];
      if (a.cfl && active) {
        cfl_fold(cfl_q<T, D>(out, M.inv_dx, M.gamma), qmax, bad);
      }
    }
    if (a.cfl && active) cfl_commit(a, t.m, qmax, bad, s_red, (a.ring + 1) % 3);
  }
}

// Fused direct step: stage 1 is recomputed wherever stage 2 needs it (every
// intermediate delayed).  U1 at a neighbour position p along an axis is the
// stage-1 update of the cell p maps onto (periodic wrap; outflow copies the
// edge cell's U1, as the ghost fill of the stage-1 state does).
template <typename T, int D>
__device__ __forceinline__ void direct_u1(const MeshDev& M, const Fields<T, D>& U0, int i, int j, int k,
                                          const Gas<T>& g, const T* coef1, T* u1) {
  T acc[D + 2];
  direct_rhs<T, D>(M, U0, i, j, k, g, coef1, acc);
  const int gc = gidx(M, i, j, k);
#pragma unroll
  for (int q = 0; q < D + 2; ++q) u1[q] = U0.f[q][gc] + acc[q];
}

template <typename T, int D, int AX>
__device__ __forceinline__ void direct_fused_axis(const MeshDev& M, const Fields<T, D>& U0, int i, int j,
                                                  int k, const T* v1c, const Gas<T>& g, const T* coef1,
                                                  T coef2, T* acc) {
  T v[5][D + 2];
  const int c[3] = {i, j, k};
#pragma unroll
  for (int o = -2; o <= 2; ++o) {
    if (o == 0) {
#pragma unroll
      for (int q = 0; q < D + 2; ++q) v[2][q] = v1c[q];
      continue;
    }
    int cc[3] = {c[0], c[1], c[2]};
    cc[AX] = map_index(c[AX] + o, M.n[AX], M.bc[AX]);
    T u1[D + 2];
    direct_u1<T, D>(M, U0, cc[0], cc[1], cc[2], g, coef1, u1);
    prim_of_cons<T, D>(u1, v[o + 2], g);
  }
  T vl[D + 2], vr[D + 2], fm[D + 2], fp[D + 2];
#pragma unroll
  for (int q = 0; q < D + 2; ++q) face_states(v[0][q], v[1][q], v[2][q], v[3][q], vl[q], vr[q]);
  hllc<T, D, AX>(vl, vr, fm, g);
#pragma unroll
  for (int q = 0; q < D + 2; ++q) face_states(v[1][q], v[2][q], v[3][q], v[4][q], vl[q], vr[q]);
  hllc<T, D, AX>(vl, vr, fp, g);
#pragma unroll
  for (int q = 0; q < D + 2; ++q) acc[q] += coef2 * (fm[q] - fp[q]);
}

template <typename T, int D, int W>
__global__ void __launch_bounds__(512) PARAISO_WAVES_ATTR(W) k_fused_direct(Args a, LdsGeom) {
  __shared__ double s_red[16];
  __shared__ int s_item;
  ItemLoop it{0, 1};
  for (int item; (item = next_item(a, it, &s_item, 0)) >= 0;) {
    const Tile t = tile_of(a, item);
    const MeshDev& M = a.meshes[t.m];
    bool active;
    const double dt = step_dt(a, t.m, active);
    if (t.first && threadIdx.x == 0) step_bookkeeping(a, t.m, dt, active);
    const Gas<T> g = gas_of<T>(M);
    T coef1[3], coef2[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      coef1[ax] = (T)((0.5 * dt) * M.inv_dx[ax]);
      coef2[ax] = (T)(dt * M.inv_dx[ax]);
    }
    const Fields<T, D> U0 = fields<T, D>(M.s[a.src]);
    const Fields<T, D> Uout = fields<T, D>(M.s[1 - a.src]);
    double qmax = 0.0;
    bool bad = false;
    const int tc = a.tile[0] * a.tile[1] * a.tile[2];
    for (int l = threadIdx.x; l < tc; l += blockDim.x) {
      const int li = l % a.tile[0], r = l / a.tile[0];
      const int lj = r % a.tile[1], lk = r / a.tile[1];
      const int i = t.org[0] + li, j = t.org[1] + lj, k = t.org[2] + lk;
      if (i >= M.n[0] || j >= M.n[1] || k >= M.n[2]) continue;
      const int gc = gidx(M, i, j, k);
      T out[D + 2];
      if (active) {
        T u1c[D + 2], v1c[D + 2], acc[D + 2];
        direct_u1<T, D>(M, U0, i, j, k, g, coef1, u1c);
        prim_of_cons<T, D>(u1c, v1c, g);
#pragma unroll
        for (int q = 0; q < D + 2; ++q) acc[q] = T(0);
        direct_fused_axis<T, D, 0>(M, U0, i, j, k, v1c, g, coef1, coef2[0], acc);
        if constexpr (D > 1) direct_fused_axis<T, D, 1>(M, U0, i, j, k, v1c, g, coef1, coef2[1], acc);
        if constexpr (D > 2) direct_fused_axis<T, D, 2>(M, U0, i, j, k, v1c, g, coef1, coef2[2], acc);
#pragma unroll
        for (int q = 0; q < D + 2; ++q) out[q] = U0.f[q][gc] + acc[q];
      } else {
#pragma unroll
        for (int q = 0; q < D + 2; ++q) out[q] = U0.f[q][gc];
      }
#pragma unroll
      for (int q = 0; q < D + 2; ++q) Uout.f[q][gc] = out[q];
      if (a.cfl && active) {
        cfl_fold(cfl_q<T, D>(out, M.inv_dx, M.gamma), qmax, bad);
      }
    }
    if (a.cfl && active) cfl_commit(a, t.m, qmax, bad, s_red, (a.ring + 1) % 3);
  }
}

}  // namespace paraiso
