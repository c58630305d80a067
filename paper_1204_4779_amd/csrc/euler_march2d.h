// Register-march kernels for 2D periodic meshes (gfx950, wave64).
//
// Each wave owns a strip of 64 columns: 64 - 2H interior columns plus H halo
// columns per side (H = 4 for the fused step, 2 for one stage) and marches
// over a chunk of rows.  x-neighbours come from the neighbouring lanes
// through DPP wave shifts (v_mov_b32_dpp wave_shr:1 / wave_shl:1); the
// y-stencil lives in registers as a sliding window of primitive rows,
// slopes and y-face fluxes.  Each face flux of the strip is evaluated once.
// In the fused step the stage-2 pipeline runs two rows behind stage 1 and
// consumes stage-1 rows straight from registers, so U1 never leaves the CU.
//
// Row pipeline of one stage: rows k = 0,1,2,... are pushed in order.  After
// row k arrives the pipeline has V(k-2), V(k-1), V(k); it forms the limited
// y-slope of row k-1, the y-face flux between rows k-2 and k-1, and then the
// complete update of row k-2 (its x-face fluxes from the lanes, its two
// y-face fluxes from this push and the previous one).
#pragma once

#include "euler_kernels.h"

namespace paraiso {

// lane l receives lane l-1 (lane 0 receives 0)
__device__ __forceinline__ float lane_from_left(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x138, 0xf, 0xf, false));
}
// lane l receives lane l+1 (lane 63 receives 0)
__device__ __forceinline__ float lane_from_right(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ double lane_from_left(double x) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x138, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_from_right(double x) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x130, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// F(l-1/2) - F(l+1/2) of the x-faces of one row of primitives held one
// column per lane.  Valid on lanes 2..61.
template <typename T>
__device__ __forceinline__ void xflux_diff(const T* v, const Gas<T>& g, T* dF) {
  T up[4], lo_next[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const T vm = lane_from_left(v[q]);
    const T vp = lane_from_right(v[q]);
    const T s = minmod(v[q] - vm, vp - v[q]);
    up[q] = v[q] + T(0.5) * s;
    lo_next[q] = lane_from_right(v[q] - T(0.5) * s);
  }
  T f[4];
  hllc<T, 2, 0>(up, lo_next, f, g);
#pragma unroll
  for (int q = 0; q < 4; ++q) dF[q] = lane_from_left(f[q]) - f[q];
}

template <typename T>
struct RowPipe {
  T a[4], b[4];  // primitives of rows k-2 and k-1
  T upa[4];      // upper y-face value of row k-2
  T g[4];        // y-face flux between rows k-3 and k-2
};

// Push V(row k) as `c`; with `n` rows pushed before this one.  When n >= 4
// the update acc = kx dFx + ky dGy of row k-2 is returned in acc and the
// function returns true.
template <typename T>
__device__ __forceinline__ bool pipe_push(RowPipe<T>& P, const T* c, int n, const Gas<T>& g, T kx, T ky,
                                          T* acc) {
  bool done = false;
  if (n >= 2) {
    T slope[4], lo_b[4], up_b[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      slope[q] = minmod(P.b[q] - P.a[q], c[q] - P.b[q]);
      lo_b[q] = P.b[q] - T(0.5) * slope[q];
      up_b[q] = P.b[q] + T(0.5) * slope[q];
    }
    if (n >= 3) {
      T G[4];
      hllc<T, 2, 1>(P.upa, lo_b, G, g);
      if (n >= 4) {
        T dF[4];
        xflux_diff<T>(P.a, g, dF);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          acc[q] = kx * dF[q];
          acc[q] += ky * (P.g[q] - G[q]);
        }
        done = true;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) P.g[q] = G[q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) P.upa[q] = up_b[q];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    P.a[q] = P.b[q];
    P.b[q] = c[q];
  }
  return done;
}

// Fused step (FUSED, periodic meshes) or one stage (!FUSED, periodic or
// outflow: the stage's ghost cells are clamped loads of its input).
// Block = threads/64 waves; the block tile is (64 - 2H) columns by
// (waves * rows) rows, wave w taking rows [w*rows, (w+1)*rows) of it.
template <typename T, int W, bool FUSED>
__global__ void __launch_bounds__(256) PARAISO_WAVES_ATTR(W) k_march2d(Args a, LdsGeom) {
  constexpr int H = FUSED ? 4 : 2;
  __shared__ double s_red[16];
  __shared__ int s_item;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int rows = a.tile[1] / (blockDim.x >> 6);
  ItemLoop it{0, 1};
  for (int item; (item = next_item(a, it, &s_item, FUSED ? 0 : a.stage - 1)) >= 0;) {
    const Tile t = tile_of(a, item);
    const MeshDev& M = a.meshes[t.m];
    bool active;
    const double dt = step_dt(a, t.m, active);
    const bool last_stage = FUSED || a.stage == 2;
    if (last_stage && t.first && threadIdx.x == 0) step_bookkeeping(a, t.m, dt, active);
    const Gas<T> g = gas_of<T>(M);
    const int nx = M.n[0], ny = M.n[1];
    const int x0 = t.org[0], y0 = t.org[1] + wave * rows;
    const int y1 = min(y0 + rows, ny);
    const int col = map_index(x0 - H + lane, nx, FUSED ? kPeriodic : M.bc[0]);
    const bool store_lane = lane >= H && lane < 64 - H && (x0 - H + lane) < nx;
    const Fields<T, 2> U0 = fields<T, 2>(M.s[a.src]);
    const Fields<T, 2> Uin = (FUSED || a.stage == 1) ? U0 : fields<T, 2>(M.w);
    const Fields<T, 2> Uout =
        (FUSED || a.stage == 2) ? fields<T, 2>(M.s[1 - a.src]) : fields<T, 2>(M.w);
    double qmax = 0.0;
    bool bad = false;
    if (y0 < ny && (active || last_stage)) {
      if (!active) {
        for (int y = y0; y < y1; ++y) {
          const int gi = y * nx + col;
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (store_lane) Uout.f[q][gi] = U0.f[q][gi];
        }
      } else {
        const double c1 = FUSED ? 0.5 * dt : (a.stage == 1 ? 0.5 * dt : dt);
        const T kx1 = (T)(c1 * M.inv_dx[0]), ky1 = (T)(c1 * M.inv_dx[1]);
        const T kx2 = (T)(dt * M.inv_dx[0]), ky2 = (T)(dt * M.inv_dx[1]);
        RowPipe<T> P1, P2;
        // base-state ring: U0 of the rows whose update is pending
        T ub[5][4];
        const int first = y0 - H;          // first row pushed into stage 1
        const int npush = (y1 - y0) + 2 * H;
        int n1 = 0, n2 = 0;
        T nxt[4];
        {
          const int gi = map_index(first, ny, FUSED ? kPeriodic : M.bc[1]) * nx + col;
#pragma unroll
          for (int q = 0; q < 4; ++q) nxt[q] = Uin.f[q][gi];
        }
        for (int k = 0; k < npush; ++k) {
          T u[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) u[q] = nxt[q];
          if (k + 1 < npush) {
            const int gi = map_index(first + k + 1, ny, FUSED ? kPeriodic : M.bc[1]) * nx + col;
#pragma unroll
            for (int q = 0; q < 4; ++q) nxt[q] = Uin.f[q][gi];
          }
          // base state of this row (U0; equals u for the fused step and stage 1)
          T base[4];
          if (FUSED || a.stage == 1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) base[q] = u[q];
          } else {
            const int gi = map_index(first + k, ny, FUSED ? kPeriodic : M.bc[1]) * nx + col;
#pragma unroll
            for (int q = 0; q < 4; ++q) base[q] = U0.f[q][gi];
          }
#pragma unroll
          for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int q = 0; q < 4; ++q) ub[s][q] = ub[s + 1][q];
#pragma unroll
          for (int q = 0; q < 4; ++q) ub[4][q] = base[q];
          T v[4];
          prim_of_cons<T, 2>(u, v, g);
          T acc[4];
          if (pipe_push<T>(P1, v, n1++, g, kx1, ky1, acc)) {
            // stage-1 output: row first + k - 2, its base is ub[2]
            T u1[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) u1[q] = ub[2][q] + acc[q];
            if (!FUSED) {
              const int y = first + k - 2;
              const int gi = y * nx + col;
              if (store_lane) {
#pragma unroll
                for (int q = 0; q < 4; ++q) Uout.f[q][gi] = u1[q];
              }
              if (last_stage && a.cfl && store_lane) {
                const double qv = cfl_q<T, 2>(u1, M.inv_dx, M.gamma);
                bad |= !(qv > 0.0);
                qmax = fmax(qmax, qv);
              }
            } else {
              T v1[4];
              prim_of_cons<T, 2>(u1, v1, g);
              T acc2[4];
              if (pipe_push<T>(P2, v1, n2++, g, kx2, ky2, acc2)) {
                // stage-2 output: row first + k - 4, base ub[0]
                const int y = first + k - 4;
                T u2[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) u2[q] = ub[0][q] + acc2[q];
                const int gi = y * nx + col;
                if (store_lane) {
#pragma unroll
                  for (int q = 0; q < 4; ++q) Uout.f[q][gi] = u2[q];
                }
                if (a.cfl && store_lane) {
                  const double qv = cfl_q<T, 2>(u2, M.inv_dx, M.gamma);
                  bad |= !(qv > 0.0);
                  qmax = fmax(qmax, qv);
                }
              }
            }
          }
        }
      }
    }
    if (a.cfl && active && last_stage) cfl_commit(a, t.m, qmax, bad, s_red, (a.ring + 1) % 3);
  }
}

}  // namespace paraiso
