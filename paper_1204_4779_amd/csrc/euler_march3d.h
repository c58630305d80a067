// Register-march stage kernel for 3D meshes (gfx950, wave64).
//
// A block of NW waves owns a tile of 60 x-columns (64 lanes with 2 halo
// columns per side) by NW y-rows (one row per wave) and marches along z
// through a chunk of planes.  Per plane:
//   * every wave loads its own row, waves 0..3 also one of the 4 halo rows,
//     converts to primitives and writes them to a double-buffered LDS plane;
//   * after one barrier, wave w evaluates the y-face below its row from the
//     LDS plane (wave NW-1 also the face above) into a 3-slot LDS ring of
//     y-fluxes, read back two planes later when that plane is assembled;
//   * the z-stencil of each column lives in registers (the row pipeline of
//     the 2D march, along z), x-neighbours come from DPP lane shifts.
// Each face flux of the tile is evaluated once.  One stage per launch (the
// halo of a fused step would cost 4 extra rows per tile); ghost cells are
// clamped (outflow) or wrapped (periodic) loads of the stage's input, which
// is how the stage fills them.
#pragma once

#include "euler_march2d.h"

namespace paraiso {

// F(l-1/2) - F(l+1/2) of the x-faces of one row held one column per lane (D = 3).
template <typename T>
__device__ __forceinline__ void xflux_diff3(const T* v, const Gas<T>& g, T* dF) {
  T up[5], lo_next[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const T vm = lane_from_left(v[q]);
    const T vp = lane_from_right(v[q]);
    const T s = minmod(v[q] - vm, vp - v[q]);
    up[q] = v[q] + T(0.5) * s;
    lo_next[q] = lane_from_right(v[q] - T(0.5) * s);
  }
  T f[5];
  hllc<T, 3, 0>(up, lo_next, f, g);
#pragma unroll
  for (int q = 0; q < 5; ++q) dF[q] = lane_from_left(f[q]) - f[q];
}

template <typename T>
struct RowPipe5 {
  T a[5], b[5];  // primitives of planes k-2 and k-1 (this column)
  T upa[5];      // upper z-face value of plane k-2
  T g[5];        // z-face flux between planes k-3 and k-2
};

// Push V(plane k) with n planes pushed before.  When n >= 4, returns true
// with dz = G(k-2 - 1/2) - G(k-2 + 1/2) and va = V(k-2).
template <typename T>
__device__ __forceinline__ bool pipe_push5(RowPipe5<T>& P, const T* c, int n, const Gas<T>& g, T* dz, T* va) {
  bool done = false;
  if (n >= 2) {
    T lo_b[5], up_b[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const T s = minmod(P.b[q] - P.a[q], c[q] - P.b[q]);
      lo_b[q] = P.b[q] - T(0.5) * s;
      up_b[q] = P.b[q] + T(0.5) * s;
    }
    if (n >= 3) {
      T G[5];
      hllc<T, 3, 2>(P.upa, lo_b, G, g);
      if (n >= 4) {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          dz[q] = P.g[q] - G[q];
          va[q] = P.a[q];
        }
        done = true;
      }
#pragma unroll
      for (int q = 0; q < 5; ++q) P.g[q] = G[q];
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) P.upa[q] = up_b[q];
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    P.a[q] = P.b[q];
    P.b[q] = c[q];
  }
  return done;
}

template <typename T, int W>
__global__ void __launch_bounds__(512) PARAISO_WAVES_ATTR(W) k_march3d(Args a, LdsGeom) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double s_red[16];
  __shared__ int s_item;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int NW = blockDim.x >> 6;
  const int NR = NW + 4;            // rows in an LDS plane
  T* sV = reinterpret_cast<T*>(smem);            // [2][5][NR][64]
  T* sG = sV + 2 * 5 * NR * 64;                  // [3][5][NW+1][64]
  const int vslot = 5 * NR * 64, gslot = 5 * (NW + 1) * 64;
  ItemLoop it{0, 1};
  for (int item; (item = next_item(a, it, &s_item, a.stage - 1)) >= 0;) {
    const Tile t = tile_of(a, item);
    const MeshDev& M = a.meshes[t.m];
    bool active;
    const double dt = step_dt(a, t.m, active);
    const bool last_stage = a.stage == 2;
    if (last_stage && t.first && threadIdx.x == 0) step_bookkeeping(a, t.m, dt, active);
    const Gas<T> g = gas_of<T>(M);
    const int nx = M.n[0], ny = M.n[1], nz = M.n[2];
    const int x0 = t.org[0], y0 = t.org[1], z0 = t.org[2];
    const int z1 = min(z0 + a.tile[2], nz);
    const int col = map_index(x0 - 2 + lane, nx, M.bc[0]);
    const int yrow = y0 + wave;                                   // this wave's row
    const int yown = map_index(yrow, ny, M.bc[1]);
    // halo rows: waves 0,1 take rows y0-2, y0-1; waves 2,3 take y0+NW, y0+NW+1
    const bool has_halo = wave < 4;
    const int hrel = wave < 2 ? wave : NW + wave;                 // LDS row of the halo row
    const int yhalo = map_index(y0 - 2 + hrel, ny, M.bc[1]);
    const bool store_lane = lane >= 2 && lane < 62 && (x0 - 2 + lane) < nx && yrow < ny;
    const Fields<T, 3> U0 = fields<T, 3>(M.s[a.src]);
    const Fields<T, 3> Uin = a.stage == 1 ? U0 : fields<T, 3>(M.w);
    const Fields<T, 3> Uout = a.stage == 2 ? fields<T, 3>(M.s[1 - a.src]) : fields<T, 3>(M.w);
    const int plane = nx * ny;
    double qmax = 0.0;
    bool bad = false;
    if (!active) {
      if (last_stage && yrow < ny)
        for (int z = z0; z < z1; ++z) {
          const int gi = z * plane + yown * nx + col;
#pragma unroll
          for (int q = 0; q < 5; ++q)
            if (store_lane) Uout.f[q][gi] = U0.f[q][gi];
        }
    } else {
      const double cdt = (a.stage == 1 ? 0.5 : 1.0) * dt;
      const T kx = (T)(cdt * M.inv_dx[0]), ky = (T)(cdt * M.inv_dx[1]), kz = (T)(cdt * M.inv_dx[2]);
      RowPipe5<T> P;
      const int first = z0 - 2;
      const int npush = (z1 - z0) + 4;
      const int own_off = yown * nx + col, halo_off = yhalo * nx + col;
      // loads run one plane ahead of their use (own row, halo row, base state)
      T u_nx[5], uh_nx[5], base_nx[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) uh_nx[q] = base_nx[q] = T(0);
      {
        const int zk = map_index(first, nz, M.bc[2]);
#pragma unroll
        for (int q = 0; q < 5; ++q) u_nx[q] = Uin.f[q][zk * plane + own_off];
      }
      for (int k = 0; k < npush; ++k) {
        // only planes that are assembled need their y-faces (not the 2 + 2 halo planes)
        const bool yplane = k >= 2 && k < npush - 2;
        T u[5], uh[5], base[5], v[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          u[q] = u_nx[q];
          uh[q] = uh_nx[q];
          base[q] = base_nx[q];
        }
        if (k + 1 < npush) {
          const int zn = map_index(first + k + 1, nz, M.bc[2]);
#pragma unroll
          for (int q = 0; q < 5; ++q) u_nx[q] = Uin.f[q][zn * plane + own_off];
          if (has_halo && k + 1 >= 2 && k + 1 < npush - 2) {
#pragma unroll
            for (int q = 0; q < 5; ++q) uh_nx[q] = Uin.f[q][zn * plane + halo_off];
          }
          if (k + 1 >= 4) {  // base of the plane assembled at push k + 1
            const int zb = first + k + 1 - 2;
#pragma unroll
            for (int q = 0; q < 5; ++q) base_nx[q] = U0.f[q][zb * plane + own_off];
          }
        }
        prim_of_cons<T, 3>(u, v, g);
        T* Vs = sV + (k & 1) * vslot;
#pragma unroll
        for (int q = 0; q < 5; ++q) Vs[(q * NR + wave + 2) * 64 + lane] = v[q];
        if (has_halo && yplane) {
          T vh[5];
          prim_of_cons<T, 3>(uh, vh, g);
#pragma unroll
          for (int q = 0; q < 5; ++q) Vs[(q * NR + hrel) * 64 + lane] = vh[q];
        }
        __syncthreads();
        // y-face below this row (LDS rows wave .. wave+3), and above for the last wave
        if (yplane) {
          T vl[5], vr[5], G[5];
#pragma unroll
          for (int q = 0; q < 5; ++q) {
            const T* c = Vs + (q * NR + wave) * 64 + lane;
            face_states(c[0], c[64], c[128], c[192], vl[q], vr[q]);
          }
          hllc<T, 3, 1>(vl, vr, G, g);
          T* Gs = sG + (k % 3) * gslot;
#pragma unroll
          for (int q = 0; q < 5; ++q) Gs[(q * (NW + 1) + wave) * 64 + lane] = G[q];
          if (wave == NW - 1) {
#pragma unroll
            for (int q = 0; q < 5; ++q) {
              const T* c = Vs + (q * NR + wave + 1) * 64 + lane;
              face_states(c[0], c[64], c[128], c[192], vl[q], vr[q]);
            }
            hllc<T, 3, 1>(vl, vr, G, g);
#pragma unroll
            for (int q = 0; q < 5; ++q) Gs[(q * (NW + 1) + NW) * 64 + lane] = G[q];
          }
        }
        // z pipeline of this column; assembles plane first + k - 2
        T accz[5];
        T va[5];
        if (pipe_push5<T>(P, v, k, g, accz, va)) {
          const int zo = first + k - 2;
          T dF[5];
          xflux_diff3<T>(va, g, dF);
          const T* Gs = sG + ((k + 1) % 3) * gslot;  // slot of plane k - 2
          T out[5];
          const int gi = zo * plane + own_off;
#pragma unroll
          for (int q = 0; q < 5; ++q) {
            const T dy = Gs[(q * (NW + 1) + wave) * 64 + lane] - Gs[(q * (NW + 1) + wave + 1) * 64 + lane];
            T acc = kx * dF[q];
            acc += ky * dy;
            acc += kz * accz[q];
            out[q] = base[q] + acc;
          }
          if (store_lane) {
#pragma unroll
            for (int q = 0; q < 5; ++q) Uout.f[q][gi] = out[q];
            if (last_stage && a.cfl) {
              const double qv = cfl_q<T, 3>(out, M.inv_dx, M.gamma);
              bad |= !(qv > 0.0);
              qmax = fmax(qmax, qv);
            }
          }
        }
      }
      __syncthreads();  // LDS reuse by the next item
    }
    if (a.cfl && active && last_stage) cfl_commit(a, t.m, qmax, bad, s_red, (a.ring + 1) % 3);
  }
}

}  // namespace paraiso
