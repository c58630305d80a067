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

// One wave's z-march through one chunk of planes.  Pushes k = 0 .. npush-1
// bring plane first + k; y-faces are formed for planes 2 <= k < npush - 2
// (the assembled ones), and from k = 4 on each push assembles plane
// first + k - 2.  The steady state (both) is unrolled six-fold, so the
// register rings and the LDS slots (plane buffer k mod 2, y-flux ring k mod
// 3) are compile-time in the unrolled body.
template <typename T>
struct PlaneMarch {
  Fields<T, 3> U0, Uin, Uout;
  Gas<T> g;
  T kx, ky, kz;
  double inv_dx[3];
  double gamma;
  int nz, plane, first, bcz;
  unsigned own_bytes, halo_bytes;  // lane offsets of the own and halo rows within a plane
  int wave, NW, NR, lane, hrel;
  bool has_halo, store_lane, cfl;
  T* sV;
  T* sG;
  int vslot, gslot;
  RowPipe5<T> P;
  T u_nx[5], uh_nx[5], base_nx[5];
  double qmax;
  bool bad;

  __device__ __forceinline__ unsigned hide(unsigned b) const {
    asm volatile("" : "+v"(b));
    return b;
  }
  static __device__ __forceinline__ __attribute__((address_space(1))) T* at(
      __attribute__((address_space(1))) T* row, unsigned bytes) {
    return (__attribute__((address_space(1))) T*)((__attribute__((address_space(1))) char*)row + bytes);
  }
  __device__ __forceinline__ int zoff(int k) const { return map_index(first + k, nz, bcz) * plane; }

  // loads of push k (own row, halo row if its y-faces are needed, base of
  // the plane assembled at push k)
  __device__ __forceinline__ void load(int k, bool yp, int npush) {
    const int zo = zoff(k);
    const unsigned ob = hide(own_bytes);
#pragma unroll
    for (int q = 0; q < 5; ++q) u_nx[q] = *at(Uin.f[q] + zo, ob);
    if (has_halo && yp) {
      const unsigned hb = hide(halo_bytes);
#pragma unroll
      for (int q = 0; q < 5; ++q) uh_nx[q] = *at(Uin.f[q] + zo, hb);
    }
    if (k >= 4) {
      const int zb = (first + k - 2) * plane;  // assembled planes lie inside the mesh
#pragma unroll
      for (int q = 0; q < 5; ++q) base_nx[q] = *at(U0.f[q] + zb, ob);
    }
  }

  // push k with V buffer VB = k mod 2 and y-flux slot GB = k mod 3 (compile
  // time in the unrolled steady state, -1: from k); YF: form the y-faces;
  // N: pipeline count (4: four or more)
  template <int VB, int GB, int N, int YF>
  __device__ __forceinline__ void push(int k, int npush) {
    const int vb = VB >= 0 ? VB : (k & 1);
    const int gb = GB >= 0 ? GB : (k % 3);
    const bool yface = YF >= 0 ? (YF != 0) : (k >= 2 && k < npush - 2);
    const int n = N >= 0 ? N : min(k, 4);
    T u[5], uh[5], base[5], v[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      u[q] = u_nx[q];
      uh[q] = uh_nx[q];
      base[q] = base_nx[q];
    }
    if (k + 1 < npush) load(k + 1, k + 1 >= 2 && k + 1 < npush - 2, npush);
    prim_of_cons<T, 3>(u, v, g);
    T* Vs = sV + vb * vslot;
#pragma unroll
    for (int q = 0; q < 5; ++q) Vs[(q * NR + wave + 2) * 64 + lane] = v[q];
    if (has_halo && yface) {
      T vh[5];
      prim_of_cons<T, 3>(uh, vh, g);
#pragma unroll
      for (int q = 0; q < 5; ++q) Vs[(q * NR + hrel) * 64 + lane] = vh[q];
    }
    __syncthreads();
    if (yface) {
      T vl[5], vr[5], G[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const T* c = Vs + (q * NR + wave) * 64 + lane;
        face_states(c[0], c[64], c[128], c[192], vl[q], vr[q]);
      }
      hllc<T, 3, 1>(vl, vr, G, g);
      T* Gs = sG + gb * gslot;
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
    T accz[5], va[5];
    if (pipe_push5<T>(P, v, n, g, accz, va)) {
      const int zo = first + k - 2;
      T dF[5];
      xflux_diff3<T>(va, g, dF);
      const int rb = gb == 0 ? 1 : (gb == 1 ? 2 : 0);  // slot of plane k - 2: (k + 1) mod 3
      const T* Gs = sG + rb * gslot;
      T out[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const T dy = Gs[(q * (NW + 1) + wave) * 64 + lane] - Gs[(q * (NW + 1) + wave + 1) * 64 + lane];
        out[q] = fma(kz, accz[q], fma(ky, dy, fma(kx, dF[q], base[q])));
      }
      if (store_lane) {
        const unsigned ob = hide(own_bytes);
#pragma unroll
        for (int q = 0; q < 5; ++q) *at(Uout.f[q] + zo * plane, ob) = out[q];
        if (cfl) {
          const double qv = cfl_q<T, 3>(out, inv_dx, gamma);
          bad |= !(qv > 0.0);
          qmax = qv > qmax ? qv : qmax;
        }
      }
    }
  }

  __device__ __forceinline__ void run(int npush) {
#pragma unroll
    for (int q = 0; q < 5; ++q) uh_nx[q] = base_nx[q] = T(0);
    load(0, false, npush);
    int k = 0;
    // warm-up and short chunks: run-time phase
#pragma clang loop unroll(disable)
    for (; k < 4 && k < npush; ++k) push<-1, -1, -1, -1>(k, npush);
    // steady state: y-faces and output, k = 4 .. npush - 3, six-fold
    for (; k + 6 <= npush - 2; k += 6) {
      push<0, 1, 4, 1>(k, npush);
      push<1, 2, 4, 1>(k + 1, npush);
      push<0, 0, 4, 1>(k + 2, npush);
      push<1, 1, 4, 1>(k + 3, npush);
      push<0, 2, 4, 1>(k + 4, npush);
      push<1, 0, 4, 1>(k + 5, npush);
    }
#pragma clang loop unroll(disable)
    for (; k < npush; ++k) push<-1, -1, 4, -1>(k, npush);
  }
};

template <typename T, int W>
__global__ void __launch_bounds__(512) PARAISO_WAVES_ATTR(W) k_march3d(Args a, LdsGeom) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double s_red[16];
  __shared__ int s_item;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int NW = blockDim.x >> 6;
  const int NR = NW + 4;            // rows in an LDS plane
  T* sV = reinterpret_cast<T*>(smem);            // [2][5][NR][64]
  T* sG = sV + 2 * 5 * NR * 64;                  // [3][5][NW+1][64]
  ItemLoop it{0, 1};
  for (int item; (item = next_item(a, it, &s_item, a.stage - 1)) >= 0;) {
    item = __builtin_amdgcn_readfirstlane(item);
    const Tile t = tile_of(a, item);
    const MeshDev& M = a.meshes[t.m];
    bool active;
    const double dt = step_dt(a, t.m, active);
    const bool last_stage = a.stage == 2;
    if (last_stage && t.first && threadIdx.x == 0) step_bookkeeping(a, t.m, dt, active);
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
      PlaneMarch<T> S;
      S.U0 = uniform(U0);
      S.Uin = uniform(a.stage == 1 ? U0 : fields<T, 3>(M.w));
      S.Uout = uniform(Uout);
      S.g = gas_of<T>(M);
      S.kx = (T)(cdt * M.inv_dx[0]);
      S.ky = (T)(cdt * M.inv_dx[1]);
      S.kz = (T)(cdt * M.inv_dx[2]);
#pragma unroll
      for (int x = 0; x < 3; ++x) S.inv_dx[x] = M.inv_dx[x];
      S.gamma = M.gamma;
      S.nz = nz;
      S.plane = plane;
      S.first = z0 - 2;
      S.bcz = M.bc[2];
      S.own_bytes = (unsigned)(yown * nx + col) * (unsigned)sizeof(T);
      S.halo_bytes = (unsigned)(yhalo * nx + col) * (unsigned)sizeof(T);
      S.wave = wave;
      S.NW = NW;
      S.NR = NR;
      S.lane = lane;
      S.hrel = hrel;
      S.has_halo = has_halo;
      S.store_lane = store_lane;
      S.cfl = last_stage && a.cfl;
      S.sV = sV;
      S.sG = sG;
      S.vslot = 5 * NR * 64;
      S.gslot = 5 * (NW + 1) * 64;
      S.qmax = 0.0;
      S.bad = false;
      S.run((z1 - z0) + 4);
      qmax = S.qmax;
      bad = S.bad;
      __syncthreads();  // LDS reuse by the next item
    }
    if (a.cfl && active && last_stage) cfl_commit(a, t.m, qmax, bad, s_red, (a.ring + 1) % 3);
  }
}

}  // namespace paraiso
