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
  double qmax;  // every lane; only the stored ones count
  unsigned long long bad;  // lanes that stored a non-physical cell
  unsigned long long store_mask;  // lanes that store

  __device__ __forceinline__ unsigned hide(unsigned b) const {
    asm volatile("" : "+v"(b));
    return b;
  }
  static __device__ __forceinline__ __attribute__((address_space(1))) T* at(
      __attribute__((address_space(1))) T* row, unsigned bytes) {
    return (__attribute__((address_space(1))) T*)((__attribute__((address_space(1))) char*)row + bytes);
  }
  __device__ __forceinline__ int zoff(int k) const { return map_index(first + k, nz, bcz) * plane; }

  // loads of push k: own row, halo row, and the base of the plane assembled
  // at push k.  All unconditional (a wave without a halo row reloads its own
  // row, a push that assembles no plane loads its input plane as the base),
  // so that no register keeps an older load's value across a branch: such a
  // merge would make the next push wait for the loads it has just issued.
  // (Pointing the loads a push does not need at rows the cache holds saves
  // traffic but measured slower.)
  __device__ __forceinline__ void load(int k) {
    const int zo = zoff(k);
    const unsigned ob = hide(own_bytes);
#pragma unroll
    for (int q = 0; q < 5; ++q) u_nx[q] = *at(Uin.f[q] + zo, ob);
    const unsigned hb = hide(halo_bytes);
#pragma unroll
    for (int q = 0; q < 5; ++q) uh_nx[q] = *at(Uin.f[q] + zo, hb);
    const int zb = k >= 4 ? (first + k - 2) * plane : zo;  // assembled planes lie inside the mesh
#pragma unroll
    for (int q = 0; q < 5; ++q) base_nx[q] = *at(U0.f[q] + zb, ob);
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
    if (k + 1 < npush) load(k + 1);
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
      }
      if (cfl) cfl_fold_wave(cfl_q<T, 3>(out, inv_dx, gamma), store_mask, qmax, bad);
    }
  }

  __device__ __forceinline__ void run(int npush) {
#pragma unroll
    for (int q = 0; q < 5; ++q) uh_nx[q] = base_nx[q] = T(0);
    load(0);
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
      S.halo_bytes = has_halo ? (unsigned)(yhalo * nx + col) * (unsigned)sizeof(T) : S.own_bytes;
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
      S.bad = 0;
      S.store_mask = __builtin_amdgcn_ballot_w64(store_lane);
      S.run((z1 - z0) + 4);
      qmax = store_lane ? S.qmax : 0.0;
      bad = S.bad != 0;
      __syncthreads();  // LDS reuse by the next item
    }
    if (a.cfl && active && last_stage) cfl_commit(a, t.m, qmax, bad, s_red, (a.ring + 1) % 3);
  }
}

}  // namespace paraiso

namespace paraiso {

// ---------------------------------------------------------------------------
// Fused 3D register march: both Runge-Kutta stages in one launch, the
// stage-1 state held on chip (the midpoint state of the time-marching
// equations "delayed" rather than stored).
//
// A block of NW waves owns a 56-column strip (64 lanes, 4 halo columns per
// side) and NW stage-1 rows; wave w computes stage 1 on row yb - 2 + w and,
// for 2 <= w < NW - 2, stage 2 on row yb + w - 2, so a block outputs NW - 4
// rows.  Marching along z, push k brings input plane first + k:
//   phase A: the primitives of the wave's own row (waves 0..3 also one of
//            the 4 halo rows) go to the LDS plane V0 (double-buffered), and
//            the stage-1 primitives of plane k - 3, finished in the previous
//            push, to the LDS plane V1 (double-buffered); one barrier;
//   phase B: stage 2 forms the y-faces of V1 plane k - 3 (3-slot ring G2),
//            pushes that plane into its z-pipeline and assembles plane k - 5
//            (base U0, x-faces by lane shifts, y-faces from the ring);
//            stage 1 forms the y-faces of V0 plane k (3-slot ring G1),
//            pushes it into its z-pipeline and assembles plane k - 2, whose
//            primitives wait in registers for the next push's phase A.
// Every face flux of each stage is evaluated once per block; the 4 extra
// stage-1 rows per block are the price of keeping U1 on chip.  Periodic
// meshes only (the stage-1 state of a ghost cell is that of the cell it
// wraps to).
// ---------------------------------------------------------------------------

template <typename T>
struct FusedPlaneMarch {
  Fields<T, 3> U0, Uout;
  Gas<T> g;
  T kx1, ky1, kz1, kx2, ky2, kz2;
  double inv_dx[3];
  double gamma;
  int nz, plane, first, Z;        // Z: output planes of the chunk
  unsigned own_bytes, halo_bytes;
  int wave, NW, lane, hrel;
  bool has_halo, out_wave, store_lane, cfl;
  T* sV0;  // [2][5][NW + 4][64]
  T* sV1;  // [2][5][NW][64]
  T* sG1;  // [3][5][NW + 1][64]
  T* sG2;  // [3][5][NW - 3][64]
  RowPipe5<T> P1, P2;
  T u_nx[5], uh_nx[5], b1_nx[5], b2_nx[5];  // next push's own row, halo row, stage-1 and stage-2 bases
  T v1p[5];                                 // stage-1 primitives of the plane finished last push
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
  __device__ __forceinline__ int zoff(int k) const { return map_index(first + k, nz, kPeriodic) * plane; }

  // loads of push k: own row and halo row of plane k, the bases of the
  // planes assembled in push k (stage 1: k - 2, stage 2: k - 5).  All
  // unconditional, as in the one-stage march (a wave without a halo row
  // reloads its own row; planes wrap, so every index is valid).
  __device__ __forceinline__ void load(int k) {
    const unsigned ob = hide(own_bytes);
    const int zo = zoff(k);
#pragma unroll
    for (int q = 0; q < 5; ++q) u_nx[q] = *at(U0.f[q] + zo, ob);
    const unsigned hb = hide(halo_bytes);
#pragma unroll
    for (int q = 0; q < 5; ++q) uh_nx[q] = *at(U0.f[q] + zo, hb);
    const int z1 = zoff(k - 2);
#pragma unroll
    for (int q = 0; q < 5; ++q) b1_nx[q] = *at(U0.f[q] + z1, ob);
    const int z2 = zoff(k - 5);
#pragma unroll
    for (int q = 0; q < 5; ++q) b2_nx[q] = *at(U0.f[q] + z2, ob);
  }

  __device__ __forceinline__ void push(int k) {
    T u[5], uh[5], b1[5], b2[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      u[q] = u_nx[q];
      uh[q] = uh_nx[q];
      b1[q] = b1_nx[q];
      b2[q] = b2_nx[q];
    }
    if (k + 1 < Z + 9) load(k + 1);
    const int NR = NW + 4;
    // phase A
    T v0[5];
    prim_of_cons<T, 3>(u, v0, g);
    {
      T* V = sV0 + (k & 1) * (5 * NR * 64);
#pragma unroll
      for (int q = 0; q < 5; ++q) V[(q * NR + wave + 2) * 64 + lane] = v0[q];
      if (has_halo && k <= Z + 5) {
        T vh[5];
        prim_of_cons<T, 3>(uh, vh, g);
#pragma unroll
        for (int q = 0; q < 5; ++q) V[(q * NR + hrel) * 64 + lane] = vh[q];
      }
    }
    const bool s2in = k >= 5;  // V1 plane k - 3 exists (stage-1 planes 2 .. Z + 5)
    if (s2in) {
      T* V = sV1 + ((k - 3) & 1) * (5 * NW * 64);
#pragma unroll
      for (int q = 0; q < 5; ++q) V[(q * NW + wave) * 64 + lane] = v1p[q];
    }
    __syncthreads();
    // phase B, stage 2: y-faces of V1 plane k - 3, then assemble plane k - 5
    if (s2in && out_wave) {
      if (k >= 7 && k <= Z + 6) {  // the y-faces of stage-2 planes 4 .. Z + 3
        const T* V = sV1 + ((k - 3) & 1) * (5 * NW * 64);
        T* Gs = sG2 + ((k - 3) % 3) * (5 * (NW - 3) * 64);
        T vl[5], vr[5], G[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const T* c = V + (q * NW + wave - 2) * 64 + lane;
          face_states(c[0], c[64], c[128], c[192], vl[q], vr[q]);
        }
        hllc<T, 3, 1>(vl, vr, G, g);
#pragma unroll
        for (int q = 0; q < 5; ++q) Gs[(q * (NW - 3) + wave - 2) * 64 + lane] = G[q];
        if (wave == NW - 3) {
#pragma unroll
          for (int q = 0; q < 5; ++q) {
            const T* c = V + (q * NW + wave - 1) * 64 + lane;
            face_states(c[0], c[64], c[128], c[192], vl[q], vr[q]);
          }
          hllc<T, 3, 1>(vl, vr, G, g);
#pragma unroll
          for (int q = 0; q < 5; ++q) Gs[(q * (NW - 3) + wave - 1) * 64 + lane] = G[q];
        }
      }
      T dz[5], va[5];
      if (pipe_push5<T>(P2, v1p, k - 5, g, dz, va)) {  // k >= 9: plane k - 5
        T dF[5];
        xflux_diff3<T>(va, g, dF);
        const T* Gs = sG2 + ((k - 5) % 3) * (5 * (NW - 3) * 64);
        T out[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const T dy = Gs[(q * (NW - 3) + wave - 2) * 64 + lane] - Gs[(q * (NW - 3) + wave - 1) * 64 + lane];
          out[q] = fma(kz2, dz[q], fma(ky2, dy, fma(kx2, dF[q], b2[q])));
        }
        if (store_lane) {
          const int zo = zoff(k - 5);
          const unsigned ob = hide(own_bytes);
#pragma unroll
          for (int q = 0; q < 5; ++q) *at(Uout.f[q] + zo, ob) = out[q];
          if (cfl) cfl_fold(cfl_q<T, 3>(out, inv_dx, gamma), qmax, bad);
        }
      }
    }
    // phase B, stage 1: y-faces of V0 plane k, then assemble plane k - 2
    if (k >= 2 && k <= Z + 5) {
      const T* V = sV0 + (k & 1) * (5 * NR * 64);
      T* Gs = sG1 + (k % 3) * (5 * (NW + 1) * 64);
      T vl[5], vr[5], G[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const T* c = V + (q * NR + wave) * 64 + lane;
        face_states(c[0], c[64], c[128], c[192], vl[q], vr[q]);
      }
      hllc<T, 3, 1>(vl, vr, G, g);
#pragma unroll
      for (int q = 0; q < 5; ++q) Gs[(q * (NW + 1) + wave) * 64 + lane] = G[q];
      if (wave == NW - 1) {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const T* c = V + (q * NR + wave + 1) * 64 + lane;
          face_states(c[0], c[64], c[128], c[192], vl[q], vr[q]);
        }
        hllc<T, 3, 1>(vl, vr, G, g);
#pragma unroll
        for (int q = 0; q < 5; ++q) Gs[(q * (NW + 1) + NW) * 64 + lane] = G[q];
      }
    }
    T dz[5], va[5];
    if (k <= Z + 7 && pipe_push5<T>(P1, v0, k < 4 ? k : 4, g, dz, va)) {  // k >= 4: plane k - 2
      T dF[5];
      xflux_diff3<T>(va, g, dF);
      const T* Gs = sG1 + ((k - 2) % 3) * (5 * (NW + 1) * 64);
      T u1[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const T dy = Gs[(q * (NW + 1) + wave) * 64 + lane] - Gs[(q * (NW + 1) + wave + 1) * 64 + lane];
        u1[q] = fma(kz1, dz[q], fma(ky1, dy, fma(kx1, dF[q], b1[q])));
      }
      prim_of_cons<T, 3>(u1, v1p, g);
    }
  }

  __device__ __forceinline__ void run() {
#pragma unroll
    for (int q = 0; q < 5; ++q) uh_nx[q] = b1_nx[q] = b2_nx[q] = v1p[q] = T(0);
    load(0);
#pragma clang loop unroll(disable)
    for (int k = 0; k < Z + 9; ++k) push(k);
  }
};

template <typename T, int W>
__global__ void __launch_bounds__(sizeof(T) == 8 ? 384 : 768) PARAISO_WAVES_ATTR(W) k_march3d_fused(Args a, LdsGeom) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double s_red[16];
  __shared__ int s_item;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int NW = blockDim.x >> 6;
  T* sV0 = reinterpret_cast<T*>(smem);
  T* sV1 = sV0 + 2 * 5 * (NW + 4) * 64;
  T* sG1 = sV1 + 2 * 5 * NW * 64;
  T* sG2 = sG1 + 3 * 5 * (NW + 1) * 64;
  ItemLoop it{0, 1};
  for (int item; (item = next_item(a, it, &s_item, 0)) >= 0;) {
    item = __builtin_amdgcn_readfirstlane(item);
    const Tile t = tile_of(a, item);
    const MeshDev& M = a.meshes[t.m];
    bool active;
    const double dt = step_dt(a, t.m, active);
    if (t.first && threadIdx.x == 0) step_bookkeeping(a, t.m, dt, active);
    const int nx = M.n[0], ny = M.n[1], nz = M.n[2];
    const int x0 = t.org[0], yb = t.org[1], z0 = t.org[2];
    const int z1 = min(z0 + a.tile[2], nz);
    const int col = map_index(x0 - 4 + lane, nx, kPeriodic);
    const bool out_wave = wave >= 2 && wave < NW - 2;
    const int yout = yb + wave - 2;                                // stage-2 row (out_wave)
    const int yown = map_index(yb - 2 + wave, ny, kPeriodic);     // stage-1 row
    // halo rows of V0: waves 0,1 take stage-1 rows -2, -1; waves 2,3 take NW, NW + 1
    const bool has_halo = wave < 4;
    const int hrel = wave < 2 ? wave : NW + wave;                  // LDS row of the halo row
    const int yhalo = map_index(yb - 4 + hrel, ny, kPeriodic);
    const bool store_lane = out_wave && lane >= 4 && lane < 60 && (x0 - 4 + lane) < nx && yout < ny;
    const Fields<T, 3> U0 = fields<T, 3>(M.s[a.src]);
    const Fields<T, 3> Uout = fields<T, 3>(M.s[1 - a.src]);
    const int plane = nx * ny;
    double qmax = 0.0;
    bool bad = false;
    if (!active) {
      if (out_wave && yout < ny) {
        const int gr = yout * nx + col;
        for (int z = z0; z < z1; ++z) {
          const int gi = z * plane + gr;
#pragma unroll
          for (int q = 0; q < 5; ++q)
            if (store_lane) Uout.f[q][gi] = U0.f[q][gi];
        }
      }
    } else {
      FusedPlaneMarch<T> S;
      S.U0 = uniform(U0);
      S.Uout = uniform(Uout);
      S.g = gas_of<T>(M);
      S.kx1 = (T)(0.5 * dt * M.inv_dx[0]);
      S.ky1 = (T)(0.5 * dt * M.inv_dx[1]);
      S.kz1 = (T)(0.5 * dt * M.inv_dx[2]);
      S.kx2 = (T)(dt * M.inv_dx[0]);
      S.ky2 = (T)(dt * M.inv_dx[1]);
      S.kz2 = (T)(dt * M.inv_dx[2]);
#pragma unroll
      for (int x = 0; x < 3; ++x) S.inv_dx[x] = M.inv_dx[x];
      S.gamma = M.gamma;
      S.nz = nz;
      S.plane = plane;
      S.first = z0 - 4;
      S.Z = z1 - z0;
      S.own_bytes = (unsigned)(yown * nx + col) * (unsigned)sizeof(T);
      S.halo_bytes = has_halo ? (unsigned)(yhalo * nx + col) * (unsigned)sizeof(T) : S.own_bytes;
      S.wave = wave;
      S.NW = NW;
      S.lane = lane;
      S.hrel = hrel;
      S.has_halo = has_halo;
      S.out_wave = out_wave;
      S.store_lane = store_lane;
      S.cfl = a.cfl != 0;
      S.sV0 = sV0;
      S.sV1 = sV1;
      S.sG1 = sG1;
      S.sG2 = sG2;
      S.qmax = 0.0;
      S.bad = false;
      S.run();
      qmax = S.qmax;
      bad = S.bad;
      __syncthreads();  // LDS reuse by the next item
    }
    if (a.cfl && active) cfl_commit(a, t.m, qmax, bad, s_red, (a.ring + 1) % 3);
  }
}

}  // namespace paraiso
