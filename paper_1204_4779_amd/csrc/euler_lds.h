// LDS-tile step kernels.
#pragma once

#include "euler_analytic.h"
#include "euler_common.h"

namespace paraiso {

// ---------------------------------------------------------------------------
// LDS-tiled stage and fused step
// ---------------------------------------------------------------------------

constexpr int kMaxR = 8;  // cells per thread kept in registers

// Load U on the region `box` (origin org - H) into LDS primitives.
template <typename T, int D>
__device__ __forceinline__ void lds_load_prims(const MeshDev& M, const Fields<T, D>& U, const Box& box,
                                               const int* org, int H, const Gas<T>& g, T* sV,
                                               int vstride) {
  for (int l = threadIdx.x; l < box.count; l += blockDim.x) {
    int i, j, k;
    box.coords(l, i, j, k);
    const int gi = map_index(org[0] - H + i, M.n[0], M.bc[0]);
    const int gj = D > 1 ? map_index(org[1] - H + j, M.n[1], M.bc[1]) : 0;
    const int gk = D > 2 ? map_index(org[2] - H + k, M.n[2], M.bc[2]) : 0;
    const int gc = gidx(M, gi, gj, gk);
    T u[D + 2], v[D + 2];
#pragma unroll
    for (int q = 0; q < D + 2; ++q) u[q] = U.f[q][gc];
    prim_of_cons<T, D>(u, v, g);
#pragma unroll
    for (int q = 0; q < D + 2; ++q) sV[q * vstride + l] = v[q];
  }
}

// Analytic boundaries: after lds_load_prims (which wraps such axes), the
// cells of the box outside the mesh on an analytic axis take the exact
// solution at their centres and time t_ghost (the time the stage's input
// stands for).  Each position is rewritten by the thread that loaded it.
template <typename T, int D>
__device__ __forceinline__ void lds_analytic_ghosts(const MeshDev& M, const Box& box, const int* org, int H, T* sV,
                                                 int vstride, double t_ghost) {
  for (int l = threadIdx.x; l < box.count; l += blockDim.x) {
    int i, j, k;
    box.coords(l, i, j, k);
    const int r[3] = {org[0] - H + i, D > 1 ? org[1] - H + j : 0, D > 2 ? org[2] - H + k : 0};
    bool ghost = false;
#pragma unroll
    for (int a = 0; a < D; ++a) ghost |= M.bc[a] == kAnalytic && (r[a] < 0 || r[a] >= M.n[a]);
    if (ghost) {
      T v[D + 2];
      exact_prims<T, D>(M, (r[0] + 0.5) * M.dx[0], D > 1 ? (r[1] + 0.5) * M.dx[1] : 0.0, t_ghost, v);
#pragma unroll
      for (int q = 0; q < D + 2; ++q) sV[q * vstride + l] = v[q];
    }
  }
}

// Does the box reach outside the mesh on an analytic axis?
template <int D>
__device__ __forceinline__ bool box_meets_analytic(const MeshDev& M, const Box& box, const int* org, int H) {
  bool meets = false;
#pragma unroll
  for (int a = 0; a < D; ++a)
    meets |= M.bc[a] == kAnalytic && (org[a] - H < 0 || org[a] - H + box.e[a] > M.n[a]);
  return meets;
}

// Options of the LDS-tile kernels, one instantiation each (bit mask).
constexpr int kOptAnalytic = 1;    // exact-solution ghosts on analytic axes
constexpr int kOptFirstOrder = 2;  // piecewise-constant reconstruction

// Face fluxes along AX for the faces in `faces` (face (i,j,k) lies on the
// lower side of cell (i,j,k) of the cell box that starts `off` cells into
// the V region).  Reads sV, writes sF.  FIRST: the face takes the values of
// the two cells beside it (first-order reconstruction).
template <typename T, int D, int AX, bool FIRST = false>
__device__ __forceinline__ void lds_fluxes(const Box& faces, const Box& vbox, int off, const T* sV,
                                           int vstride, T* sF, int fstride, const Gas<T>& g) {
  const int s = AX == 0 ? 1 : (AX == 1 ? vbox.e[0] : vbox.e[0] * vbox.e[1]);
  for (int l = threadIdx.x; l < faces.count; l += blockDim.x) {
    int i, j, k;
    faces.coords(l, i, j, k);
    const int c = ((k + (D > 2 ? off : 0)) * vbox.e[1] + (j + (D > 1 ? off : 0))) * vbox.e[0] + i + off;
    T vl[D + 2], vr[D + 2], f[D + 2];
#pragma unroll
    for (int q = 0; q < D + 2; ++q) {
      const T* y = sV + q * vstride + c;
      if constexpr (FIRST) {
        vl[q] = y[-s];
        vr[q] = y[0];
      } else {
        face_states(y[-2 * s], y[-s], y[0], y[s], vl[q], vr[q]);
      }
    }
    hllc<T, D, AX>(vl, vr, f, g);
#pragma unroll
    for (int q = 0; q < D + 2; ++q) sF[q * fstride + l] = f[q];
  }
}

// acc[r] += coef (F[lower face] - F[upper face]) for the cells a thread owns.
template <typename T, int D, int AX>
__device__ __forceinline__ void lds_accumulate(const Box& cells, const Box& faces, const T* sF, int fstride,
                                               T coef, T (*acc)[D + 2]) {
  const int s = AX == 0 ? 1 : (AX == 1 ? faces.e[0] : faces.e[0] * faces.e[1]);
#pragma unroll
  for (int r = 0; r < kMaxR; ++r) {
    const int l = threadIdx.x + r * blockDim.x;
    if (l < cells.count) {
      int i, j, k;
      cells.coords(l, i, j, k);
      const int f = (k * faces.e[1] + j) * faces.e[0] + i;
#pragma unroll
      for (int q = 0; q < D + 2; ++q) acc[r][q] += coef * (sF[q * fstride + f] - sF[q * fstride + f + s]);
    }
  }
}

// Manifest choices of the LDS-tile kernels (what a tile keeps in LDS
// between the phases of an axis; the paper's Manifest/Delayed annotation of
// the interpolation and Riemann-solver results):
constexpr int kKeepFluxes = 0;  // face fluxes, each face's states formed where its flux is
constexpr int kKeepStates = 1;  // face states; each cell then solves both its faces
constexpr int kKeepBoth = 2;    // face states, then face fluxes

// Face values of every cell from the left neighbour of the first face in
// `faces` to the right neighbour of the last (along AX): sLo = value on the
// cell's lower face, sUp = on its upper face, indexed like sV.  The same
// arithmetic as face_states, so every later result is bitwise unchanged.
template <typename T, int D, int AX>
__device__ __forceinline__ void lds_face_values(const Box& faces, const Box& vbox, int off, const T* sV,
                                                int vstride, T* sLo, T* sUp) {
  const int s = AX == 0 ? 1 : (AX == 1 ? vbox.e[0] : vbox.e[0] * vbox.e[1]);
  int e[3] = {faces.e[0], faces.e[1], faces.e[2]};
  e[AX] += 1;
  const Box cellbox = make_box_dev(e[0], e[1], e[2]);
  for (int l = threadIdx.x; l < cellbox.count; l += blockDim.x) {
    int i, j, k;
    cellbox.coords(l, i, j, k);
    const int c = ((k + (D > 2 ? off : 0)) * vbox.e[1] + (j + (D > 1 ? off : 0))) * vbox.e[0] + i + off - s;
#pragma unroll
    for (int q = 0; q < D + 2; ++q) {
      const T* y = sV + q * vstride + c;
      const T half = T(0.5) * minmod(y[0] - y[-s], y[s] - y[0]);
      sLo[q * vstride + c] = y[0] - half;
      sUp[q * vstride + c] = y[0] + half;
    }
  }
}

// Face fluxes along AX from kept face values.
template <typename T, int D, int AX>
__device__ __forceinline__ void lds_fluxes_kept(const Box& faces, const Box& vbox, int off, const T* sLo,
                                                const T* sUp, int vstride, T* sF, int fstride, const Gas<T>& g) {
  const int s = AX == 0 ? 1 : (AX == 1 ? vbox.e[0] : vbox.e[0] * vbox.e[1]);
  for (int l = threadIdx.x; l < faces.count; l += blockDim.x) {
    int i, j, k;
    faces.coords(l, i, j, k);
    const int c = ((k + (D > 2 ? off : 0)) * vbox.e[1] + (j + (D > 1 ? off : 0))) * vbox.e[0] + i + off;
    T vl[D + 2], vr[D + 2], f[D + 2];
#pragma unroll
    for (int q = 0; q < D + 2; ++q) {
      vl[q] = sUp[q * vstride + c - s];
      vr[q] = sLo[q * vstride + c];
    }
    hllc<T, D, AX>(vl, vr, f, g);
#pragma unroll
    for (int q = 0; q < D + 2; ++q) sF[q * fstride + l] = f[q];
  }
}

// acc[r] += coef (F[lower face] - F[upper face]) with both face fluxes of
// each cell solved by the cell itself from kept face values (each face twice).
template <typename T, int D, int AX>
__device__ __forceinline__ void lds_accumulate_solving(const Box& cells, const Box& vbox, int off, const T* sLo,
                                                       const T* sUp, int vstride, const Gas<T>& g, T coef,
                                                       T (*acc)[D + 2]) {
  const int s = AX == 0 ? 1 : (AX == 1 ? vbox.e[0] : vbox.e[0] * vbox.e[1]);
#pragma unroll
  for (int r = 0; r < kMaxR; ++r) {
    const int l = threadIdx.x + r * blockDim.x;
    if (l < cells.count) {
      int i, j, k;
      cells.coords(l, i, j, k);
      const int c = ((k + (D > 2 ? off : 0)) * vbox.e[1] + (j + (D > 1 ? off : 0))) * vbox.e[0] + i + off;
      T vl[D + 2], vr[D + 2], flo[D + 2], fup[D + 2];
#pragma unroll
      for (int q = 0; q < D + 2; ++q) {
        vl[q] = sUp[q * vstride + c - s];
        vr[q] = sLo[q * vstride + c];
      }
      hllc<T, D, AX>(vl, vr, flo, g);
#pragma unroll
      for (int q = 0; q < D + 2; ++q) {
        vl[q] = sUp[q * vstride + c];
        vr[q] = sLo[q * vstride + c + s];
      }
      hllc<T, D, AX>(vl, vr, fup, g);
#pragma unroll
      for (int q = 0; q < D + 2; ++q) acc[r][q] += coef * (flo[q] - fup[q]);
    }
  }
}

// One axis of the LDS-tile update: fluxes of the faces along AX, summed into acc.
template <typename T, int D, int AX, bool FIRST, int KEEP>
__device__ __forceinline__ void lds_axis(const LdsGeom& G, const Box& cells, const Box& faces, const Box& vbox,
                                         int off, const T* sV, T* sF, T* sKeep, const Gas<T>& g, T coef,
                                         T (*acc)[D + 2]) {
  if constexpr (KEEP == kKeepFluxes) {
    lds_fluxes<T, D, AX, FIRST>(faces, vbox, off, sV, G.vstride, sF, G.fstride, g);
    __syncthreads();
    lds_accumulate<T, D, AX>(cells, faces, sF, G.fstride, coef, acc);
  } else {
    T* sLo = sKeep;
    T* sUp = sKeep + (D + 2) * G.vstride;
    lds_face_values<T, D, AX>(faces, vbox, off, sV, G.vstride, sLo, sUp);
    __syncthreads();
    if constexpr (KEEP == kKeepBoth) {
      lds_fluxes_kept<T, D, AX>(faces, vbox, off, sLo, sUp, G.vstride, sF, G.fstride, g);
      __syncthreads();
      lds_accumulate<T, D, AX>(cells, faces, sF, G.fstride, coef, acc);
    } else {
      lds_accumulate_solving<T, D, AX>(cells, vbox, off, sLo, sUp, G.vstride, g, coef, acc);
    }
  }
}

template <typename T, int D, bool FIRST = false, int KEEP = kKeepFluxes>
__device__ __forceinline__ void lds_all_axes(const LdsGeom& G, const Box& cells, const Box* faces,
                                             const Box& vbox, int off, const T* sV, T* sF,
                                             const Gas<T>& g, const T* coef, T (*acc)[D + 2],
                                             T* sKeep = nullptr) {
  lds_axis<T, D, 0, FIRST, KEEP>(G, cells, faces[0], vbox, off, sV, sF, sKeep, g, coef[0], acc);
  if constexpr (D > 1) {
    __syncthreads();
    lds_axis<T, D, 1, FIRST, KEEP>(G, cells, faces[1], vbox, off, sV, sF, sKeep, g, coef[1], acc);
  }
  if constexpr (D > 2) {
    __syncthreads();
    lds_axis<T, D, 2, FIRST, KEEP>(G, cells, faces[2], vbox, off, sV, sF, sKeep, g, coef[2], acc);
  }
}

// Unfused LDS stage: U_out = U0 + cdt L(U_in) on the tile.  OPT (kOpt*
// bits): analytic ghosts, first-order reconstruction; separate
// instantiations keep the plain kernel's code and registers.
template <typename T, int D, int W, int OPT = 0, int KEEP = kKeepFluxes>
__global__ void __launch_bounds__(512) PARAISO_WAVES_ATTR(W) k_stage_lds(Args a, LdsGeom G) {
  constexpr bool AN = (OPT & kOptAnalytic) != 0;
  constexpr bool FIRST = (OPT & kOptFirstOrder) != 0;
  static_assert(KEEP == kKeepFluxes || OPT == 0, "kept face states: plain second-order kernel only");
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double s_red[16];
  __shared__ int s_item;
  T* sV = reinterpret_cast<T*>(smem);
  T* sF = sV + (D + 2) * G.vstride;
  ItemLoop it{0, 1};
  for (int item; (item = next_item(a, it, &s_item, a.stage - 1)) >= 0;) {
    const Tile t = tile_of(a, item);
    const MeshDev& M = a.meshes[t.m];
    bool active;
    const double dt = step_dt(a, t.m, active);
    if (a.stage == 2 && t.first && threadIdx.x == 0) step_bookkeeping(a, t.m, dt, active);
    if (!active && a.stage == 1) continue;
    const Gas<T> g = gas_of<T>(M);
    const double cdt = (a.stage == 1 ? 0.5 : 1.0) * dt;
    T coef[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) coef[ax] = (T)(cdt * M.inv_dx[ax]);
    const Fields<T, D> U0 = fields<T, D>(M.s[a.src]);
    const Fields<T, D> Uin = a.stage == 1 ? U0 : fields<T, D>(M.w);
    const Fields<T, D> Uout = a.stage == 1 ? fields<T, D>(M.w) : fields<T, D>(M.s[1 - a.src]);

    T acc[kMaxR][D + 2];
#pragma unroll
    for (int r = 0; r < kMaxR; ++r)
#pragma unroll
      for (int q = 0; q < D + 2; ++q) acc[r][q] = T(0);
    if (active) {
      __syncthreads();  // previous item's readers of sV / sF are done
      lds_load_prims<T, D>(M, Uin, G.vin, t.org, G.halo, g, sV, G.vstride);
      if constexpr (AN) {
        // stage 1 reads U0 at time t, stage 2 the midpoint state at t + dt/2
        if (box_meets_analytic<D>(M, G.vin, t.org, G.halo)) {
          const double t_ghost = a.ctl[t.m].t[a.ring] + (a.stage == 2 ? 0.5 * dt : 0.0);
          lds_analytic_ghosts<T, D>(M, G.vin, t.org, G.halo, sV, G.vstride, t_ghost);
        }
      }
      __syncthreads();
      lds_all_axes<T, D, FIRST, KEEP>(G, G.tile, G.fx, G.vin, G.halo, sV, sF, g, coef, acc,
                                      sF + (D + 2) * G.fstride);
    }
    double qmax = 0.0;
    bool bad = false;
#pragma unroll
    for (int r = 0; r < kMaxR; ++r) {
      const int l = threadIdx.x + r * blockDim.x;
      if (l < G.tile.count) {
        int li, lj, lk;
        G.tile.coords(l, li, lj, lk);
        const int i = t.org[0] + li, j = t.org[1] + lj, k = t.org[2] + lk;
        if (i < M.n[0] && j < M.n[1] && k < M.n[2]) {
          const int gc = gidx(M, i, j, k);
          T out[D + 2];
#pragma unroll
          for (int q = 0; q < D + 2; ++q) {
            out[q] = U0.f[q][gc] + acc[r][q];
            Uout.f[q][gc] = out[q];
          }
          if (a.cfl && active) {
            cfl_fold(cfl_q<T, D>(out, M.inv_dx, M.gamma), qmax, bad);
          }
        }
      }
    }
    if (a.cfl && active) cfl_commit(a, t.m, qmax, bad, s_red, (a.ring + 1) % 3);
  }
}

// Fused LDS step: V0 on tile+4 -> stage 1 on tile+2 (kept in LDS) -> stage 2
// on the tile.  Outflow: stage-1 values outside the mesh are replaced by the
// edge cell's stage-1 value, which is what filling ghost cells of U1 does.
// OPT: kOptFirstOrder or 0 (analytic boundaries need the unfused kernel).
template <typename T, int D, int W, int OPT = 0, int KEEP = kKeepFluxes>
__global__ void __launch_bounds__(512) PARAISO_WAVES_ATTR(W) k_fused_lds(Args a, LdsGeom G) {
  constexpr bool FIRST = (OPT & kOptFirstOrder) != 0;
  static_assert(KEEP == kKeepFluxes || OPT == 0, "kept face states: plain second-order kernel only");
  static_assert((OPT & kOptAnalytic) == 0, "analytic ghosts run on the unfused kernel");
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double s_red[16];
  __shared__ int s_item;
  T* sV = reinterpret_cast<T*>(smem);
  T* sF = sV + (D + 2) * G.vstride;
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
    T acc[kMaxR][D + 2];
#pragma unroll
    for (int r = 0; r < kMaxR; ++r)
#pragma unroll
      for (int q = 0; q < D + 2; ++q) acc[r][q] = T(0);
    if (active) {
      // ---- stage 1 on tile + 2 ----
      __syncthreads();
      lds_load_prims<T, D>(M, U0, G.vin, t.org, 4, g, sV, G.vstride);
      __syncthreads();
      lds_all_axes<T, D, FIRST, KEEP>(G, G.c1, G.fx, G.vin, 2, sV, sF, g, coef1, acc, sF + (D + 2) * G.fstride);
      __syncthreads();  // all stage-1 readers of V0 done: sV now holds V1 on tile + 2
#pragma unroll
      for (int r = 0; r < kMaxR; ++r) {
        const int l = threadIdx.x + r * blockDim.x;
        if (l < G.c1.count) {
          int li, lj, lk;
          G.c1.coords(l, li, lj, lk);
          const int gi = map_index(t.org[0] - 2 + li, M.n[0], M.bc[0]);
          const int gj = D > 1 ? map_index(t.org[1] - 2 + lj, M.n[1], M.bc[1]) : 0;
          const int gk = D > 2 ? map_index(t.org[2] - 2 + lk, M.n[2], M.bc[2]) : 0;
          const int gc = gidx(M, gi, gj, gk);
          T u1[D + 2], v1[D + 2];
#pragma unroll
          for (int q = 0; q < D + 2; ++q) u1[q] = U0.f[q][gc] + acc[r][q];
          prim_of_cons<T, D>(u1, v1, g);
#pragma unroll
          for (int q = 0; q < D + 2; ++q) sV[q * G.vstride + l] = v1[q];
        }
      }
      __syncthreads();
      // outflow: positions outside the mesh take the edge cell's stage-1 state
      bool any_outflow = false;
#pragma unroll
      for (int ax = 0; ax < D; ++ax) any_outflow |= (M.bc[ax] == kOutflow);
      if (any_outflow) {
        for (int l = threadIdx.x; l < G.c1.count; l += blockDim.x) {
          int li, lj, lk;
          G.c1.coords(l, li, lj, lk);
          const int p[3] = {t.org[0] - 2 + li, t.org[1] - 2 + lj, t.org[2] - 2 + lk};
          int src[3] = {li, lj, lk};
          bool moved = false;
#pragma unroll
          for (int ax = 0; ax < D; ++ax) {
            if (M.bc[ax] == kOutflow && (p[ax] < 0 || p[ax] >= M.n[ax])) {
              const int cp = p[ax] < 0 ? 0 : M.n[ax] - 1;
              src[ax] = cp - (t.org[ax] - 2);
              moved = true;
            }
          }
          if (moved) {
            const int sl = (src[2] * G.c1.e[1] + src[1]) * G.c1.e[0] + src[0];
            T v[D + 2];
#pragma unroll
            for (int q = 0; q < D + 2; ++q) v[q] = sV[q * G.vstride + sl];
            // sources lie inside the mesh and are never themselves moved, so
            // reads and writes of this pass touch disjoint positions
#pragma unroll
            for (int q = 0; q < D + 2; ++q) sV[q * G.vstride + l] = v[q];
          }
        }
      }
      __syncthreads();
      // ---- stage 2 on the tile ----
#pragma unroll
      for (int r = 0; r < kMaxR; ++r)
#pragma unroll
        for (int q = 0; q < D + 2; ++q) acc[r][q] = T(0);
      lds_all_axes<T, D, FIRST, KEEP>(G, G.tile, G.fx2, G.c1, 2, sV, sF, g, coef2, acc, sF + (D + 2) * G.fstride);
    }
    double qmax = 0.0;
    bool bad = false;
#pragma unroll
    for (int r = 0; r < kMaxR; ++r) {
      const int l = threadIdx.x + r * blockDim.x;
      if (l < G.tile.count) {
        int li, lj, lk;
        G.tile.coords(l, li, lj, lk);
        const int i = t.org[0] + li, j = t.org[1] + lj, k = t.org[2] + lk;
        if (i < M.n[0] && j < M.n[1] && k < M.n[2]) {
          const int gc = gidx(M, i, j, k);
          T out[D + 2];
#pragma unroll
          for (int q = 0; q < D + 2; ++q) {
            out[q] = U0.f[q][gc] + (active ? acc[r][q] : T(0));
            Uout.f[q][gc] = out[q];
          }
          if (a.cfl && active) {
            cfl_fold(cfl_q<T, D>(out, M.inv_dx, M.gamma), qmax, bad);
          }
        }
      }
    }
    if (a.cfl && active) cfl_commit(a, t.m, qmax, bad, s_red, (a.ring + 1) % 3);
  }
}

}  // namespace paraiso
