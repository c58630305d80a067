// HIP kernels of the Euler step (gfx950, wave64).
//
// Work is split into items: one item is one tile of one mesh, so a single
// mesh and a batch of uneven meshes go through the same kernels.  A kernel
// either maps its blocks onto items (XCD-aware: the 8 XCDs each get a
// contiguous run of tiles so halo re-reads hit the same L2) or, in the
// persistent form, runs a few blocks per CU that pull items from 8 per-XCD
// queues and steal from the others once their own is drained.
//
// Device-resident time stepping (paraiso_advance): each mesh has a control
// block with 3-slot rings for t, the step count and the CFL maximum.  Step n
// reads slot n%3, the block owning tile 0 of the mesh writes slot (n+1)%3 of
// t and the step count and clears slot (n+2)%3 of the maximum, and every
// block folds its cells' CFL terms of the new state into slot (n+1)%3 with an
// integer atomic max on the FP64 bit pattern (positive doubles order like
// their bits).  No grid barrier is needed.
#pragma once

#include "euler_device.h"

namespace paraiso {

// Problem whose exact solution fills the ghost cells of analytic boundaries
// (the paper's convergence tests, on the unit square): a function of
// s = (x - 1/2) cs + (y - 1/2) sn + 1/2 with the velocity along (cs, sn).
struct Analytic {
  int kind;              // 0 none, 1 entropy wave, 2 sound wave, 3 shock tube
  int pad_;
  double cs, sn;         // direction of the wave normal / tube axis
  double amp;            // sound-wave amplitude
  double ps, us;         // shock tube: star pressure and velocity (host-computed)
};

struct MeshDev {
  void* s[2][kMaxFields];  // the caller's two state buffers
  void* w[kMaxFields];     // stage-1 state (unfused variants), in the workspace
  int n[3];
  int bc[3];
  int nt[3];               // tiles per axis
  int item0;               // first item of this mesh
  int nitems;
  int chunk0;              // first cell chunk of this mesh (CFL and totals reductions)
  int nchunks;
  int ncells;
  int pad_;
  double dx[3];
  double inv_dx[3];
  double gamma;
  double inv_gm1;          // 1 / (gamma - 1)
  double vol;              // cell volume
  Analytic an;             // for meshes with an analytic boundary
};

// Exact primitive state of M.an at point (x, y) and time t, in FP64:
//   entropy wave  rho = 2 + sin 2 pi (s - t), v_n = 1, p = 1;
//   sound wave    w = A sin 2 pi (s - t): rho = gamma (1 + w), v_n = w,
//                 p = 1 + gamma w (a right-going acoustic wave, sound speed 1);
//   shock tube    (1, 0, 1) | (0.125, 0, 0.1) at s = 1/2, the exact Riemann
//                 solution at (s - 1/2)/t: left state, left fan, left and
//                 right star states, right fan or shock, right state.
__device__ inline void riemann_side(double gamma, double rk, double uk, double pk, double ps, double us,
                                    double xi, double sgn, double* o) {
  // sgn = +1 for the left wave (sampled where xi <= u*), -1 for the right one
  const double ck = sqrt(gamma * pk / rk);
  const double g1 = (gamma - 1.0) / (gamma + 1.0);
  if (ps > pk) {  // shock
    const double sk = uk - sgn * ck * sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pk + (gamma - 1.0) / (2.0 * gamma));
    if (sgn * (xi - sk) <= 0.0) {
      o[0] = rk; o[1] = uk; o[2] = pk;
    } else {
      o[0] = rk * (ps / pk + g1) / (g1 * ps / pk + 1.0); o[1] = us; o[2] = ps;
    }
  } else {        // rarefaction
    const double head = uk - sgn * ck;
    const double tail = us - sgn * ck * pow(ps / pk, (gamma - 1.0) / (2.0 * gamma));
    if (sgn * (xi - head) <= 0.0) {
      o[0] = rk; o[1] = uk; o[2] = pk;
    } else if (sgn * (xi - tail) > 0.0) {
      o[0] = rk * pow(ps / pk, 1.0 / gamma); o[1] = us; o[2] = ps;
    } else {
      const double c = 2.0 / (gamma + 1.0) * (ck + sgn * 0.5 * (gamma - 1.0) * (uk - xi));
      o[0] = rk * pow(c / ck, 2.0 / (gamma - 1.0));
      o[1] = 2.0 / (gamma + 1.0) * (sgn * ck + 0.5 * (gamma - 1.0) * uk + xi);
      o[2] = pk * pow(c / ck, 2.0 * gamma / (gamma - 1.0));
    }
  }
}

template <typename T, int D>
__device__ inline void exact_prims(const MeshDev& M, double x, double y, double t, T* v) {
  const Analytic& A = M.an;
  const double s = (x - 0.5) * A.cs + (D > 1 ? (y - 0.5) * A.sn : 0.0) + 0.5;
  const double two_pi = 6.283185307179586;
  double rho, vn, p;
  if (A.kind == 1) {
    rho = 2.0 + sin(two_pi * (s - t));
    vn = 1.0;
    p = 1.0;
  } else if (A.kind == 2) {
    const double w = A.amp * sin(two_pi * (s - t));
    rho = M.gamma * (1.0 + w);
    vn = w;
    p = 1.0 + M.gamma * w;
  } else {
    double o[3];
    if (!(t > 0.0)) {
      o[0] = s < 0.5 ? 1.0 : 0.125; o[1] = 0.0; o[2] = s < 0.5 ? 1.0 : 0.1;
    } else {
      const double xi = (s - 0.5) / t;
      if (xi <= A.us)
        riemann_side(M.gamma, 1.0, 0.0, 1.0, A.ps, A.us, xi, 1.0, o);
      else
        riemann_side(M.gamma, 0.125, 0.0, 0.1, A.ps, A.us, xi, -1.0, o);
    }
    rho = o[0]; vn = o[1]; p = o[2];
  }
  v[0] = (T)rho;
  v[1] = (T)(vn * A.cs);
  if constexpr (D > 1) v[2] = (T)(vn * A.sn);
  if constexpr (D > 2) v[3] = T(0);
  v[D + 1] = (T)p;
}

struct Ctl {
  double t[3];
  unsigned long long qbits[3];
  long long steps[3];
  int flags;  // bit 0: non-physical or non-finite state seen
  int pad_;
};

struct Params {
  double t_end;
  double cfl;
  long long max_steps;
};

struct Args {
  const MeshDev* meshes;
  Ctl* ctl;
  const Params* prm;
  const double* dt;        // per-mesh explicit dt (device), or null: device-resident dt
  unsigned int* queue;     // [3 ring slots][2 launch kinds][8 XCD queues]
  double* partials;        // totals: [item][kMaxFields]
  int nmeshes;
  int nitems;
  int tile[3];
  int src;                 // buffer holding U0
  int ring;                // ring slot of this step
  int stage;               // unfused: 1 or 2; fused: 0
  int cfl;                 // 1: fold the CFL term of the output state (stage 2 / fused)
  int persistent;
  int xcd_begin[9];        // item partition over the 8 XCD queues
};

// ---------------------------------------------------------------------------
// item scheduling
// ---------------------------------------------------------------------------

// Contiguous run of items for the XCD that block b lands on (blocks are
// dispatched round-robin over the 8 XCDs).
__device__ __forceinline__ int xcd_item(int b, int nitems) {
  const int per = nitems >> 3, rem = nitems & 7;
  const int x = b & 7, slot = b >> 3;
  return x * per + (x < rem ? x : rem) + slot;
}

struct ItemLoop {
  int home;
  int first;
};

__device__ __forceinline__ int next_item(const Args& a, ItemLoop& it, int* s_item, int kind) {
  if (!a.persistent) {
    if (!it.first) return -1;
    it.first = 0;
    return xcd_item((int)blockIdx.x, a.nitems);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned int* q = a.queue + (a.ring * 2 + kind) * 8;
    int item = -1;
    while (it.home < 8) {
      const int x = ((int)blockIdx.x + it.home) & 7;
      const unsigned cnt = (unsigned)(a.xcd_begin[x + 1] - a.xcd_begin[x]);
      if (cnt > 0u) {
        const unsigned idx = atomicAdd(q + x, 1u);
        if (idx < cnt) {
          item = a.xcd_begin[x] + (int)idx;
          break;
        }
      }
      ++it.home;
    }
    *s_item = item;
  }
  __syncthreads();
  return *s_item;
}

__device__ __forceinline__ int find_mesh(const MeshDev* ms, int nm, int item) {
  int lo = 0, hi = nm - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ms[mid].item0 <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Per-block view of one item.
struct Tile {
  int m;
  int org[3];  // global index of the tile's first cell
  bool first;  // tile 0 of its mesh
};

__device__ __forceinline__ Tile tile_of(const Args& a, int item) {
  Tile t;
  t.m = find_mesh(a.meshes, a.nmeshes, item);
  const MeshDev& M = a.meshes[t.m];
  const int local = item - M.item0;
  const int tx = local % M.nt[0];
  const int r = local / M.nt[0];
  const int ty = r % M.nt[1];
  const int tz = r / M.nt[1];
  t.org[0] = tx * a.tile[0];
  t.org[1] = ty * a.tile[1];
  t.org[2] = tz * a.tile[2];
  t.first = (local == 0);
  return t;
}

// dt of mesh m for this step; `active` false once t >= t_end or the step
// budget is spent (the step then copies U0 to the output).
__device__ __forceinline__ double step_dt(const Args& a, int m, bool& active) {
  if (a.dt) {
    active = true;
    return a.dt[m];
  }
  const Ctl& c = a.ctl[m];
  const double t = c.t[a.ring];
  const long long st = c.steps[a.ring];
  active = (t < a.prm->t_end) && (st < a.prm->max_steps);
  if (!active) return 0.0;
  double dt = a.prm->cfl / __longlong_as_double((long long)c.qbits[a.ring]);
  if (dt > a.prm->t_end - t) dt = a.prm->t_end - t;
  return dt;
}

// Ring bookkeeping done once per mesh and step by the block owning tile 0.
__device__ __forceinline__ void step_bookkeeping(const Args& a, int m, double dt, bool active) {
  const int nx = (a.ring + 1) % 3, nn = (a.ring + 2) % 3;
  Ctl& c = a.ctl[m];
  // t and the step count advance with explicit steps too (analytic
  // boundaries read the time)
  c.t[nx] = active ? c.t[a.ring] + dt : c.t[a.ring];
  c.steps[nx] = c.steps[a.ring] + (active ? 1 : 0);
  if (!a.dt) c.qbits[nn] = 0ull;
  if (m == 0 && a.queue) {
#pragma unroll
    for (int k = 0; k < 16; ++k) a.queue[nn * 16 + k] = 0u;
  }
}

// Block-wide max of a double (all threads call; result valid in thread 0).
__device__ __forceinline__ double block_max(double v, double* s_red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) s_red[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int k = 1; k < nw; ++k) v = fmax(v, s_red[k]);
  }
  return v;
}

// Fold a block's CFL maximum (and its non-physical flag) into mesh m's ring.
__device__ __forceinline__ void cfl_commit(const Args& a, int m, double qmax, bool bad, double* s_red,
                                           int slot) {
  const double v = block_max(bad ? -1.0 : qmax, s_red);
  // any thread's bad flag: encoded as a negative maximum is not enough (max
  // ignores it), so flag separately
  if (bad) atomicOr(&a.ctl[m].flags, 1);
  if (threadIdx.x == 0 && v > 0.0)
    atomicMax(&a.ctl[m].qbits[slot], (unsigned long long)__double_as_longlong(v));
}

// Tile geometry handed to the LDS kernels (computed on the host).
struct LdsGeom {
  Box vin;      // primitive region loaded (tile + halo H)
  Box c1;       // stage-1 cells (fused: tile + 2) / the tile (unfused)
  Box tile;     // output cells
  Box fx[3];    // stage-1 faces per axis (fused) / faces per axis (unfused)
  Box fx2[3];   // stage-2 faces per axis (fused)
  int halo;     // H: 4 fused, 2 unfused
  int vstride;  // fields stride in the V region (elements)
  int fstride;  // fields stride in the flux buffer
  int rows;     // 2D register march: rows per wave
};

template <typename T, int D>
struct Fields {
  // field arrays live in device global memory: typing them so lets the
  // compiler emit global (not flat) loads and stores
  __attribute__((address_space(1))) T* f[D + 2];
};

// The same field pointers moved to scalar registers.  They are read from
// the mesh table in global memory, which the compiler must load per lane
// (the kernel writes global memory); every lane holds the same values, so
// reading them from the first lane is exact, and scalar bases let each
// access use the scalar-base form with a 32-bit lane offset.
template <typename T, int D>
__device__ __forceinline__ Fields<T, D> uniform(Fields<T, D> f) {
#pragma unroll
  for (int q = 0; q < D + 2; ++q) {
    const unsigned long long v = (unsigned long long)f.f[q];
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    f.f[q] = (__attribute__((address_space(1))) T*)(((unsigned long long)hi << 32) | lo);
  }
  return f;
}

template <typename T, int D>
__device__ __forceinline__ Fields<T, D> fields(void* const* p) {
  Fields<T, D> r;
#pragma unroll
  for (int q = 0; q < D + 2; ++q) r.f[q] = (__attribute__((address_space(1))) T*)(p[q]);
  return r;
}

template <typename T>
__device__ __forceinline__ Gas<T> gas_of(const MeshDev& M) {
  Gas<T> g;
  g.gamma = (T)M.gamma;
  g.gm1 = (T)(M.gamma - 1.0);
  g.inv_gm1 = (T)M.inv_gm1;
  return g;
}

__device__ __forceinline__ int gidx(const MeshDev& M, int i, int j, int k) {
  return (k * M.n[1] + j) * M.n[0] + i;
}

#define PARAISO_WAVES_ATTR(W) __attribute__((amdgpu_waves_per_eu((W) > 0 ? (W) : 1, (W) > 0 ? (W) : 8)))

// ---------------------------------------------------------------------------
// control-block initialisation and standalone CFL reduction
// ---------------------------------------------------------------------------

// t[ring] = t0[m], steps[ring] = 0, every CFL slot and queue counter cleared.
// Reset the control ring at slot `ring`: the time from t0, or kept (keep = 1:
// the time and step count in slot `ring` stay), or zero.
static __global__ void k_ctl_init(Ctl* ctl, const double* t0, int nmeshes, int ring, unsigned int* queue,
                                  int keep) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < nmeshes) {
    Ctl& c = ctl[m];
    const double t_old = c.t[ring];
    const long long st_old = c.steps[ring];
    for (int s = 0; s < 3; ++s) {
      c.qbits[s] = 0ull;
      c.t[s] = 0.0;
      c.steps[s] = 0;
    }
    c.t[ring] = t0 ? t0[m] : (keep ? t_old : 0.0);
    c.steps[ring] = (!t0 && keep) ? st_old : 0;
    c.flags = 0;
  }
  if (m < 48 && queue) queue[m] = 0u;
}

constexpr int kChunk = 4096;  // cells per block in the standalone reductions

__device__ __forceinline__ int find_mesh_chunk(const MeshDev* ms, int nm, int chunk) {
  int lo = 0, hi = nm - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ms[mid].chunk0 <= chunk) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// CFL maximum of the current state into qbits[ring]; one block per chunk of
// kChunk cells in storage order.
template <typename T, int D>
__global__ void __launch_bounds__(256) k_cfl(Args a) {
  __shared__ double s_red[16];
  const int chunk = blockIdx.x;
  const int m = find_mesh_chunk(a.meshes, a.nmeshes, chunk);
  const MeshDev& M = a.meshes[m];
  const Fields<T, D> U = fields<T, D>(M.s[a.src]);
  const int c0 = (chunk - M.chunk0) * kChunk;
  const int c1 = min(c0 + kChunk, M.ncells);
  double qmax = 0.0;
  bool bad = false;
  for (int c = c0 + (int)threadIdx.x; c < c1; c += blockDim.x) {
    T u[D + 2];
#pragma unroll
    for (int q = 0; q < D + 2; ++q) u[q] = U.f[q][c];
    const double q = cfl_q<T, D>(u, M.inv_dx, M.gamma);
    bad |= !(q > 0.0);
    qmax = fmax(qmax, q);
  }
  cfl_commit(a, m, qmax, bad, s_red, a.ring);
}

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
        const double q = cfl_q<T, D>(out, M.inv_dx, M.gamma);
        bad |= !(q > 0.0);
        qmax = fmax(qmax, q);
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
        const double q = cfl_q<T, D>(out, M.inv_dx, M.gamma);
        bad |= !(q > 0.0);
        qmax = fmax(qmax, q);
      }
    }
    if (a.cfl && active) cfl_commit(a, t.m, qmax, bad, s_red, (a.ring + 1) % 3);
  }
}

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

template <typename T, int D, bool FIRST = false>
__device__ __forceinline__ void lds_all_axes(const LdsGeom& G, const Box& cells, const Box* faces,
                                             const Box& vbox, int off, const T* sV, T* sF,
                                             const Gas<T>& g, const T* coef, T (*acc)[D + 2]) {
  lds_fluxes<T, D, 0, FIRST>(faces[0], vbox, off, sV, G.vstride, sF, G.fstride, g);
  __syncthreads();
  lds_accumulate<T, D, 0>(cells, faces[0], sF, G.fstride, coef[0], acc);
  if constexpr (D > 1) {
    __syncthreads();
    lds_fluxes<T, D, 1, FIRST>(faces[1], vbox, off, sV, G.vstride, sF, G.fstride, g);
    __syncthreads();
    lds_accumulate<T, D, 1>(cells, faces[1], sF, G.fstride, coef[1], acc);
  }
  if constexpr (D > 2) {
    __syncthreads();
    lds_fluxes<T, D, 2, FIRST>(faces[2], vbox, off, sV, G.vstride, sF, G.fstride, g);
    __syncthreads();
    lds_accumulate<T, D, 2>(cells, faces[2], sF, G.fstride, coef[2], acc);
  }
}

// Unfused LDS stage: U_out = U0 + cdt L(U_in) on the tile.  OPT (kOpt*
// bits): analytic ghosts, first-order reconstruction; separate
// instantiations keep the plain kernel's code and registers.
template <typename T, int D, int W, int OPT = 0>
__global__ void __launch_bounds__(512) PARAISO_WAVES_ATTR(W) k_stage_lds(Args a, LdsGeom G) {
  constexpr bool AN = (OPT & kOptAnalytic) != 0;
  constexpr bool FIRST = (OPT & kOptFirstOrder) != 0;
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
      lds_all_axes<T, D, FIRST>(G, G.tile, G.fx, G.vin, G.halo, sV, sF, g, coef, acc);
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
            const double q = cfl_q<T, D>(out, M.inv_dx, M.gamma);
            bad |= !(q > 0.0);
            qmax = fmax(qmax, q);
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
template <typename T, int D, int W, int OPT = 0>
__global__ void __launch_bounds__(512) PARAISO_WAVES_ATTR(W) k_fused_lds(Args a, LdsGeom G) {
  constexpr bool FIRST = (OPT & kOptFirstOrder) != 0;
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
      lds_all_axes<T, D, FIRST>(G, G.c1, G.fx, G.vin, 2, sV, sF, g, coef1, acc);
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
      lds_all_axes<T, D, FIRST>(G, G.tile, G.fx2, G.c1, 2, sV, sF, g, coef2, acc);
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
            const double q = cfl_q<T, D>(out, M.inv_dx, M.gamma);
            bad |= !(q > 0.0);
            qmax = fmax(qmax, q);
          }
        }
      }
    }
    if (a.cfl && active) cfl_commit(a, t.m, qmax, bad, s_red, (a.ring + 1) % 3);
  }
}

// ---------------------------------------------------------------------------
// conserved totals: per-item FP64 partial sums in a fixed tree order, then a
// per-mesh fixed-order sum of the partials
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ void __launch_bounds__(256) k_totals_partial(Args a) {
  __shared__ double s_sum[kMaxFields][256];
  const int chunk = blockIdx.x;
  const int m = find_mesh_chunk(a.meshes, a.nmeshes, chunk);
  const MeshDev& M = a.meshes[m];
  const Fields<T, D> U = fields<T, D>(M.s[a.src]);
  const int c0 = (chunk - M.chunk0) * kChunk;
  const int c1 = min(c0 + kChunk, M.ncells);
  double s[D + 2];
#pragma unroll
  for (int q = 0; q < D + 2; ++q) s[q] = 0.0;
  for (int c = c0 + (int)threadIdx.x; c < c1; c += 256) {
#pragma unroll
    for (int q = 0; q < D + 2; ++q) s[q] += (double)U.f[q][c];
  }
#pragma unroll
  for (int q = 0; q < D + 2; ++q) s_sum[q][threadIdx.x] = s[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int q = 0; q < D + 2; ++q) s_sum[q][threadIdx.x] += s_sum[q][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < D + 2) a.partials[(size_t)chunk * kMaxFields + threadIdx.x] = s_sum[threadIdx.x][0];
}

// The exact conserved state of mesh m's analytic problem at time t, at every
// cell centre, into state buffer `buf` (prims and conversion in FP64).
template <typename T, int D>
__global__ void __launch_bounds__(256) k_exact_state(Args a, int m, double t, int buf) {
  const MeshDev& M = a.meshes[m];
  const Fields<T, D> U = fields<T, D>(M.s[buf]);
  const int c = blockIdx.x * 256 + (int)threadIdx.x;
  if (c >= M.ncells) return;
  const int i = c % M.n[0];
  const int j = (c / M.n[0]) % M.n[1];
  double v[D + 2];
  exact_prims<double, D>(M, (i + 0.5) * M.dx[0], D > 1 ? (j + 0.5) * M.dx[1] : 0.0, t, v);
  double ke = 0.0;
  U.f[0][c] = (T)v[0];
#pragma unroll
  for (int q = 1; q <= D; ++q) {
    U.f[q][c] = (T)(v[0] * v[q]);
    ke += v[q] * v[q];
  }
  U.f[D + 1][c] = (T)(v[D + 1] * M.inv_gm1 + 0.5 * v[0] * ke);
}

// One block per mesh: out[m*(D+2)+q] = vol * sum of the mesh's partials.
template <int D>
__global__ void __launch_bounds__(256) k_totals_final(Args a, double* out) {
  __shared__ double s_sum[kMaxFields][256];
  const int m = blockIdx.x;
  const MeshDev& M = a.meshes[m];
  double s[D + 2];
#pragma unroll
  for (int q = 0; q < D + 2; ++q) s[q] = 0.0;
  for (int it = threadIdx.x; it < M.nchunks; it += 256) {
#pragma unroll
    for (int q = 0; q < D + 2; ++q) s[q] += a.partials[(size_t)(M.chunk0 + it) * kMaxFields + q];
  }
#pragma unroll
  for (int q = 0; q < D + 2; ++q) s_sum[q][threadIdx.x] = s[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int q = 0; q < D + 2; ++q) s_sum[q][threadIdx.x] += s_sum[q][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < D + 2) out[m * (D + 2) + threadIdx.x] = s_sum[threadIdx.x][0] * M.vol;
}

}  // namespace paraiso
