// Register-march kernels for 2D meshes (gfx950, wave64): the fused step on
// periodic meshes, one stage on periodic or outflow meshes.
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

#include "euler_common.h"

namespace paraiso {

// Fused step, rows shared between the waves of a block.  The waves of a
// block are stacked along y.  Wave w computes stage 1 on its own rows only
// (input rows from 2 above to 2 below them) and its stage-2 outputs are
// shifted down by two rows: rows [y0 + 2, y1 + 2) of its range [y0, y1).
// The four stage-1 rows below its range are the first four stage-1 rows of
// wave w + 1, which that wave leaves in LDS; only the last wave of a block
// computes them itself.  So stage 1 is recomputed for four rows per block
// instead of eight per wave, at the cost of one barrier per work item; the
// last wave, which has the extra work, takes two rows fewer.  With one wave
// per block, or fewer than 6 rows per wave, every wave works as a last wave.
__host__ __device__ constexpr bool march2d_shares(int nwaves, int rows) { return nwaves > 1 && rows >= 6; }
// Rows of one work item of the fused march.
__host__ __device__ constexpr int march2d_item_rows(int nwaves, int rows) {
  return nwaves * rows - (march2d_shares(nwaves, rows) ? 2 : 0);
}

// Wave shifts by one lane.  The edge lane that has no source gets 0 from
// the DPP bound control, not from the old operand: with old ignored the
// compiler neither zeroes a destination register before each DPP move
// (one v_mov per 32-bit half, 64 per row push in FP64) nor loses the
// folding of FP32 shifts into their consumer (v_sub_f32_dpp).
// lane l receives lane l-1 (lane 0 receives 0)
__device__ __forceinline__ float lane_from_left(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x138, 0xf, 0xf, true));
}
// lane l receives lane l+1 (lane 63 receives 0)
__device__ __forceinline__ float lane_from_right(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double lane_from_left(double x) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x138, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xf, 0xf, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_from_right(double x) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x130, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xf, 0xf, true);
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

// Push V(row k) as `c` into a stage pipeline that has received N rows
// before this one (N = 4 stands for 4 or more: the steady state; N = -1
// takes the count from n at run time).  When the count is 4 or more the
// updated row k-2, base + kx dFx + ky dGy, is written to out.
template <typename T, int N>
__device__ __forceinline__ void pipe_push(RowPipe<T>& P, const T* c, const Gas<T>& g, T kx, T ky, const T* base,
                                          T* out, int n = N) {
  if (N >= 2 || (N < 0 && n >= 2)) {
    T lo_b[4], up_b[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T slope = minmod(P.b[q] - P.a[q], c[q] - P.b[q]);
      lo_b[q] = P.b[q] - T(0.5) * slope;
      up_b[q] = P.b[q] + T(0.5) * slope;
    }
    if (N >= 3 || (N < 0 && n >= 3)) {
      T G[4];
      hllc<T, 2, 1>(P.upa, lo_b, G, g);
      if (N >= 4 || (N < 0 && n >= 4)) {
        T dF[4];
        xflux_diff<T>(P.a, g, dF);
#pragma unroll
        for (int q = 0; q < 4; ++q) out[q] = fma(ky, P.g[q] - G[q], fma(kx, dF[q], base[q]));
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
}

// State of one wave marching one strip of one work item.  The y-windows
// (two stage pipelines, the base-state ring ub and the prefetched row) are
// shifted by plain assignments every push; the caller unrolls the steady
// state six-fold, so that after inlining the shifts are register renames
// and the loop carries no copies (every ring period divides six).
template <typename T, bool FUSED, bool AN = false>
struct StripMarch {
  Fields<T, 2> U0, Uin, Uout;
  Gas<T> g;
  T kx1, ky1, kx2, ky2;
  double inv_dx[2];  // held in registers: the CFL epilogue reads them every row
  double gamma;
  int nx, ny, first, bcy;
  unsigned col;
  bool base_is_input;  // the stage's base state is its input (fused step, stage 1)
  bool cfl, store_lane;  // cfl: fold the CFL quantity of every stored cell
  RowPipe<T> P1, P2;
  T ub[5][4];  // base state of rows k-4 .. k
  T nxt[4];    // input row k+1, loaded one push ahead
  double qmax;
  bool bad;
  // fused step: this wave's first four stage-1 rows for the wave above
  // (null: not needed) and the next wave's, read at the end (null: this wave
  // computes the four rows below its range itself); [row][field][lane]
  T* share_out;
  const T* share_in;
  int lane;
  // analytic boundaries (AN, one stage): the stage's input ghost cells come
  // from the ghost arrays (exact solution at the time of the stage's input)
  const __attribute__((address_space(1))) T* gsrc;  // this stage's set, field 0
  int gS;         // field stride of the ghost arrays
  int gx;         // lane's column + 2, clamped to [0, nx + 3]: its place in a ghost row
  int gxj;        // lane's ghost column 0..3 on an analytic x axis, else -1
  bool grows;     // y is analytic

  // Row offsets are wave-uniform (scalar registers) and the column a 32-bit
  // unsigned byte offset per lane, so each access is one global load or
  // store with a scalar base and no per-lane 64-bit address arithmetic.
  // (The empty asm keeps the offset from being folded into hoisted 64-bit
  // lane addresses by loop-invariant code motion.)
  __device__ __forceinline__ unsigned lane_bytes() const {
    unsigned c = col * (unsigned)sizeof(T);
    asm volatile("" : "+v"(c));
    return c;
  }
  static __device__ __forceinline__ __attribute__((address_space(1))) T* at(
      __attribute__((address_space(1))) T* row, unsigned bytes) {
    return (__attribute__((address_space(1))) T*)((__attribute__((address_space(1))) char*)row + bytes);
  }

  __device__ __forceinline__ void load_row(int k, T* u) const {
    const int ro = map_index(first + k, ny, bcy) * nx;  // in range for any row
    const unsigned c = lane_bytes();
    if constexpr (AN) {
      // One load per field from a per-lane address: the mesh row, a ghost
      // row (analytic y, a row outside the mesh) or the lane's ghost column
      // (analytic x, a lane outside the mesh).  No branch: a value merged
      // from two loads across a branch makes the wave wait at the merge for
      // the newest of them.
      const int r = first + k;
      int j = r < 0 ? r + 2 : r - ny + 2;  // ghost row 0..3 (clamped: the prefetch may run past)
      j = j < 0 ? 0 : (j > 3 ? 3 : j);
      int rr = r + 2;
      rr = rr < 0 ? 0 : (rr > ny + 3 ? ny + 3 : rr);
      const bool grow = grows && (r < 0 || r >= ny);
      const int goff = grow ? 4 * (ny + 4) + j * (nx + 4) + gx : (gxj < 0 ? 0 : gxj) * (ny + 4) + rr;
      const bool ghost = grow || gxj >= 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) u[q] = *(ghost ? gsrc + goff + q * gS : at(Uin.f[q] + ro, c));
      return;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) u[q] = *at(Uin.f[q] + ro, c);
  }

  __device__ __forceinline__ void emit(int y, const T* u) {
    // the fused step's outputs are shifted by two rows and wrap (periodic)
    const int ro = (FUSED ? map_index(y, ny, kPeriodic) : y) * nx;
    if (store_lane) {
      const unsigned c = lane_bytes();
#pragma unroll
      for (int q = 0; q < 4; ++q) *at(Uout.f[q] + ro, c) = u[q];
      if (cfl) {
        cfl_fold(cfl_q<T, 2>(u, inv_dx, gamma), qmax, bad);
      }
    }
  }

  // Row k enters stage 1, which has received S1 rows before it (4: four or
  // more); in the fused step a completed stage-1 row enters stage 2, which
  // has received S2 rows before it.
  template <int S1, int S2>
  __device__ __forceinline__ void push(int k, int n2 = S2, T* v1_out = nullptr) {
    T u[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) u[q] = nxt[q];
    load_row(k + 1, nxt);  // in range for any k (wrapped or clamped); unused after the last row
    T base[4];
    if (base_is_input) {
#pragma unroll
      for (int q = 0; q < 4; ++q) base[q] = u[q];
    } else {
      const int ro = map_index(first + k, ny, bcy) * nx;
      const unsigned c = lane_bytes();
#pragma unroll
      for (int q = 0; q < 4; ++q) base[q] = *at(U0.f[q] + ro, c);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int q = 0; q < 4; ++q) ub[s][q] = ub[s + 1][q];
#pragma unroll
    for (int q = 0; q < 4; ++q) ub[4][q] = base[q];
    T v[4];
    prim_of_cons<T, 2>(u, v, g);
    // stage-1 output: row first + k - 2, base ub[2]
    T u1[4];
    pipe_push<T, S1>(P1, v, g, kx1, ky1, ub[2], u1);
    if constexpr (S1 >= 4) {
      if constexpr (!FUSED) {
        emit(first + k - 2, u1);
      } else {
        T v1[4];
        prim_of_cons<T, 2>(u1, v1, g);
        if (v1_out) {
#pragma unroll
          for (int q = 0; q < 4; ++q) v1_out[q * 64 + lane] = v1[q];
        }
        // stage-2 output: row first + k - 4, base ub[0]
        T u2[4];
        pipe_push<T, S2>(P2, v1, g, kx2, ky2, ub[0], u2, n2);
        if constexpr (S2 >= 4) emit(first + k - 4, u2);
      }
    }
  }

  // Stage 2 only: push a stage-1 row of the next wave (from LDS).
  __device__ __forceinline__ void push_shared(int k, const T* row) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int q = 0; q < 4; ++q) ub[s][q] = ub[s + 1][q];
    T v1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v1[q] = row[q * 64 + lane];
    T u2[4];
    pipe_push<T, 4>(P2, v1, g, kx2, ky2, ub[0], u2);
    emit(first + k - 4, u2);
  }

  // All rows of the strip: npush stage-1 pushes (output rows + 4, + 4 more
  // for a fused-step wave that computes the rows below its range itself).
  // `barrier`: the block shares rows; every wave of the block, active or
  // not, passes one barrier per work item.
  __device__ __forceinline__ void run(int npush, bool barrier) {
    load_row(0, nxt);
    int k = 0;
    // stage-1 warm-up (cheap pushes, straight-line code)
    push<0, 0>(k++);
    push<1, 0>(k++);
    push<2, 0>(k++);
    push<3, 0>(k++);
    if constexpr (FUSED) {
      // stage-2 warm-up as a loop: as straight-line code the compiler
      // overlaps these four pushes and needs ~50 more VGPRs.  Their stage-1
      // rows are this wave's first four.
#pragma clang loop unroll(disable)
      for (int n2 = 0; n2 < 4; ++n2) push<4, -1>(k++, n2, share_out ? share_out + n2 * 256 : nullptr);
      if (barrier) __syncthreads();
    }
    // steady state, unrolled six-fold
    for (; k + 6 <= npush; k += 6) {
      push<4, 4>(k);
      push<4, 4>(k + 1);
      push<4, 4>(k + 2);
      push<4, 4>(k + 3);
      push<4, 4>(k + 4);
      push<4, 4>(k + 5);
    }
    for (; k < npush; ++k) push<4, 4>(k);
    if constexpr (FUSED) {
      if (share_in) {
#pragma clang loop unroll(disable)
        for (int j = 0; j < 4; ++j) push_shared(k++, share_in + j * 256);
      }
    }
  }
};

// Fused step (FUSED, periodic meshes) or one stage (!FUSED, periodic or
// outflow: the stage's ghost cells are clamped loads of its input; with AN
// also analytic, ghost cells from the ghost arrays k_analytic_ghosts fills).
// Block = threads/64 waves stacked along y, `rows` rows each: the block
// tile is (64 - 2H) columns by march2d_item_rows(waves, rows) rows (the
// last wave of a sharing block takes rows - 2).
template <typename T, int W, bool FUSED, bool AN = false>
__global__ void __launch_bounds__(256) PARAISO_WAVES_ATTR(W) k_march2d(Args a, LdsGeom G) {
  static_assert(!(AN && FUSED), "analytic boundaries: one stage per launch");
  constexpr int H = FUSED ? 4 : 2;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double s_red[16];
  __shared__ int s_item;
  const int lane = threadIdx.x & 63;
  // wave-uniform, so the row loop is scalar control flow
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nwaves = blockDim.x >> 6;
  const int rows = G.rows;
  const bool share = FUSED && march2d_shares(nwaves, rows);
  const int item_rows = FUSED ? march2d_item_rows(nwaves, rows) : rows * nwaves;
  T* const lds_rows = reinterpret_cast<T*>(smem);  // [wave][4 rows][4 fields][64 lanes]
  ItemLoop it{0, 1};
  for (int item; (item = next_item(a, it, &s_item, FUSED ? 0 : a.stage - 1)) >= 0;) {
    item = __builtin_amdgcn_readfirstlane(item);  // the same for the whole block
    const Tile t = tile_of(a, item);
    const MeshDev& M = a.meshes[t.m];
    bool active;
    const double dt = step_dt(a, t.m, active);
    const bool last_stage = FUSED || a.stage == 2;
    if (last_stage && t.first && threadIdx.x == 0) step_bookkeeping(a, t.m, dt, active);
    const int nx = M.n[0], ny = M.n[1];
    const int x0 = t.org[0];
    const int yb1 = min(t.org[1] + item_rows, ny);  // end of the block's rows
    const int y0 = t.org[1] + wave * rows;
    const int y1 = min(y0 + rows, yb1);
    const bool last_wave = y1 >= yb1;
    const int col = map_index(x0 - H + lane, nx, FUSED ? kPeriodic : M.bc[0]);
    const bool store_lane = lane >= H && lane < 64 - H && (x0 - H + lane) < nx;
    const Fields<T, 2> U0 = fields<T, 2>(M.s[a.src]);
    double qmax = 0.0;
    bool bad = false;
    const Fields<T, 2> Uout =
        (FUSED || a.stage == 2) ? fields<T, 2>(M.s[1 - a.src]) : fields<T, 2>(M.w);
    if (!active) {
      if (last_stage) {
        for (int y = y0; y < y1; ++y) {
          const int gi = y * nx + col;
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (store_lane) Uout.f[q][gi] = U0.f[q][gi];
        }
      }
    } else if (y0 < y1) {
      StripMarch<T, FUSED, AN> S;
      S.U0 = uniform(U0);
      S.Uin = uniform((FUSED || a.stage == 1) ? U0 : fields<T, 2>(M.w));
      S.Uout = uniform(Uout);
      S.g = gas_of<T>(M);
      const double c1 = FUSED ? 0.5 * dt : (a.stage == 1 ? 0.5 * dt : dt);
      S.kx1 = (T)(c1 * M.inv_dx[0]);
      S.ky1 = (T)(c1 * M.inv_dx[1]);
      S.kx2 = (T)(dt * M.inv_dx[0]);
      S.ky2 = (T)(dt * M.inv_dx[1]);
      S.inv_dx[0] = M.inv_dx[0];
      S.inv_dx[1] = M.inv_dx[1];
      S.gamma = M.gamma;
      S.nx = nx;
      S.ny = ny;
      S.col = (unsigned)col;
      S.first = y0 - 2;
      S.bcy = FUSED ? kPeriodic : M.bc[1];
      S.base_is_input = FUSED || a.stage == 1;
      S.cfl = a.cfl != 0 && last_stage;
      S.store_lane = store_lane;
      S.qmax = 0.0;
      S.bad = false;
      S.lane = lane;
      if constexpr (AN) {
        S.gS = ghost_stride(nx, ny);
        S.gsrc = (const __attribute__((address_space(1))) T*)(reinterpret_cast<const T*>(M.ghost) +
                                                              (a.stage == 2 ? 4 * S.gS : 0));
        const int xc = x0 - H + lane;
        int gj = xc < 0 ? xc + 2 : xc - nx + 2;
        gj = gj < 0 ? 0 : (gj > 3 ? 3 : gj);
        S.gxj = (M.bc[0] == kAnalytic && (xc < 0 || xc >= nx)) ? gj : -1;
        S.gx = xc + 2 < 0 ? 0 : (xc + 2 > nx + 3 ? nx + 3 : xc + 2);
        S.grows = M.bc[1] == kAnalytic;
      }
      // fused: a wave that is not the block's last reads the next wave's
      // first four stage-1 rows; every wave but the first leaves its own
      S.share_out = (share && wave > 0) ? lds_rows + wave * 1024 : nullptr;
      S.share_in = (share && !last_wave) ? lds_rows + (wave + 1) * 1024 : nullptr;
      const int npush = (y1 - y0) + (FUSED ? (S.share_in ? 4 : 8) : 4);
      S.run(npush, share);
      qmax = S.qmax;
      bad = S.bad;
    } else if (share) {
      __syncthreads();  // an idle wave passes the block's one barrier too
    }
    if (a.cfl && active && last_stage) cfl_commit(a, t.m, qmax, bad, s_red, (a.ring + 1) % 3);
  }
}

}  // namespace paraiso
