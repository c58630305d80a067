// Shared parts of the Euler-step kernels (gfx950, wave64): mesh table,
// control rings, work items, the CFL and totals reductions.
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
// their bits).  A 3-slot ring of non-physical flags follows the same rule:
// the CFL epilogue flags slot (n+1)%3, and a step whose slot n%3 is flagged
// does not advance (the offending state, its time and its step count stay).
// No grid barrier is needed.
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
  void* ghost;             // 2D analytic meshes: the exact solution on the ghost cells of both
                           // stages, [stage][field][ghost cell] (see ghost_stride), in the workspace
};

// Ghost cells of a 2D mesh kept for the register march: the 2 columns on
// each side for every row from -2 to ny+1 (4 (ny+4) cells), then the 2 rows
// on each side for every column from -2 to nx+1 (4 (nx+4) cells).
__host__ __device__ constexpr int ghost_stride(int nx, int ny) { return 4 * (ny + 4) + 4 * (nx + 4); }

// The CFL maximum of a ring slot lives in kQSub sub-slots: block b folds its
// maximum into sub-slot b mod kQSub (for 8, the XCD the block runs on), so
// the one atomic per block of a launch spreads over kQSub addresses instead
// of queueing on one when the blocks end together; readers take the largest
// sub-slot (bit patterns of non-negative doubles order as unsigned integers).
constexpr int kQSub = 8;

struct Ctl {
  double t[3];
  unsigned long long qbits[3][kQSub];
  long long steps[3];
  int flags[3];  // per ring slot: bit 0 set when the state of that slot is non-physical or non-finite
  int pad_;
};

__host__ __device__ inline unsigned long long qbits_max(const Ctl& c, int slot) {
  unsigned long long b = c.qbits[slot][0];
  for (int k = 1; k < kQSub; ++k) b = c.qbits[slot][k] > b ? c.qbits[slot][k] : b;
  return b;
}

__host__ __device__ inline void qbits_clear(Ctl& c, int slot) {
  for (int k = 0; k < kQSub; ++k) c.qbits[slot][k] = 0ull;
}

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

// dt of mesh m for this step; `active` false once t >= t_end, the step
// budget is spent or the input state was found non-physical (the step then
// copies U0 to the output, and time and step count stay).  The flag is read
// from this step's ring slot, which no block of this launch writes, so every
// block of a launch takes the same decision.
__device__ __forceinline__ double step_dt(const Args& a, int m, bool& active) {
  if (a.dt) {
    active = true;
    return a.dt[m];
  }
  const Ctl& c = a.ctl[m];
  const double t = c.t[a.ring];
  const long long st = c.steps[a.ring];
  active = (t < a.prm->t_end) && (st < a.prm->max_steps) && c.flags[a.ring] == 0;
  if (!active) return 0.0;
  double dt = a.prm->cfl / __longlong_as_double((long long)qbits_max(c, a.ring));
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
  if (!a.dt) qbits_clear(c, nn);
  // an inactive step copies its input, so its output keeps the input's flag;
  // an active step's CFL epilogue sets slot nx itself (cleared a step ago)
  if (!active) c.flags[nx] = c.flags[a.ring];
  c.flags[nn] = 0;
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
  if (bad) atomicOr(&a.ctl[m].flags[slot], 1);
  if (threadIdx.x == 0 && v > 0.0)
    atomicMax(&a.ctl[m].qbits[slot][blockIdx.x % kQSub], (unsigned long long)__double_as_longlong(v));
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
      qbits_clear(c, s);
      c.t[s] = 0.0;
      c.steps[s] = 0;
      c.flags[s] = 0;
    }
    c.t[ring] = t0 ? t0[m] : (keep ? t_old : 0.0);
    c.steps[ring] = (!t0 && keep) ? st_old : 0;
  }
  if (m < 48 && queue) queue[m] = 0u;
}

// Start of paraiso_advance for up to kInlineMeshes meshes, with the
// parameter block and the start times passed by value (no host-to-device
// copy): writes the parameter block, then resets each mesh's control ring at
// slot `ring` as k_ctl_init does with a time array.
constexpr int kInlineMeshes = 16;
struct InlineTimes {
  double t[kInlineMeshes];
};
static __global__ void k_advance_init(Ctl* ctl, Params* prm, Params p, InlineTimes t0, int nmeshes, int ring,
                                      unsigned int* queue) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m == 0) *prm = p;
  if (m < nmeshes) {
    Ctl& c = ctl[m];
    for (int s = 0; s < 3; ++s) {
      qbits_clear(c, s);
      c.t[s] = 0.0;
      c.steps[s] = 0;
      c.flags[s] = 0;
    }
    c.t[ring] = t0.t[m];
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

// CFL maximum of the current state into the sub-slots of qbits[ring]; one block of 256
// threads per chunk of kChunk cells in storage order.  A full chunk is read
// with 16-byte loads (4 FP32 or 2 FP64 cells per load and field), all of a
// thread's loads issued before its arithmetic; a mesh's last, partial chunk
// (or a field array whose chunk start is not 16-byte aligned) cell by cell.
template <typename T, int D>
__global__ void __launch_bounds__(256) k_cfl(Args a) {
  __shared__ double s_red[16];
  constexpr int V = 16 / (int)sizeof(T);        // cells per 16-byte load
  constexpr int kIter = kChunk / (256 * V);     // loads per field and thread
  static_assert(kChunk % (256 * V) == 0, "a chunk is a whole number of vector rounds");
  const int chunk = blockIdx.x;
  const int m = find_mesh_chunk(a.meshes, a.nmeshes, chunk);
  const MeshDev& M = a.meshes[m];
  const Fields<T, D> U = fields<T, D>(M.s[a.src]);
  const int c0 = (chunk - M.chunk0) * kChunk;
  const int n = min(kChunk, M.ncells - c0);  // cells of this chunk (c0 + kChunk may pass 2^31 - 1)
  double qmax = 0.0;
  bool bad = false;
  bool aligned = true;
#pragma unroll
  for (int q = 0; q < D + 2; ++q) aligned &= ((unsigned long long)(U.f[q] + c0) & 15ull) == 0;
  if (n == kChunk && aligned) {
    using Vec = __attribute__((ext_vector_type(16 / sizeof(T)))) T;
    Vec w[kIter][D + 2];
#pragma unroll
    for (int it = 0; it < kIter; ++it)
#pragma unroll
      for (int q = 0; q < D + 2; ++q)
        w[it][q] = *reinterpret_cast<const __attribute__((address_space(1))) Vec*>(
            U.f[q] + c0 + (it * 256 + (int)threadIdx.x) * V);
#pragma unroll
    for (int it = 0; it < kIter; ++it)
#pragma unroll
      for (int j = 0; j < V; ++j) {
        T u[D + 2];
#pragma unroll
        for (int q = 0; q < D + 2; ++q) u[q] = w[it][q][j];
        cfl_fold(cfl_q<T, D>(u, M.inv_dx, M.gamma), qmax, bad);
      }
  } else {
    // four cells per thread in flight: the loads of the next iterations are
    // issued before this one's arithmetic
#pragma unroll 4
    for (int i = (int)threadIdx.x; i < n; i += blockDim.x) {
      T u[D + 2];
#pragma unroll
      for (int q = 0; q < D + 2; ++q) u[q] = U.f[q][c0 + i];
      cfl_fold(cfl_q<T, D>(u, M.inv_dx, M.gamma), qmax, bad);
    }
  }
  cfl_commit(a, m, qmax, bad, s_red, a.ring);
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
  const int n = min(kChunk, M.ncells - c0);  // cells of this chunk (c0 + kChunk may pass 2^31 - 1)
  double s[D + 2];
#pragma unroll
  for (int q = 0; q < D + 2; ++q) s[q] = 0.0;
  for (int i = (int)threadIdx.x; i < n; i += 256) {
#pragma unroll
    for (int q = 0; q < D + 2; ++q) s[q] += (double)U.f[q][c0 + i];
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

