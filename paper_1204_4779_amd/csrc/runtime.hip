// Host runtime and C ABI of the Euler-step library (see include/paraiso.h).
//
// The runtime validates descriptors, lays out the caller's workspace, picks
// and launches kernels for the selected variant, keeps the time-stepping
// state on the device, and replays captured HIP graphs of six steps (the
// period of the buffer ping-pong times the 3-slot control ring).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "euler_kernels.h"
#include "euler_march2d.h"
#include "euler_resident1d.h"
#include "kernel_table.h"
#include "paraiso.h"

using namespace paraiso;

namespace {
// message of the last failure on this thread, in a fixed buffer so that
// setting it never allocates (the no-allocation entry point reports through it)
thread_local char g_err[512];
}

void paraiso_set_error_text(const char* msg) { std::snprintf(g_err, sizeof(g_err), "%s", msg); }
void paraiso_set_error(const std::string& msg) { paraiso_set_error_text(msg.c_str()); }

namespace {

int fail(int code, const std::string& msg) {
  paraiso_set_error(msg);
  return code;
}

// A HIP call of the library failed: report it, and take the error off HIP's
// per-thread record so that the caller's next HIP call does not see it again.
int hip_fail(const std::string& what, hipError_t e) {
  (void)hipGetLastError();
  return fail(PARAISO_ERR_HIP, what + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call)                                \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return hip_fail(#call, e_); \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

const KernelTable* table_for(int dtype, int ndim) {
  if (dtype == PARAISO_F32) {
    if (ndim == 1) return table_f32_1();
    if (ndim == 2) return table_f32_2();
    return table_f32_3();
  }
  if (ndim == 1) return table_f64_1();
  if (ndim == 2) return table_f64_2();
  return table_f64_3();
}

int64_t cells_of(const paraiso_mesh& m) { return m.n[0] * m.n[1] * m.n[2]; }

bool has_analytic(const paraiso_mesh& m) {
  for (int a = 0; a < m.ndim; ++a)
    if (m.bc[a] == PARAISO_ANALYTIC) return true;
  return false;
}

bool first_order(const paraiso_mesh& m) { return m.order == 1; }

bool any_analytic(const paraiso_mesh* ms, int count) {
  for (int i = 0; i < count; ++i)
    if (has_analytic(ms[i])) return true;
  return false;
}

// Star state of the ideal-gas Riemann problem (rho, u, p)_L | (rho, u, p)_R
// (Toro, Riemann Solvers and Numerical Methods for Fluid Dynamics, ch. 4):
// p* is the root of phi(p) = g_L(p) + g_R(p) + u_R - u_L, where g_K is the
// velocity jump across the K wave (shock above p_K, rarefaction below);
// Newton's method from the acoustic (linearised) estimate.  u* follows from
// either side.  Returns false if the data generate a vacuum.
bool riemann_star_state(double gamma, const double L[3], const double R[3], double* ps, double* us) {
  const double gp = gamma + 1.0, gm = gamma - 1.0;
  auto jump = [&](const double K[3], double p, double& slope) {
    const double c = std::sqrt(gamma * K[2] / K[0]);
    if (p <= K[2]) {
      const double r = std::pow(p / K[2], gm / (2.0 * gamma));
      slope = r / (K[0] * c * (p / K[2]));
      return 2.0 * c / gm * (r - 1.0);
    }
    const double A = 2.0 / (gp * K[0]), B = gm / gp * K[2];
    const double root = std::sqrt(A / (B + p));
    slope = root * (1.0 - 0.5 * (p - K[2]) / (B + p));
    return root * (p - K[2]);
  };
  const double cL = std::sqrt(gamma * L[2] / L[0]), cR = std::sqrt(gamma * R[2] / R[0]);
  const double du = R[1] - L[1];
  if (2.0 * (cL + cR) / gm <= du) return false;
  double p = 0.5 * (L[2] + R[2]) - 0.125 * du * (L[0] + R[0]) * (cL + cR);
  p = std::max(p, 1e-8 * std::min(L[2], R[2]));
  for (int it = 0; it < 200; ++it) {
    double sL, sR;
    const double phi = jump(L, p, sL) + jump(R, p, sR) + du;
    double next = p - phi / (sL + sR);
    if (!(next > 0.0)) next = 0.5 * p;
    const bool done = std::fabs(next - p) <= 1e-15 * 0.5 * (next + p);
    p = next;
    if (done) break;
  }
  double sL, sR;
  const double gL = jump(L, p, sL), gR = jump(R, p, sR);
  *ps = p;
  *us = 0.5 * (L[1] + R[1] + gR - gL);
  return true;
}

int validate_mesh(const paraiso_mesh& m, int idx) {
  const std::string w = "mesh " + std::to_string(idx) + ": ";
  if (m.ndim < 1 || m.ndim > 3) return fail(PARAISO_ERR_INVALID_ARG, w + "ndim must be 1, 2 or 3");
  if (m.dtype != PARAISO_F32 && m.dtype != PARAISO_F64)
    return fail(PARAISO_ERR_INVALID_ARG, w + "dtype must be PARAISO_F32 or PARAISO_F64");
  if (!(m.gamma > 1.0) || !std::isfinite(m.gamma))
    return fail(PARAISO_ERR_INVALID_ARG, w + "gamma must be finite and > 1");
  if (m.order != 0 && m.order != 1 && m.order != 2)
    return fail(PARAISO_ERR_INVALID_ARG, w + "order must be 0 (= 2), 1 or 2");
  for (int a = 0; a < 3; ++a) {
    if (m.n[a] < 1) return fail(PARAISO_ERR_INVALID_ARG, w + "n[a] must be >= 1");
    if (a >= m.ndim) {
      if (m.n[a] != 1) return fail(PARAISO_ERR_INVALID_ARG, w + "n[a] must be 1 for a >= ndim");
      continue;
    }
    if (!(m.dx[a] > 0.0) || !std::isfinite(m.dx[a]))
      return fail(PARAISO_ERR_INVALID_ARG, w + "dx[a] must be finite and > 0");
    if (m.bc[a] != PARAISO_PERIODIC && m.bc[a] != PARAISO_OUTFLOW && m.bc[a] != PARAISO_ANALYTIC)
      return fail(PARAISO_ERR_INVALID_ARG, w + "bc[a] must be PARAISO_PERIODIC, PARAISO_OUTFLOW or PARAISO_ANALYTIC");
  }
  if (m.n[0] > (1 << 30) || m.n[1] > (1 << 30) || m.n[2] > (1 << 30) || cells_of(m) >= (int64_t(1) << 31))
    return fail(PARAISO_ERR_UNSUPPORTED, w + "more than 2^31 - 1 cells");
  const size_t esz = m.dtype == PARAISO_F32 ? 4 : 8;
  const size_t bytes = (size_t)cells_of(m) * esz;
  const int nf = m.ndim + 2;
  std::vector<std::pair<uintptr_t, uintptr_t>> ranges;
  for (int b = 0; b < 2; ++b)
    for (int q = 0; q < nf; ++q) {
      const uintptr_t p = (uintptr_t)m.state[b][q];
      if (!p) return fail(PARAISO_ERR_INVALID_ARG, w + "null state pointer");
      if (p % 16) return fail(PARAISO_ERR_INVALID_ARG, w + "state arrays must be 16-byte aligned");
      ranges.push_back({p, p + bytes});
    }
  std::sort(ranges.begin(), ranges.end());
  for (size_t k = 1; k < ranges.size(); ++k)
    if (ranges[k].first < ranges[k - 1].second)
      return fail(PARAISO_ERR_INVALID_ARG, w + "state arrays overlap");
  return PARAISO_OK;
}

int validate_meshes(const paraiso_mesh* ms, int count) {
  if (!ms) return fail(PARAISO_ERR_INVALID_ARG, "null mesh array");
  if (count < 1) return fail(PARAISO_ERR_INVALID_ARG, "count must be >= 1");
  for (int i = 0; i < count; ++i) {
    int rc = validate_mesh(ms[i], i);
    if (rc) return rc;
    if (ms[i].ndim != ms[0].ndim || ms[i].dtype != ms[0].dtype)
      return fail(PARAISO_ERR_INVALID_ARG, "all meshes of a batch must share ndim and dtype");
    if (first_order(ms[i]) != first_order(ms[0]))
      return fail(PARAISO_ERR_INVALID_ARG, "all meshes of a batch must share the reconstruction order");
  }
  return PARAISO_OK;
}

// The analytic 2D register march addresses its ghost arrays (both stages,
// 4 fields, ghost_stride cells each) with 32-bit offsets: meshes whose
// arrays pass that (n[0] + n[1] near 2^26 or more) take the LDS tiles, which
// evaluate the exact solution in place and keep no ghost arrays.
bool ghosts_fit(const paraiso_mesh& m) {
  const int64_t stride = 4 * ((int64_t)m.n[1] + 4) + 4 * ((int64_t)m.n[0] + 4);
  return 8 * stride < (int64_t(1) << 31);
}

bool all_ghosts_fit(const paraiso_mesh* ms, int count) {
  for (int i = 0; i < count; ++i)
    if (ms[i].ndim == 2 && has_analytic(ms[i]) && !ghosts_fit(ms[i])) return false;
  return true;
}

// Ghost arrays of a 2D mesh with an analytic axis (both stages, d+2 fields),
// for the register march; none where that march cannot run.
size_t ghost_bytes(const paraiso_mesh& m) {
  if (m.ndim != 2 || !has_analytic(m) || !ghosts_fit(m)) return 0;
  const size_t esize = m.dtype == PARAISO_F32 ? 4 : 8;
  return align256(2 * 4 * (size_t)ghost_stride((int)m.n[0], (int)m.n[1]) * esize);
}

struct Layout {
  size_t meshes = 0, ctl = 0, params = 0, dt = 0, queue = 0, out = 0, partials = 0, u1 = 0, ghost = 0, total = 0;
  int total_chunks = 0;
};

Layout layout_of(const paraiso_mesh* ms, int count) {
  Layout L;
  size_t off = 0;
  L.meshes = off;
  off += align256(sizeof(MeshDev) * count);
  L.ctl = off;
  off += align256(sizeof(Ctl) * count);
  L.params = off;
  off += align256(sizeof(Params));
  L.dt = off;
  off += align256(sizeof(double) * count);
  L.queue = off;
  off += align256(sizeof(unsigned) * 48);
  L.out = off;
  off += align256(sizeof(double) * kMaxFields * count);
  int chunks = 0;
  for (int m = 0; m < count; ++m) chunks += (int)((cells_of(ms[m]) + kChunk - 1) / kChunk);
  L.total_chunks = chunks;
  L.partials = off;
  off += align256(sizeof(double) * kMaxFields * (size_t)chunks);
  L.u1 = off;
  const size_t esz = ms[0].dtype == PARAISO_F32 ? 4 : 8;
  for (int m = 0; m < count; ++m) off += (size_t)(ms[m].ndim + 2) * align256((size_t)cells_of(ms[m]) * esz);
  L.ghost = off;
  for (int m = 0; m < count; ++m) off += ghost_bytes(ms[m]);
  L.total = off;
  return L;
}

struct Launch {
  const void* fn = nullptr;
  dim3 grid, block;
  size_t shmem = 0;
  bool with_geom = false;
};

}  // namespace

struct paraiso_ctx {
  int count = 0, ndim = 0, dtype = 0, esize = 4;
  std::vector<paraiso_mesh> meshes;
  std::vector<MeshDev> hm;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  Layout L;
  MeshDev* d_meshes = nullptr;
  Ctl* d_ctl = nullptr;
  Params* d_params = nullptr;
  double* d_dt = nullptr;
  unsigned* d_queue = nullptr;
  double* d_out = nullptr;
  double* d_partials = nullptr;
  const KernelTable* tab = nullptr;
  paraiso_variant var{};
  bool fused = false, lds = false, persistent = false, resident = false;
  bool ghosts = false;  // the variant reads the ghost arrays: fill them before every step
  int ghost_blocks = 1;  // blocks per mesh of the ghost fill (one ghost cell per thread)
  int nitems = 0;
  int xcd_begin[9] = {};
  LdsGeom geom{};
  Launch step;  // fused kernel, or the stage kernel launched twice
  int eff_tile[3] = {1, 1, 1};  // tile of one work item for the kernels
  int cur = 0, ring = 0;
  hipGraphExec_t graph[6] = {};
  int device = 0, num_cus = 0, max_lds = 0;
  bool ctl_ready = false;          // the control ring holds a time to keep
  std::vector<char> analytic_set;  // per mesh: problem given by paraiso_set_analytic
  // pinned host staging for the synchronous calls' small copies (the
  // parameter block and start times of an advance, the control blocks read
  // back): page-locked, so each copy is one DMA instead of a staged one
  char* h_pin = nullptr;
  size_t pin_ctl = 0;  // offset of the control-block area
};

namespace {

Box make_box(int e0, int e1, int e2) {
  Box b;
  b.e[0] = e0;
  b.e[1] = e1;
  b.e[2] = e2;
  b.count = e0 * e1 * e2;
  b.d0 = FastDiv::make((uint32_t)e0);
  b.d01 = FastDiv::make((uint32_t)(e0 * e1));
  return b;
}

void drop_graphs(paraiso_ctx* c) {
  for (auto& g : c->graph) {
    if (g) hipGraphExecDestroy(g);
    g = nullptr;
  }
}

Args base_args(const paraiso_ctx* c) {
  Args a{};
  a.meshes = c->d_meshes;
  a.ctl = c->d_ctl;
  a.prm = c->d_params;
  a.dt = nullptr;
  a.queue = c->d_queue;
  a.partials = c->d_partials;
  a.nmeshes = c->count;
  a.nitems = c->nitems;
  for (int k = 0; k < 3; ++k) a.tile[k] = c->eff_tile[k];
  a.persistent = c->persistent ? 1 : 0;
  for (int k = 0; k < 9; ++k) a.xcd_begin[k] = c->xcd_begin[k];
  return a;
}

int launch(const Launch& l, Args a, const LdsGeom& g, hipStream_t s) {
  void* args2[] = {(void*)&a, (void*)&g};
  HIP_TRY(hipLaunchKernel(l.fn, l.grid, l.block, args2, l.shmem, s));
  return PARAISO_OK;
}

// Enqueue one step in phase (cur, ring); explicit: dt from d_dt.
int enqueue_step(const paraiso_ctx* c, int cur, int ring, bool explicit_dt, hipStream_t s) {
  Args a = base_args(c);
  a.dt = explicit_dt ? c->d_dt : nullptr;
  a.src = cur;
  a.ring = ring;
  if (c->fused || c->resident) {
    a.stage = 0;
    a.cfl = explicit_dt ? 0 : 1;
    return launch(c->step, a, c->geom, s);
  }
  if (c->ghosts) {
    // exact ghost cells of both stages of this step, from the device-held t and dt
    void* args[] = {(void*)&a};
    HIP_TRY(hipLaunchKernel(c->tab->analytic_ghosts, dim3(c->count, c->ghost_blocks), dim3(256), args, 0, s));
  }
  a.stage = 1;
  a.cfl = 0;
  int rc = launch(c->step, a, c->geom, s);
  if (rc) return rc;
  a.stage = 2;
  a.cfl = explicit_dt ? 0 : 1;
  return launch(c->step, a, c->geom, s);
}

int capture_graph(paraiso_ctx* c, int phase) {
  const int cur0 = phase / 3, ring0 = phase % 3;
  HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed));
  int rc = PARAISO_OK;
  for (int s = 0; s < 6 && !rc; ++s) rc = enqueue_step(c, (cur0 + s) & 1, (ring0 + s) % 3, false, c->cap);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->cap, &g);
  if (rc) {
    if (g) hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail("hipStreamEndCapture", e);
  e = hipGraphInstantiate(&c->graph[phase], g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) {
    c->graph[phase] = nullptr;
    return hip_fail("hipGraphInstantiate", e);
  }
  return PARAISO_OK;
}

// Device-dt steps: whole six-step periods from the graphs (captured when the
// variant is applied; again here only if that capture was dropped), the rest
// eagerly.
int run_steps(paraiso_ctx* c, int64_t n) {
  while (n >= 6) {
    const int phase = c->cur * 3 + c->ring;
    if (!c->graph[phase]) {
      int rc = capture_graph(c, phase);
      if (rc) return rc;
    }
    HIP_TRY(hipGraphLaunch(c->graph[phase], c->stream));
    n -= 6;
  }
  while (n > 0) {
    int rc = enqueue_step(c, c->cur, c->ring, false, c->stream);
    if (rc) return rc;
    c->cur ^= 1;
    c->ring = (c->ring + 1) % 3;
    --n;
  }
  return PARAISO_OK;
}

// Reset the control ring: time from d_t0 (device), else the time held so far.
int ctl_init(paraiso_ctx* c, const double* d_t0) {
  const int blocks = (std::max(c->count, 48) + 255) / 256;
  hipLaunchKernelGGL(k_ctl_init, dim3(blocks), dim3(256), 0, c->stream, c->d_ctl, d_t0, c->count, c->ring,
                     c->d_queue, c->ctl_ready ? 1 : 0);
  HIP_TRY(hipGetLastError());
  return PARAISO_OK;
}

int launch_cfl(paraiso_ctx* c) {
  Args a = base_args(c);
  a.src = c->cur;
  a.ring = c->ring;
  void* args[] = {(void*)&a};
  HIP_TRY(hipLaunchKernel(c->tab->cfl, dim3(c->L.total_chunks), dim3(256), args, 0, c->stream));
  return PARAISO_OK;
}

// The march kernels address a lane's cell with a 32-bit byte offset from a
// scalar base: within a row in 2D, within a plane in 3D.
bool march_offsets_fit(const paraiso_mesh* meshes, int count) {
  for (int m = 0; m < count; ++m) {
    const paraiso_mesh& p = meshes[m];
    const int64_t span = p.ndim == 2 ? p.n[0] : p.n[0] * p.n[1];
    const int64_t esize = p.dtype == PARAISO_F64 ? 8 : 4;
    if (span * esize >= (int64_t(1) << 32)) return false;
  }
  return true;
}

// Dynamic LDS of the fused 3D march with nw waves: V0 and V1 planes
// (double-buffered, nw + 4 and nw rows), stage-1 and stage-2 y-flux rings
// (3 slots, nw + 1 and nw - 3 faces), 5 fields of 64 lanes each.
size_t march3d_fused_lds(int nw, int esize) {
  return (size_t)esize * 5 * 64 * (2 * (size_t)(nw + 4) + 2 * (size_t)nw + 3 * (size_t)(nw + 1) + 3 * (size_t)(nw - 3));
}

int64_t max_cells(const paraiso_mesh* meshes, int count) {
  int64_t n = 1;
  for (int m = 0; m < count; ++m) n = std::max<int64_t>(n, cells_of(meshes[m]));
  return n;
}

int validate_variant(const paraiso_ctx* c, const paraiso_variant& v, std::string& why) {
  const int d = c->ndim;
  for (int a = 0; a < 3; ++a) {
    if (a < d && (v.tile[a] < 1 || v.tile[a] > 4096)) {
      why = "tile[a] must be in [1, 4096] on active axes";
      return PARAISO_ERR_UNSUPPORTED;
    }
    if (a >= d && v.tile[a] != 1) {
      why = "tile[a] must be 1 on unused axes";
      return PARAISO_ERR_UNSUPPORTED;
    }
  }
  if (v.lds < 0 || v.lds > 3) return why = "lds must be 0, 1, 2 or 3", PARAISO_ERR_UNSUPPORTED;
  if (v.lds == 3) {
    if (d != 1) return why = "resident kernel (lds = 3) exists for 1D meshes only", PARAISO_ERR_UNSUPPORTED;
    if (v.threads != 0 && v.threads != 512 && v.threads != 1024)
      return why = "resident kernel: threads must be 0 (chosen from the largest mesh), 512 or 1024",
             PARAISO_ERR_UNSUPPORTED;
    const int cap = v.threads ? kResidentPerThread * v.threads : kResidentCells;
    for (const auto& m : c->meshes) {
      if (m.n[0] > cap)
        return why = "resident kernel: at most " + std::to_string(cap) + " cells per mesh with this workgroup",
               PARAISO_ERR_UNSUPPORTED;
      if ((size_t)c->esize * (6 * (size_t)m.n[0] + 3) + 256 > (size_t)c->max_lds)
        return why = "resident kernel: mesh does not fit in LDS", PARAISO_ERR_UNSUPPORTED;
    }
  }
  if (v.lds == 2) {
    if (d == 1) return why = "register march (lds = 2) exists for 2D and 3D meshes", PARAISO_ERR_UNSUPPORTED;
    if (v.tile[0] != 64) return why = "register march: tile[0] must be 64 (one wave of columns)", PARAISO_ERR_UNSUPPORTED;
    if (!march_offsets_fit(c->meshes.data(), c->count))
      return why = "register march: a row (2D) or plane (3D) spans 4 GiB or more", PARAISO_ERR_UNSUPPORTED;
    if (!all_ghosts_fit(c->meshes.data(), c->count))
      return why = "register march: the ghost arrays of an analytic mesh pass 32-bit offsets", PARAISO_ERR_UNSUPPORTED;
    if (d == 2) {
      if (v.fuse)
        for (const auto& m : c->meshes)
          if (m.bc[0] != PARAISO_PERIODIC || m.bc[1] != PARAISO_PERIODIC)
            return why = "fused register march needs periodic boundaries", PARAISO_ERR_UNSUPPORTED;
      if (v.threads != 0 && (v.threads < 64 || v.threads > 256 || v.threads % 64))
        return why = "register march: threads must be 64, 128, 192 or 256", PARAISO_ERR_UNSUPPORTED;
    } else if (v.fuse) {
      for (const auto& m : c->meshes)
        if (m.bc[0] != PARAISO_PERIODIC || m.bc[1] != PARAISO_PERIODIC || m.bc[2] != PARAISO_PERIODIC)
          return why = "fused 3D register march needs periodic boundaries", PARAISO_ERR_UNSUPPORTED;
      if (v.tile[1] < 6 || v.tile[1] > 12)
        return why = "fused 3D register march: tile[1] (stage-1 rows = waves per block) must be 6..12",
               PARAISO_ERR_UNSUPPORTED;
      if (v.threads != 0 && v.threads != 64 * v.tile[1])
        return why = "fused 3D register march: threads must be 64 * tile[1]", PARAISO_ERR_UNSUPPORTED;
      if (march3d_fused_lds(v.tile[1], c->esize) + 16 * sizeof(double) + 64 > (size_t)c->max_lds)
        return why = "fused 3D register march: LDS of " + std::to_string(v.tile[1]) + " rows exceeds the limit",
               PARAISO_ERR_UNSUPPORTED;
    } else {
      if (v.tile[1] != 4 && v.tile[1] != 8)
        return why = "3D register march: tile[1] (rows = waves per block) must be 4 or 8", PARAISO_ERR_UNSUPPORTED;
      if (v.threads != 0 && v.threads != 64 * v.tile[1])
        return why = "3D register march: threads must be 64 * tile[1]", PARAISO_ERR_UNSUPPORTED;
    }
  }
  if (any_analytic(c->meshes.data(), c->count) && !(v.fuse == 0 && (v.lds == 1 || (v.lds == 2 && d == 2))))
    return why = "analytic boundaries run on the unfused LDS-tile kernel (lds = 1, fuse = 0) or, in 2D, the "
                 "one-stage register march (lds = 2, fuse = 0)",
           PARAISO_ERR_UNSUPPORTED;
  if (first_order(c->meshes[0]) && v.lds != 1)
    return why = "first-order reconstruction runs on the LDS-tile kernels (lds = 1)", PARAISO_ERR_UNSUPPORTED;
  if (v.manifest < 0 || v.manifest > 2) return why = "manifest must be 0, 1 or 2", PARAISO_ERR_UNSUPPORTED;
  if (v.manifest != 0 && v.lds != 1)
    return why = "manifest 1 and 2 are choices of the LDS-tile kernels (lds = 1)", PARAISO_ERR_UNSUPPORTED;
  if (v.manifest != 0 && (any_analytic(c->meshes.data(), c->count) || first_order(c->meshes[0])))
    return why = "kept face states: second-order meshes without analytic boundaries", PARAISO_ERR_UNSUPPORTED;
  if (v.persistent != 0 && v.persistent != 1) return why = "persistent must be 0 or 1", PARAISO_ERR_UNSUPPORTED;
  if (!(v.waves_per_eu == 0 || v.waves_per_eu == 3 || v.waves_per_eu == 4 || v.waves_per_eu == 5))
    return why = "waves_per_eu must be 0, 3, 4 or 5", PARAISO_ERR_UNSUPPORTED;
  // (the fused 3D march runs one wave per stage-1 row, up to 768 threads; its own check below)
  const bool fused3d = v.lds == 2 && c->ndim == 3 && v.fuse;
  // (the resident kernel's counts are checked above)
  if (v.threads != 0 && !fused3d && v.lds != 3 && (v.threads < 64 || v.threads > 512 || v.threads % 64))
    return why = "threads must be 0 or a multiple of 64 in [64, 512]", PARAISO_ERR_UNSUPPORTED;
  const int64_t tc = (int64_t)v.tile[0] * v.tile[1] * v.tile[2];
  if (tc > (1 << 22)) return why = "tile has more than 2^22 cells", PARAISO_ERR_UNSUPPORTED;
  return PARAISO_OK;
}

int apply_variant(paraiso_ctx* c, const paraiso_variant& vin) {
  std::string why;
  paraiso_variant v = vin;
  int rc = validate_variant(c, v, why);
  if (rc) return fail(rc, "variant: " + why);
  const int d = c->ndim, nf = d + 2;
  const int threads = v.lds == 3 ? (v.threads ? v.threads : resident_threads_for(max_cells(c->meshes.data(), c->count)))
                      : (v.lds == 2 && d == 3) ? 64 * v.tile[1] : (v.threads ? v.threads : 256);
  // tile of one work item: the variant's tile, or for the register march
  // (64 - 2H) columns by rows-per-wave times waves-per-block
  int et[3] = {v.tile[0], v.tile[1], v.tile[2]};
  if (v.lds == 2 && d == 2) {
    et[0] = 64 - 2 * (v.fuse ? 4 : 2);
    et[1] = v.fuse ? march2d_item_rows(threads / 64, v.tile[1]) : v.tile[1] * (threads / 64);
  } else if (v.lds == 2) {
    et[0] = v.fuse ? 56 : 60;              // 64 lanes less 4 (fused) or 2 halo columns per side
    et[1] = v.fuse ? v.tile[1] - 4 : v.tile[1];  // output rows: waves, less 4 stage-1 halo rows when fused
  }
  // items
  int64_t items = 0;
  for (int m = 0; m < c->count; ++m) {
    MeshDev& M = c->hm[m];
    int64_t nt = 1;
    for (int a = 0; a < 3; ++a) {
      M.nt[a] = (int)((M.n[a] + et[a] - 1) / et[a]);
      nt *= M.nt[a];
    }
    if (items + nt >= (int64_t(1) << 31)) return fail(PARAISO_ERR_UNSUPPORTED, "variant: too many tiles");
    M.item0 = (int)items;
    M.nitems = (int)nt;
    items += nt;
  }
  const int nitems = (int)items;
  // geometry
  LdsGeom G{};
  size_t shmem = 0;
  const int H = v.fuse ? 4 : 2;
  int e[3], t[3];
  for (int a = 0; a < 3; ++a) {
    t[a] = v.tile[a];
    e[a] = a < d ? v.tile[a] + 2 * H : 1;
  }
  G.halo = H;
  G.vin = make_box(e[0], e[1], e[2]);
  G.tile = make_box(t[0], t[1], t[2]);
  int c1[3];
  for (int a = 0; a < 3; ++a) c1[a] = (v.fuse && a < d) ? t[a] + 4 : t[a];
  G.c1 = make_box(c1[0], c1[1], c1[2]);
  int fmax_count = 0;
  for (int a = 0; a < 3; ++a) {
    int f[3] = {c1[0], c1[1], c1[2]};
    int f2[3] = {t[0], t[1], t[2]};
    if (a < d) {
      f[a] += 1;
      f2[a] += 1;
    }
    G.fx[a] = make_box(f[0], f[1], f[2]);
    G.fx2[a] = make_box(f2[0], f2[1], f2[2]);
    if (a < d) fmax_count = std::max(fmax_count, std::max(G.fx[a].count, G.fx2[a].count));
  }
  G.vstride = G.vin.count;
  G.fstride = fmax_count;
  if (v.lds == 3) {
    int64_t nmax = 1;
    for (const auto& m : c->meshes) nmax = std::max<int64_t>(nmax, m.n[0]);
    shmem = (size_t)c->esize * (6 * (size_t)nmax + 3);
  }
  G.rows = v.tile[1];
  if (v.lds == 2 && d == 2 && v.fuse && march2d_shares(threads / 64, v.tile[1])) {
    // each wave but the first leaves its first four stage-1 rows in LDS
    shmem = (size_t)c->esize * 4 * 4 * 64 * (threads / 64);
  }
  if (v.lds == 2 && d == 3) {
    const int nw = v.tile[1];
    shmem = v.fuse ? march3d_fused_lds(nw, c->esize)
                   : (size_t)c->esize * 5 * 64 * (2 * (size_t)(nw + 4) + 3 * (size_t)(nw + 1));
    if (shmem + 16 * sizeof(double) + 64 > (size_t)c->max_lds)
      return fail(PARAISO_ERR_UNSUPPORTED, "variant: 3D march needs " + std::to_string(shmem) + " bytes of LDS");
  }
  if (v.lds == 1) {
    // primitives, one axis' face fluxes and, when kept, the face values (lower and upper) of that axis
    shmem = (size_t)c->esize * nf * ((size_t)G.vstride + G.fstride + (v.manifest ? 2 * (size_t)G.vstride : 0));
    const size_t static_lds = 16 * sizeof(double) + 64;
    if (shmem + static_lds > (size_t)c->max_lds)
      return fail(PARAISO_ERR_UNSUPPORTED, "variant: LDS tile needs " + std::to_string(shmem) + " bytes, limit " +
                                               std::to_string(c->max_lds));
    if (G.tile.count > kMaxR * threads || G.c1.count > kMaxR * threads)
      return fail(PARAISO_ERR_UNSUPPORTED, "variant: more than " + std::to_string(kMaxR) +
                                               " cells per thread; use more threads or a smaller tile");
  }
  // fused direct needs 4 cells of halo along each axis inside the mesh's
  // periodic wrap; nothing else to check
  const int ws = waves_slot(v.waves_per_eu);
  Launch L;
  if (v.lds == 3) L.fn = c->tab->resident1d[threads == 512 ? 0 : 1];
  else if (v.lds == 2 && d == 3) L.fn = v.fuse ? c->tab->march3d_fused[ws] : c->tab->march3d_stage[ws];
  else if (v.lds == 2)
    L.fn = v.fuse ? c->tab->march_fused[ws]
                  : (any_analytic(c->meshes.data(), c->count) ? c->tab->march_stage_an[ws] : c->tab->march_stage[ws]);
  else if (v.lds == 1) {
    const int opt = (any_analytic(c->meshes.data(), c->count) ? kOptAnalytic : 0) |
                    (first_order(c->meshes[0]) ? kOptFirstOrder : 0);
    if (v.manifest) L.fn = v.fuse ? c->tab->fused_lds_keep[v.manifest - 1][ws] : c->tab->stage_lds_keep[v.manifest - 1][ws];
    else if (v.fuse) L.fn = opt ? c->tab->fused_lds_first[ws] : c->tab->fused_lds[ws];
    else L.fn = opt ? c->tab->stage_lds_opt[opt - 1][ws] : c->tab->stage_lds[ws];
  } else if (v.fuse) L.fn = c->tab->fused_direct[ws];
  else L.fn = c->tab->stage_direct[ws];
  if (!L.fn) return fail(PARAISO_ERR_UNSUPPORTED, "variant: no kernel for this combination");
  L.block = dim3(threads);
  L.shmem = shmem;
  L.with_geom = true;
  if (shmem > 65536) HIP_TRY(hipFuncSetAttribute(L.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  // grid: one workgroup per item, unless that grid passes the launch limit of
  // 2^32 work-items (very long rows of very few rows, tiny tiles): then the
  // persistent queue, which takes any number of items
  if (v.lds != 3 && (int64_t)nitems * threads >= (int64_t(1) << 32)) v.persistent = 1;
  int grid = nitems;
  if (v.persistent) {
    int per_cu = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, L.fn, threads, shmem));
    if (per_cu < 1) return fail(PARAISO_ERR_UNSUPPORTED, "variant: kernel does not fit on a CU");
    grid = std::min<int64_t>((int64_t)per_cu * c->num_cus, nitems);
    grid = std::max(grid, 1);
  }
  if (v.lds == 3) grid = c->count;
  L.grid = dim3(grid);
  {
    hipFuncAttributes fa{};
    HIP_TRY(hipFuncGetAttributes(&fa, L.fn));
    if (fa.maxThreadsPerBlock > 0 && threads > fa.maxThreadsPerBlock)
      return fail(PARAISO_ERR_UNSUPPORTED, "variant: kernel allows at most " + std::to_string(fa.maxThreadsPerBlock) +
                                               " threads per block");
  }
  // commit
  const int per = nitems / 8, rem = nitems % 8;
  for (int x = 0; x <= 8; ++x) c->xcd_begin[x] = x * per + std::min(x, rem);
  HIP_TRY(hipMemcpyAsync(c->d_meshes, c->hm.data(), sizeof(MeshDev) * c->count, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  drop_graphs(c);
  v.threads = threads;
  c->var = v;
  for (int a = 0; a < 3; ++a) c->eff_tile[a] = et[a];
  // kernels of different variants keep the work-queue ring differently: start clean
  {
    int rc2 = ctl_init(c, nullptr);
    if (rc2) return rc2;
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  c->fused = v.fuse != 0;
  c->lds = v.lds != 0;
  c->persistent = v.persistent != 0;
  c->resident = v.lds == 3;
  c->ghosts = v.lds == 2 && d == 2 && any_analytic(c->meshes.data(), c->count);
  c->ghost_blocks = 1;
  for (const auto& m : c->meshes)
    if (ghost_bytes(m))
      c->ghost_blocks = std::max<int>(c->ghost_blocks, (2 * ghost_stride((int)m.n[0], (int)m.n[1]) + 255) / 256);
  c->nitems = nitems;
  c->geom = G;
  c->step = L;
  // the six step graphs of paraiso_advance, captured and instantiated now so
  // that no advance pays for them (the resident kernel replays no graphs)
  if (!c->resident)
    for (int phase = 0; phase < 6; ++phase) {
      int rc3 = capture_graph(c, phase);
      if (rc3) return rc3;
    }
  return PARAISO_OK;
}

// The LDS-tile variant: every dimension, boundary and size.
void lds_variant(int ndim, paraiso_variant* v) {
  std::memset(v, 0, sizeof(*v));
  v->tile[0] = v->tile[1] = v->tile[2] = 1;
  v->lds = 1;
  v->threads = 256;
  if (ndim == 1) {
    v->tile[0] = 256;
    v->fuse = 1;
  } else if (ndim == 2) {
    v->tile[0] = 32;
    v->tile[1] = 16;
    v->fuse = 1;
  } else {
    v->tile[0] = 16;
    v->tile[1] = 8;
    v->tile[2] = 4;
    v->fuse = 0;
  }
}

// The default: the fastest family measured on an MI355X for the case.
//   1D: the resident kernel when every mesh fits one workgroup's LDS
//       (160 KiB on gfx950), else LDS tiles;
//   2D: the fused register march when every mesh is periodic on both axes
//       (FP32 20 rows x 4 waves, FP64 40 rows x 4 waves), else LDS tiles;
//   3D: the register march, 4 rows x 64-plane chunks, at most 168 VGPRs.
// Batches take the plain grid too, one workgroup per tile: on the 512-mesh
// batch it ran as fast as the persistent queue or faster for every family
// (fused 2D march +4%, one-stage march +19%, LDS tile equal, per-cell +9%),
// since the hardware starts a new workgroup as soon as one ends, while a
// persistent workgroup waits out two barriers and a device-scope atomic
// for every tile it pulls.
void default_variant(const paraiso_mesh* meshes, int count, paraiso_variant* v) {
  const int d = meshes[0].ndim;
  const bool f64 = meshes[0].dtype == PARAISO_F64;
  lds_variant(d, v);
  if (any_analytic(meshes, count)) {
    v->fuse = 0;  // ghosts at each stage's own time
    if (d == 2 && !first_order(meshes[0]) && march_offsets_fit(meshes, count) && all_ghosts_fit(meshes, count)) {
      // the one-stage register march with ghost arrays
      v->lds = 2;
      v->tile[0] = 64;
      v->tile[1] = 8;
      v->threads = 256;
      // FP64: 173 VGPRs uncapped (2 waves per SIMD); capped at 168 the kernel
      // runs 3, which also lets a 1024^2 mesh's 576 blocks be resident at once
      if (f64) v->waves_per_eu = 3;
    }
  } else if (first_order(meshes[0])) {
    // first-order reconstruction: the LDS-tile kernels only
  } else if (d == 1) {
    int64_t nmax = 1;
    for (int m = 0; m < count; ++m) nmax = std::max<int64_t>(nmax, meshes[m].n[0]);
    const size_t esize = f64 ? 8 : 4;
    if (nmax <= kResidentCells && esize * (6 * (size_t)nmax + 3) + 256 <= 163840) {
      v->lds = 3;
      v->fuse = 1;
      v->tile[0] = (int32_t)nmax;
      v->threads = resident_threads_for(nmax);
    }
  } else if (!march_offsets_fit(meshes, count)) {
    // rows or planes beyond the march kernels' 32-bit offsets: LDS tiles
  } else if (d == 2) {
    bool periodic = true;
    for (int m = 0; m < count; ++m)
      periodic = periodic && meshes[m].bc[0] == PARAISO_PERIODIC && meshes[m].bc[1] == PARAISO_PERIODIC;
    if (periodic) {
      v->tile[0] = 64;
      v->tile[1] = f64 ? 40 : 20;
      v->lds = 2;
      v->fuse = 1;
      v->threads = 256;
    }
  } else {
    v->tile[0] = 64;
    v->tile[1] = 4;
    v->tile[2] = 64;
    v->lds = 2;
    v->fuse = 0;
    v->waves_per_eu = 3;
    v->threads = 256;
  }
}

// The control-block area of the pinned staging buffer.
Ctl* pinned_ctl(paraiso_ctx* c) { return reinterpret_cast<Ctl*>(c->h_pin + c->pin_ctl); }

// Every analytic mesh needs its exact solution before it can be stepped.
int check_problems(const paraiso_ctx* c) {
  for (int m = 0; m < c->count; ++m)
    if (has_analytic(c->meshes[m]) && !c->analytic_set[m])
      return fail(PARAISO_ERR_INVALID_ARG,
                  "mesh " + std::to_string(m) + ": analytic boundary without a problem (paraiso_set_analytic)");
  return PARAISO_OK;
}

}  // namespace

extern "C" {

const char* paraiso_last_error(void) { return g_err; }

const char* paraiso_version(void) { return "paraiso-mi355x 0.1 (gfx950)"; }

int32_t paraiso_workspace_bytes(const paraiso_mesh* meshes, int32_t count, size_t* bytes) {
  if (!bytes) return fail(PARAISO_ERR_INVALID_ARG, "null output pointer");
  int rc = validate_meshes(meshes, count);
  if (rc) return rc;
  *bytes = layout_of(meshes, count).total;
  return PARAISO_OK;
}

int32_t paraiso_default_variant(const paraiso_mesh* meshes, int32_t count, paraiso_variant* v) {
  if (!v) return fail(PARAISO_ERR_INVALID_ARG, "null variant pointer");
  int rc = validate_meshes(meshes, count);
  if (rc) return rc;
  default_variant(meshes, count, v);
  return PARAISO_OK;
}

int32_t paraiso_init(const paraiso_mesh* meshes, int32_t count, void* workspace, size_t workspace_bytes,
                     void* hip_stream, paraiso_ctx** out) {
  if (!out) return fail(PARAISO_ERR_INVALID_ARG, "null context pointer");
  *out = nullptr;
  int rc = validate_meshes(meshes, count);
  if (rc) return rc;
  if (!workspace) return fail(PARAISO_ERR_INVALID_ARG, "null workspace");
  if ((uintptr_t)workspace % 256) return fail(PARAISO_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  Layout L = layout_of(meshes, count);
  if (workspace_bytes < L.total)
    return fail(PARAISO_ERR_WORKSPACE, "workspace has " + std::to_string(workspace_bytes) + " bytes, needs " +
                                           std::to_string(L.total));
  paraiso_ctx* c = new (std::nothrow) paraiso_ctx();
  if (!c) return fail(PARAISO_ERR_INVALID_ARG, "out of host memory");
  c->count = count;
  c->ndim = meshes[0].ndim;
  c->dtype = meshes[0].dtype;
  c->esize = c->dtype == PARAISO_F32 ? 4 : 8;
  c->meshes.assign(meshes, meshes + count);
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)workspace;
  c->ws_bytes = workspace_bytes;
  c->L = L;
  c->d_meshes = (MeshDev*)(c->ws + L.meshes);
  c->d_ctl = (Ctl*)(c->ws + L.ctl);
  c->d_params = (Params*)(c->ws + L.params);
  c->d_dt = (double*)(c->ws + L.dt);
  c->d_queue = (unsigned*)(c->ws + L.queue);
  c->d_out = (double*)(c->ws + L.out);
  c->d_partials = (double*)(c->ws + L.partials);
  c->tab = table_for(c->dtype, c->ndim);
  auto bail = [&](int code) {
    if (c->cap) hipStreamDestroy(c->cap);
    if (c->h_pin) hipHostFree(c->h_pin);
    delete c;
    return code;
  };
  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, c->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&c->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
  c->pin_ctl = align256((L.dt - L.params) + sizeof(double) * count);
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_pin, c->pin_ctl + sizeof(Ctl) * count, hipHostMallocDefault);
  if (e != hipSuccess) return bail(hip_fail("device query", e));
  // host mesh table
  c->hm.resize(count);
  size_t u1off = L.u1;
  size_t goff = L.ghost;
  int chunk = 0;
  for (int m = 0; m < count; ++m) {
    const paraiso_mesh& pm = meshes[m];
    MeshDev& M = c->hm[m];
    std::memset(&M, 0, sizeof(M));
    const int nf = pm.ndim + 2;
    for (int b = 0; b < 2; ++b)
      for (int q = 0; q < kMaxFields; ++q) M.s[b][q] = q < nf ? pm.state[b][q] : nullptr;
    const size_t fbytes = align256((size_t)cells_of(pm) * c->esize);
    for (int q = 0; q < kMaxFields; ++q) M.w[q] = q < nf ? (void*)(c->ws + u1off + q * fbytes) : nullptr;
    u1off += nf * fbytes;
    M.ghost = ghost_bytes(pm) ? (void*)(c->ws + goff) : nullptr;
    goff += ghost_bytes(pm);
    double vol = 1.0;
    for (int a = 0; a < 3; ++a) {
      M.n[a] = (int)pm.n[a];
      M.bc[a] = a < pm.ndim ? pm.bc[a] : PARAISO_PERIODIC;
      M.dx[a] = a < pm.ndim ? pm.dx[a] : 1.0;
      M.inv_dx[a] = 1.0 / M.dx[a];
      if (a < pm.ndim) vol *= pm.dx[a];
    }
    M.gamma = pm.gamma;
    M.inv_gm1 = 1.0 / (pm.gamma - 1.0);
    M.vol = vol;
    M.ncells = (int)cells_of(pm);
    M.chunk0 = chunk;
    M.nchunks = (int)(((int64_t)M.ncells + kChunk - 1) / kChunk);  // ncells + kChunk - 1 may pass 2^31 - 1
    chunk += M.nchunks;
  }
  paraiso_variant v;
  default_variant(meshes, count, &v);
  rc = apply_variant(c, v);
  if (rc == PARAISO_ERR_UNSUPPORTED) {
    // a device with less LDS than gfx950: the LDS-tile family always applies
    lds_variant(c->ndim, &v);
    if (any_analytic(meshes, count)) v.fuse = 0;
    rc = apply_variant(c, v);
  }
  if (rc) return bail(rc);
  rc = ctl_init(c, nullptr);
  if (rc) return bail(rc);
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return bail(hip_fail("init", e));
  c->ctl_ready = true;
  c->analytic_set.assign(count, 0);
  *out = c;
  return PARAISO_OK;
}

int32_t paraiso_set_variant(paraiso_ctx* c, const paraiso_variant* v) {
  if (!c || !v) return fail(PARAISO_ERR_INVALID_ARG, "null argument");
  paraiso_variant old = c->var;
  int rc = apply_variant(c, *v);
  if (rc) {
    const std::string msg = g_err;
    apply_variant(c, old);
    paraiso_set_error(msg);
  }
  return rc;
}

int32_t paraiso_get_variant(const paraiso_ctx* c, paraiso_variant* v) {
  if (!c || !v) return fail(PARAISO_ERR_INVALID_ARG, "null argument");
  *v = c->var;
  return PARAISO_OK;
}

int32_t paraiso_current(const paraiso_ctx* c, int32_t* idx) {
  if (!c || !idx) return fail(PARAISO_ERR_INVALID_ARG, "null argument");
  *idx = c->cur;
  return PARAISO_OK;
}

int32_t paraiso_cfl_dt(paraiso_ctx* c, double cfl, double* dt_out) {
  if (!c || !dt_out) return fail(PARAISO_ERR_INVALID_ARG, "null argument");
  if (!(cfl > 0.0 && cfl <= 1.0)) return fail(PARAISO_ERR_INVALID_ARG, "cfl must be in (0, 1]");
  int rc = ctl_init(c, nullptr);
  if (!rc) rc = launch_cfl(c);
  if (rc) return rc;
  const Ctl* h = pinned_ctl(c);
  HIP_TRY(hipMemcpyAsync((void*)h, c->d_ctl, sizeof(Ctl) * c->count, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (int m = 0; m < c->count; ++m) {
    if (h[m].flags[c->ring]) return fail(PARAISO_ERR_NONFINITE, "mesh " + std::to_string(m) + ": non-physical state");
    uint64_t bits = qbits_max(h[m], c->ring);
    double q;
    std::memcpy(&q, &bits, sizeof(q));
    if (!(q > 0.0)) return fail(PARAISO_ERR_NONFINITE, "mesh " + std::to_string(m) + ": no signal speed");
    dt_out[m] = cfl / q;
  }
  return PARAISO_OK;
}

int32_t paraiso_step(paraiso_ctx* c, const double* dt) {
  if (!c || !dt) return fail(PARAISO_ERR_INVALID_ARG, "null argument");
  if (int rc0 = check_problems(c)) return rc0;
  for (int m = 0; m < c->count; ++m)
    if (!(dt[m] >= 0.0) || !std::isfinite(dt[m])) return fail(PARAISO_ERR_INVALID_ARG, "dt must be finite and >= 0");
  HIP_TRY(hipMemcpyAsync(c->d_dt, dt, sizeof(double) * c->count, hipMemcpyHostToDevice, c->stream));
  int rc = enqueue_step(c, c->cur, c->ring, true, c->stream);
  if (rc) return rc;
  c->cur ^= 1;
  c->ring = (c->ring + 1) % 3;
  return PARAISO_OK;
}

int32_t paraiso_advance(paraiso_ctx* c, double t_end, double cfl, int64_t max_steps, double* t_inout,
                        int64_t* steps_out) {
  if (!c || !t_inout || !steps_out) return fail(PARAISO_ERR_INVALID_ARG, "null argument");
  if (int rc0 = check_problems(c)) return rc0;
  if (!(cfl > 0.0 && cfl <= 1.0)) return fail(PARAISO_ERR_INVALID_ARG, "cfl must be in (0, 1]");
  if (max_steps < 0) return fail(PARAISO_ERR_INVALID_ARG, "max_steps must be >= 0");
  if (std::isnan(t_end) || t_end == -INFINITY) return fail(PARAISO_ERR_INVALID_ARG, "t_end must be a number or +inf");
  for (int m = 0; m < c->count; ++m)
    if (!std::isfinite(t_inout[m])) return fail(PARAISO_ERR_INVALID_ARG, "t_inout must be finite");
  const Params p{t_end, cfl, (long long)max_steps};
  int rc = PARAISO_OK;
  if (c->count <= kInlineMeshes) {
    // parameter block and start times as kernel arguments: no copy
    InlineTimes t0{};
    for (int m = 0; m < c->count; ++m) t0.t[m] = t_inout[m];
    hipLaunchKernelGGL(k_advance_init, dim3(1), dim3(64), 0, c->stream, c->d_ctl, c->d_params, p, t0, c->count,
                       c->ring, c->d_queue);
    HIP_TRY(hipGetLastError());
  } else {
    // the parameter block and the start times, adjacent in the workspace, in one copy
    const size_t dt_off = c->L.dt - c->L.params;
    std::memcpy(c->h_pin, &p, sizeof(p));
    std::memcpy(c->h_pin + dt_off, t_inout, sizeof(double) * c->count);
    HIP_TRY(hipMemcpyAsync(c->d_params, c->h_pin, dt_off + sizeof(double) * c->count, hipMemcpyHostToDevice,
                           c->stream));
    rc = ctl_init(c, c->d_dt);
  }
  if (!rc) rc = launch_cfl(c);
  if (rc) return rc;
  Ctl* h = pinned_ctl(c);
  if (c->resident) {
    // the whole advance in one launch; it counts as one buffer flip
    rc = enqueue_step(c, c->cur, c->ring, false, c->stream);
    if (rc) return rc;
    c->cur ^= 1;
    c->ring = (c->ring + 1) % 3;
    HIP_TRY(hipMemcpyAsync(h, c->d_ctl, sizeof(Ctl) * c->count, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int m = 0; m < c->count; ++m) {
      t_inout[m] = h[m].t[c->ring];
      steps_out[m] = h[m].steps[c->ring];
    }
    for (int m = 0; m < c->count; ++m)
      if (h[m].flags[c->ring]) return fail(PARAISO_ERR_NONFINITE, "mesh " + std::to_string(m) + ": non-physical state");
    return PARAISO_OK;
  }
  std::vector<double> t0(t_inout, t_inout + c->count);
  int64_t launched = 0;
  int64_t chunk = std::isinf(t_end) ? max_steps : std::min<int64_t>(max_steps, 32);
  for (;;) {
    rc = run_steps(c, chunk);
    if (rc) return rc;
    launched += chunk;
    HIP_TRY(hipMemcpyAsync(h, c->d_ctl, sizeof(Ctl) * c->count, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    bool done = true;
    int64_t want = 0;
    for (int m = 0; m < c->count; ++m) {
      if (h[m].flags[c->ring]) {
        for (int k = 0; k < c->count; ++k) {
          t_inout[k] = h[k].t[c->ring];
          steps_out[k] = h[k].steps[c->ring];
        }
        return fail(PARAISO_ERR_NONFINITE, "mesh " + std::to_string(m) + ": non-physical state");
      }
      const double t = h[m].t[c->ring];
      const int64_t st = h[m].steps[c->ring];
      if (t < t_end && st < max_steps) {
        done = false;
        int64_t est = max_steps - st;
        if (st > 0 && t > t0[m]) {
          const double avg = (t - t0[m]) / (double)st;
          const double need = std::ceil((t_end - t) / avg * 1.05) + 2.0;
          if (need < (double)est) est = (int64_t)need;
        }
        want = std::max(want, est);
      }
    }
    if (done) break;
    chunk = std::max<int64_t>(1, std::min<int64_t>(want, max_steps));
  }
  for (int m = 0; m < c->count; ++m) {
    t_inout[m] = h[m].t[c->ring];
    steps_out[m] = h[m].steps[c->ring];
  }
  return PARAISO_OK;
}

int32_t paraiso_set_analytic(paraiso_ctx* c, int32_t mesh, const paraiso_analytic* an) {
  if (!c || !an) return fail(PARAISO_ERR_INVALID_ARG, "null argument");
  if (mesh < 0 || mesh >= c->count) return fail(PARAISO_ERR_INVALID_ARG, "mesh index out of range");
  const paraiso_mesh& pm = c->meshes[mesh];
  if (!has_analytic(pm)) return fail(PARAISO_ERR_INVALID_ARG, "mesh has no PARAISO_ANALYTIC axis");
  if (an->kind != PARAISO_ENTROPY_WAVE && an->kind != PARAISO_SOUND_WAVE && an->kind != PARAISO_SHOCK_TUBE)
    return fail(PARAISO_ERR_INVALID_ARG, "kind must be PARAISO_ENTROPY_WAVE, PARAISO_SOUND_WAVE or PARAISO_SHOCK_TUBE");
  if (!std::isfinite(an->angle)) return fail(PARAISO_ERR_INVALID_ARG, "angle must be finite");
  if (pm.ndim == 1 && an->angle != 0.0) return fail(PARAISO_ERR_INVALID_ARG, "angle must be 0 in 1D");
  if (an->kind == PARAISO_SOUND_WAVE && !(std::fabs(an->amplitude) < 1.0))
    return fail(PARAISO_ERR_INVALID_ARG, "sound-wave amplitude must be finite with |amplitude| < 1");
  Analytic A{};
  A.kind = an->kind;
  A.cs = pm.ndim > 1 ? std::cos(an->angle) : 1.0;
  A.sn = pm.ndim > 1 ? std::sin(an->angle) : 0.0;
  A.amp = an->kind == PARAISO_SOUND_WAVE ? an->amplitude : 0.0;
  if (an->kind == PARAISO_SHOCK_TUBE) {
    const double L[3] = {1.0, 0.0, 1.0}, R[3] = {0.125, 0.0, 0.1};
    if (!riemann_star_state(pm.gamma, L, R, &A.ps, &A.us))
      return fail(PARAISO_ERR_INVALID_ARG, "shock tube: vacuum forms for this gamma");
  }
  c->hm[mesh].an = A;
  HIP_TRY(hipMemcpyAsync(&c->d_meshes[mesh], &c->hm[mesh], sizeof(MeshDev), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->analytic_set[mesh] = 1;
  return PARAISO_OK;
}

int32_t paraiso_exact_state(paraiso_ctx* c, int32_t mesh, double t, int32_t buffer) {
  if (!c) return fail(PARAISO_ERR_INVALID_ARG, "null argument");
  if (mesh < 0 || mesh >= c->count) return fail(PARAISO_ERR_INVALID_ARG, "mesh index out of range");
  if (buffer != 0 && buffer != 1) return fail(PARAISO_ERR_INVALID_ARG, "buffer must be 0 or 1");
  if (!std::isfinite(t)) return fail(PARAISO_ERR_INVALID_ARG, "t must be finite");
  if (!c->analytic_set[mesh]) return fail(PARAISO_ERR_INVALID_ARG, "mesh has no analytic problem set");
  Args a = base_args(c);
  int m = mesh, b = buffer;
  void* args[] = {(void*)&a, (void*)&m, (void*)&t, (void*)&b};
  const int64_t cells = cells_of(c->meshes[mesh]);
  HIP_TRY(hipLaunchKernel(c->tab->exact_state, dim3((unsigned)((cells + 255) / 256)), dim3(256), args, 0,
                          c->stream));
  return PARAISO_OK;
}

int32_t paraiso_set_time(paraiso_ctx* c, const double* t) {
  if (!c || !t) return fail(PARAISO_ERR_INVALID_ARG, "null argument");
  for (int m = 0; m < c->count; ++m)
    if (!std::isfinite(t[m])) return fail(PARAISO_ERR_INVALID_ARG, "t must be finite");
  HIP_TRY(hipMemcpyAsync(c->d_dt, t, sizeof(double) * c->count, hipMemcpyHostToDevice, c->stream));
  int rc = ctl_init(c, c->d_dt);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return PARAISO_OK;
}

int32_t paraiso_get_time(paraiso_ctx* c, double* t_out) {
  if (!c || !t_out) return fail(PARAISO_ERR_INVALID_ARG, "null argument");
  std::vector<Ctl> h(c->count);
  HIP_TRY(hipMemcpyAsync(h.data(), c->d_ctl, sizeof(Ctl) * c->count, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (int m = 0; m < c->count; ++m) t_out[m] = h[m].t[c->ring];
  return PARAISO_OK;
}

int32_t paraiso_totals(paraiso_ctx* c, double* out) {
  if (!c || !out) return fail(PARAISO_ERR_INVALID_ARG, "null argument");
  Args a = base_args(c);
  a.src = c->cur;
  void* args[] = {(void*)&a};
  HIP_TRY(hipLaunchKernel(c->tab->totals_partial, dim3(c->L.total_chunks), dim3(256), args, 0, c->stream));
  void* args2[] = {(void*)&a, (void*)&c->d_out};
  HIP_TRY(hipLaunchKernel(c->tab->totals_final, dim3(c->count), dim3(256), args2, 0, c->stream));
  const int nf = c->ndim + 2;
  std::vector<double> h((size_t)c->count * nf);
  HIP_TRY(hipMemcpyAsync(h.data(), c->d_out, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  std::memcpy(out, h.data(), sizeof(double) * h.size());
  return PARAISO_OK;
}

int32_t paraiso_destroy(paraiso_ctx* c) {
  if (!c) return PARAISO_OK;
  drop_graphs(c);
  if (c->cap) hipStreamDestroy(c->cap);
  if (c->h_pin) hipHostFree(c->h_pin);
  delete c;
  return PARAISO_OK;
}

}  // extern "C"
