// paraiso_cfl_dt_static: the CFL time step of up to PARAISO_STATIC_MESHES
// meshes without a context or a caller's workspace, for callers that cannot
// allocate device memory.  It runs the same reduction kernel as
// paraiso_cfl_dt (k_cfl: FP64 per-cell term, wave shuffles, one atomic
// maximum per block) over a mesh table and control blocks that live in a
// file-scope device array instead of a workspace.
//
// Nothing here allocates: the host side works in fixed-size arrays on the
// stack, errors go to the fixed thread-local message buffer, and the device
// side uses `scratch`, whose address on each device comes from
// hipGetSymbolAddress on that device (the array's name in host code is only
// a host-side stand-in).  Every call on a device shares that device's
// scratch: calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "euler_common.h"
#include "kernel_table.h"
#include "paraiso.h"

void paraiso_set_error_text(const char* msg);

namespace paraiso {
namespace {

constexpr size_t round256(size_t x) { return (x + 255) & ~size_t(255); }
constexpr size_t kTableBytes = round256(sizeof(MeshDev) * PARAISO_STATIC_MESHES);
constexpr size_t kCtlBytes = round256(sizeof(Ctl) * PARAISO_STATIC_MESHES);
constexpr size_t kScratchBytes = kTableBytes + kCtlBytes;
static_assert(kScratchBytes <= 48 * 1024, "static scratch: at most 48 KiB per device");

// The mesh table (MeshDev[PARAISO_STATIC_MESHES]) followed by the control
// blocks (Ctl[PARAISO_STATIC_MESHES]); each device holds its own copy.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device

int fail(int code, const char* msg) {
  paraiso_set_error_text(msg);
  return code;
}

// Zero n 8-byte words: the control blocks are cleared by an ordinary kernel
// launch on the caller's stream, not a memset.
static_assert(sizeof(Ctl) % 8 == 0, "control blocks are whole 8-byte words");
__global__ void __launch_bounds__(256) k_zero_words(unsigned long long* p, int n) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < n) p[i] = 0ull;
}

// A HIP call failed: report it and take it off HIP's per-thread error record.
int hip_fail(hipError_t e) {
  (void)hipGetLastError();
  return fail(PARAISO_ERR_HIP, hipGetErrorString(e));
}

// The device address of this device's scratch, looked up once per device
// with that device current.
int scratch_address(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) return fail(PARAISO_ERR_UNSUPPORTED, "cfl_dt_static: device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      return e != hipSuccess ? hip_fail(e) : fail(PARAISO_ERR_HIP, "hipGetSymbolAddress gave no address");
    }
    g_scratch_ptr[device] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_ptr[device];
  return PARAISO_OK;
}

const KernelTable* table(int dtype, int ndim) {
  if (dtype == PARAISO_F32) return ndim == 1 ? table_f32_1() : (ndim == 2 ? table_f32_2() : table_f32_3());
  return ndim == 1 ? table_f64_1() : (ndim == 2 ? table_f64_2() : table_f64_3());
}

// What the reduction reads of a mesh: element type, sizes, cell sizes, gamma
// and the fields of the chosen buffer.
int check_mesh(const paraiso_mesh& m, const paraiso_mesh& first, int buffer) {
  if (m.ndim < 1 || m.ndim > 3) return fail(PARAISO_ERR_INVALID_ARG, "cfl_dt_static: ndim must be 1, 2 or 3");
  if (m.dtype != PARAISO_F32 && m.dtype != PARAISO_F64)
    return fail(PARAISO_ERR_INVALID_ARG, "cfl_dt_static: dtype must be PARAISO_F32 or PARAISO_F64");
  if (m.ndim != first.ndim || m.dtype != first.dtype)
    return fail(PARAISO_ERR_INVALID_ARG, "cfl_dt_static: all meshes must share ndim and dtype");
  if (!(m.gamma > 1.0) || !std::isfinite(m.gamma))
    return fail(PARAISO_ERR_INVALID_ARG, "cfl_dt_static: gamma must be finite and > 1");
  int64_t cells = 1;
  for (int a = 0; a < 3; ++a) {
    if (m.n[a] < 1 || m.n[a] > (int64_t(1) << 30)) return fail(PARAISO_ERR_INVALID_ARG, "cfl_dt_static: n[a] out of range");
    if (a >= m.ndim && m.n[a] != 1) return fail(PARAISO_ERR_INVALID_ARG, "cfl_dt_static: n[a] must be 1 for a >= ndim");
    if (a < m.ndim && (!(m.dx[a] > 0.0) || !std::isfinite(m.dx[a])))
      return fail(PARAISO_ERR_INVALID_ARG, "cfl_dt_static: dx[a] must be finite and > 0");
    cells *= m.n[a];
  }
  if (cells >= (int64_t(1) << 31)) return fail(PARAISO_ERR_UNSUPPORTED, "cfl_dt_static: more than 2^31 - 1 cells");
  for (int q = 0; q < m.ndim + 2; ++q) {
    const uintptr_t p = (uintptr_t)m.state[buffer][q];
    if (!p) return fail(PARAISO_ERR_INVALID_ARG, "cfl_dt_static: null state pointer");
    if (p % 16) return fail(PARAISO_ERR_INVALID_ARG, "cfl_dt_static: state arrays must be 16-byte aligned");
  }
  return PARAISO_OK;
}

}  // namespace
}  // namespace paraiso

using namespace paraiso;

extern "C" int32_t paraiso_cfl_dt_static(const paraiso_mesh* meshes, int32_t count, int32_t buffer, double cfl,
                                         double* dt_out, void* hip_stream) {
  if (!meshes || !dt_out) return fail(PARAISO_ERR_INVALID_ARG, "cfl_dt_static: null argument");
  if (count < 1) return fail(PARAISO_ERR_INVALID_ARG, "cfl_dt_static: count must be >= 1");
  if (count > PARAISO_STATIC_MESHES)
    return fail(PARAISO_ERR_UNSUPPORTED,
                "cfl_dt_static: count exceeds PARAISO_STATIC_MESHES, the capacity of the static scratch");
  if (buffer != 0 && buffer != 1) return fail(PARAISO_ERR_INVALID_ARG, "cfl_dt_static: buffer must be 0 or 1");
  if (!(cfl > 0.0 && cfl <= 1.0)) return fail(PARAISO_ERR_INVALID_ARG, "cfl_dt_static: cfl must be in (0, 1]");
  for (int m = 0; m < count; ++m)
    if (int rc = check_mesh(meshes[m], meshes[0], buffer)) return rc;

  int device = 0;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return hip_fail(e);
  unsigned char* base = nullptr;
  if (int rc = scratch_address(device, &base)) return rc;
  MeshDev* d_table = reinterpret_cast<MeshDev*>(base);
  Ctl* d_ctl = reinterpret_cast<Ctl*>(base + kTableBytes);
  hipStream_t stream = (hipStream_t)hip_stream;

  // the mesh table: what k_cfl reads (fields, sizes, chunk numbering)
  MeshDev h_table[PARAISO_STATIC_MESHES];
  std::memset(h_table, 0, sizeof(MeshDev) * count);
  int chunks = 0;
  for (int m = 0; m < count; ++m) {
    const paraiso_mesh& pm = meshes[m];
    MeshDev& M = h_table[m];
    for (int b = 0; b < 2; ++b)
      for (int q = 0; q < pm.ndim + 2; ++q) M.s[b][q] = pm.state[buffer][q];
    for (int a = 0; a < 3; ++a) {
      M.n[a] = (int)pm.n[a];
      M.dx[a] = a < pm.ndim ? pm.dx[a] : 1.0;
      M.inv_dx[a] = 1.0 / M.dx[a];
    }
    M.gamma = pm.gamma;
    M.inv_gm1 = 1.0 / (pm.gamma - 1.0);
    M.ncells = (int)(pm.n[0] * pm.n[1] * pm.n[2]);
    M.chunk0 = chunks;
    M.nchunks = (int)(((int64_t)M.ncells + kChunk - 1) / kChunk);  // ncells + kChunk - 1 may pass 2^31 - 1
    chunks += M.nchunks;
  }
  e = hipMemcpyAsync(d_table, h_table, sizeof(MeshDev) * count, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(e);
  // the control blocks start at zero: the last call's maxima and flags stay in scratch
  const int words = (int)(sizeof(Ctl) * count / 8);
  hipLaunchKernelGGL(k_zero_words, dim3((words + 255) / 256), dim3(256), 0, stream,
                     reinterpret_cast<unsigned long long*>(d_ctl), words);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e);

  Args a;
  std::memset(&a, 0, sizeof(a));
  a.meshes = d_table;
  a.ctl = d_ctl;
  a.nmeshes = count;
  a.src = 0;  // the table's buffer 0 and 1 both name the caller's `buffer`
  a.ring = 0;
  void* args[] = {(void*)&a};
  e = hipLaunchKernel(table(meshes[0].dtype, meshes[0].ndim)->cfl, dim3(chunks), dim3(256), args, 0, stream);
  Ctl h_ctl[PARAISO_STATIC_MESHES];
  if (e == hipSuccess) e = hipMemcpyAsync(h_ctl, d_ctl, sizeof(Ctl) * count, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e);
  for (int m = 0; m < count; ++m) {
    double q;
    const unsigned long long bits = qbits_max(h_ctl[m], 0);
    std::memcpy(&q, &bits, sizeof(q));
    if (h_ctl[m].flags[0] || !(q > 0.0)) return fail(PARAISO_ERR_NONFINITE, "cfl_dt_static: non-physical state");
    dt_out[m] = cfl / q;
  }
  return PARAISO_OK;
}
