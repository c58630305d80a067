// The linear-wave example of the paper (section "An Example of Orthotope
// Machine Data-Flow Graph"): f_t = g, g_t = c^2 f_xx on a periodic line,
//   f^{n+1}[i] = f^n[i] + dt g^n[i]
//   g^{n+1}[i] = g^n[i] + (c^2 dt / dx^2)(f^{n+1}[i+1] + f^{n+1}[i-1] - 2 f^{n+1}[i])
// with the discrete energy after every step,
//   E^{n+1} = sum_i (c^2 ((f^{n+1}[i+1] - f^{n+1}[i-1]) / 2dx)^2 + ((g^n[i] + g^{n+1}[i]) / 2)^2) dx / 2.
//
// One workgroup runs all steps of one line.  Thread t holds the R = ceil(n /
// 256) consecutive cells [tR, tR + R) in registers (the kernel is
// instantiated for R up to 1, 2, 3, 4, 6, 8, 12 and 16), so all but the two end
// cells find their neighbours in registers; the end values of every thread
// go through LDS (double-buffered by step parity), which costs one barrier
// per step.  The energy is summed in FP64 in a fixed order (per thread in
// cell order, a butterfly within each wave, the waves in order); the
// per-wave partials of a step are added by thread 0 after the next step's
// barrier, so that barrier is the only one.  Many lines run side by side,
// one workgroup each.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "paraiso.h"

void paraiso_set_error(const std::string& msg);

namespace {

constexpr int kWaveThreads = 256;

struct WaveDev {
  int n;
  int pad_;
  double k;        // c^2 dt / dx^2
  double dt;
  double c2;       // c^2
  double inv2dx;   // 1 / (2 dx)
  double half_dx;  // dx / 2
  double* f;
  double* g;
  double* energy;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One step of the cells a thread holds (cnt <= R of them; FULL: cnt == R,
// no per-cell predicates).  f holds f^{n+1} on entry; returns the thread's
// energy sum, in cell order, two interleaved accumulators.
template <int R, bool FULL>
__device__ __forceinline__ double wave_cells(const WaveDev& P, double* f, double* g, int cnt, double left_end,
                                             double right_end) {
  double e0 = 0.0, e1 = 0.0;
  double fl = left_end;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (FULL || r < cnt) {
      const double fr = (FULL ? r + 1 < R : r + 1 < cnt) ? f[r + 1 < R ? r + 1 : r] : right_end;
      const double g1 = g[r] + P.k * (fr + fl - 2.0 * f[r]);
      const double dfdx = (fr - fl) * P.inv2dx;
      const double gm = (g[r] + g1) * 0.5;
      const double term = (P.c2 * dfdx * dfdx + gm * gm) * P.half_dx;
      if (r & 1) e1 += term; else e0 += term;
      g[r] = g1;
      fl = f[r];
    }
  }
  return e0 + e1;
}

template <int R>
__global__ void __launch_bounds__(kWaveThreads) k_wave1d(const WaveDev* probs, long long steps) {
  __shared__ double sFirst[2][kWaveThreads], sLast[2][kWaveThreads];
  __shared__ double sPart[2][kWaveThreads / 64];
  const WaveDev P = probs[blockIdx.x];
  const int tid = threadIdx.x;
  const int n = P.n;
  if (n > R * kWaveThreads) return;                      // a line longer than the launch allows: untouched
  const int Rl = (n + kWaveThreads - 1) / kWaveThreads;  // cells per thread of this line, <= R
  const int active = (n + Rl - 1) / Rl;                  // threads holding cells
  const int i0 = tid * Rl;
  const int cnt = tid < active ? min(Rl, n - i0) : 0;
  const int prev = tid == 0 ? active - 1 : tid - 1;      // holder of cell i0 - 1 (periodic)
  const int next = tid == active - 1 ? 0 : tid + 1;      // holder of cell i0 + cnt
  const bool full = cnt == R;
  double f[R], g[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    f[r] = r < cnt ? P.f[i0 + r] : 0.0;
    g[r] = r < cnt ? P.g[i0 + r] : 0.0;
  }
  for (long long s = 0; s < steps; ++s) {
    const int b = (int)(s & 1);
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r < cnt) f[r] = f[r] + P.dt * g[r];
    if (cnt > 0) {
      sFirst[b][tid] = f[0];
      double last = f[0];
#pragma unroll
      for (int r = 1; r < R; ++r)
        if (r == cnt - 1) last = f[r];
      sLast[b][tid] = last;
    }
    __syncthreads();
    if (tid == 0 && s > 0 && P.energy) {
      double tot = 0.0;
#pragma unroll
      for (int w = 0; w < kWaveThreads / 64; ++w) tot += sPart[b ^ 1][w];
      P.energy[s - 1] = tot;
    }
    double e = 0.0;
    if (cnt > 0) {
      const double left_end = sLast[b][prev];
      const double right_end = sFirst[b][next];
      e = full ? wave_cells<R, true>(P, f, g, cnt, left_end, right_end)
               : wave_cells<R, false>(P, f, g, cnt, left_end, right_end);
    }
    e = wave_sum(e);
    if ((tid & 63) == 0) sPart[b][tid >> 6] = e;
  }
  __syncthreads();
  if (tid == 0 && steps > 0 && P.energy) {
    double tot = 0.0;
#pragma unroll
    for (int w = 0; w < kWaveThreads / 64; ++w) tot += sPart[(steps - 1) & 1][w];
    P.energy[steps - 1] = tot;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r < cnt) {
      P.f[i0 + r] = f[r];
      P.g[i0 + r] = g[r];
    }
  }
}

// Cells per thread of the instantiated kernels, and the kernel for a launch
// whose longest line has max_cells cells.
constexpr int kWaveR[] = {1, 2, 3, 4, 6, 8, 12, 16};

const void* wave_kernel(int64_t max_cells) {
  const int need = (int)((max_cells + kWaveThreads - 1) / kWaveThreads);
  if (need <= 1) return (const void*)k_wave1d<1>;
  if (need <= 2) return (const void*)k_wave1d<2>;
  if (need <= 3) return (const void*)k_wave1d<3>;
  if (need <= 4) return (const void*)k_wave1d<4>;
  if (need <= 6) return (const void*)k_wave1d<6>;
  if (need <= 8) return (const void*)k_wave1d<8>;
  if (need <= 12) return (const void*)k_wave1d<12>;
  return (const void*)k_wave1d<16>;
}

int wave_fail(int code, const std::string& msg) {
  if (code == PARAISO_ERR_HIP) (void)hipGetLastError();  // not left for the caller's next HIP call
  paraiso_set_error(msg);
  return code;
}

size_t wave_table_bytes(int count) { return ((size_t)count * sizeof(WaveDev) + 255) & ~size_t(255); }

}  // namespace

extern "C" {

int32_t paraiso_wave_workspace_bytes(int32_t count, size_t* bytes) {
  if (!bytes) return wave_fail(PARAISO_ERR_INVALID_ARG, "null output pointer");
  if (count < 1) return wave_fail(PARAISO_ERR_INVALID_ARG, "count must be >= 1");
  *bytes = wave_table_bytes(count);
  return PARAISO_OK;
}

int32_t paraiso_wave_prepare(const paraiso_wave* probs, int32_t count, void* workspace, size_t workspace_bytes,
                             void* hip_stream) {
  if (!probs || !workspace) return wave_fail(PARAISO_ERR_INVALID_ARG, "null argument");
  if (count < 1) return wave_fail(PARAISO_ERR_INVALID_ARG, "count must be >= 1");
  if ((uintptr_t)workspace % 256) return wave_fail(PARAISO_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (workspace_bytes < wave_table_bytes(count))
    return wave_fail(PARAISO_ERR_WORKSPACE, "workspace has " + std::to_string(workspace_bytes) + " bytes, needs " +
                                                std::to_string(wave_table_bytes(count)));
  WaveDev* host = new (std::nothrow) WaveDev[count];
  if (!host) return wave_fail(PARAISO_ERR_INVALID_ARG, "out of host memory");
  for (int m = 0; m < count; ++m) {
    const paraiso_wave& p = probs[m];
    const std::string w = "line " + std::to_string(m) + ": ";
    int rc = PARAISO_OK;
    std::string why;
    if (p.n < 3 || p.n > PARAISO_WAVE_MAX_CELLS) {
      rc = PARAISO_ERR_INVALID_ARG;
      why = "n must be in [3, " + std::to_string(PARAISO_WAVE_MAX_CELLS) + "]";
    } else if (!(std::isfinite(p.c) && p.c >= 0.0) || !(std::isfinite(p.dx) && p.dx > 0.0) ||
               !(std::isfinite(p.dt) && p.dt >= 0.0)) {
      rc = PARAISO_ERR_INVALID_ARG;
      why = "c and dt must be finite and >= 0, dx finite and > 0";
    } else if (!p.f || !p.g || ((uintptr_t)p.f % 8) || ((uintptr_t)p.g % 8) ||
               ((uintptr_t)p.energy % 8)) {
      rc = PARAISO_ERR_INVALID_ARG;
      why = "f and g must be non-null, f, g and energy 8-byte aligned";
    }
    if (rc) {
      delete[] host;
      return wave_fail(rc, w + why);
    }
    WaveDev& d = host[m];
    d.n = (int)p.n;
    d.pad_ = 0;
    d.k = p.c * p.c * p.dt / (p.dx * p.dx);
    d.dt = p.dt;
    d.c2 = p.c * p.c;
    d.inv2dx = 1.0 / (2.0 * p.dx);
    d.half_dx = 0.5 * p.dx;
    d.f = p.f;
    d.g = p.g;
    d.energy = p.energy;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t e = hipMemcpyAsync(workspace, host, sizeof(WaveDev) * count, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host table is freed next
  delete[] host;
  if (e != hipSuccess) return wave_fail(PARAISO_ERR_HIP, std::string("table upload: ") + hipGetErrorString(e));
  return PARAISO_OK;
}

int32_t paraiso_wave_run(const void* workspace, int32_t count, int64_t steps, int64_t max_cells, void* hip_stream) {
  if (!workspace) return wave_fail(PARAISO_ERR_INVALID_ARG, "null workspace");
  if (count < 1) return wave_fail(PARAISO_ERR_INVALID_ARG, "count must be >= 1");
  if (steps < 0) return wave_fail(PARAISO_ERR_INVALID_ARG, "steps must be >= 0");
  if (max_cells < 3 || max_cells > PARAISO_WAVE_MAX_CELLS)
    return wave_fail(PARAISO_ERR_INVALID_ARG, "max_cells must be in [3, " + std::to_string(PARAISO_WAVE_MAX_CELLS) + "]");
  if ((uintptr_t)workspace % 256) return wave_fail(PARAISO_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  const WaveDev* table = (const WaveDev*)workspace;
  long long st = (long long)steps;
  void* args[] = {(void*)&table, (void*)&st};
  hipError_t e = hipLaunchKernel(wave_kernel(max_cells), dim3(count), dim3(kWaveThreads), args, 0,
                                 (hipStream_t)hip_stream);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return wave_fail(PARAISO_ERR_HIP, std::string("k_wave1d: ") + hipGetErrorString(e));
  return PARAISO_OK;
}

int32_t paraiso_wave_advance(const paraiso_wave* probs, int32_t count, int64_t steps, void* workspace,
                             size_t workspace_bytes, void* hip_stream) {
  if (steps < 0) return wave_fail(PARAISO_ERR_INVALID_ARG, "steps must be >= 0");
  int32_t rc = paraiso_wave_prepare(probs, count, workspace, workspace_bytes, hip_stream);
  if (rc) return rc;
  int64_t max_cells = 3;
  for (int m = 0; m < count; ++m) max_cells = probs[m].n > max_cells ? probs[m].n : max_cells;
  return paraiso_wave_run(workspace, count, steps, max_cells, hip_stream);
}

}  // extern "C"
