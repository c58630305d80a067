// Resident kernel for small 1D meshes (gfx950).
//
// One workgroup holds one whole mesh (up to kResidentCells cells, a few per
// thread in registers, primitives and face fluxes exchanged through LDS) and
// runs a whole advance in a single launch: each step forms the face fluxes
// of stage 1 and stage 2 (one flux per face), the CFL maximum of the new
// state as a block reduction in FP64, dt = cfl / max clamped to t_end, and
// t and the step count, until t_end or the step budget is reached.  A 1D
// shock tube of 1024 cells needs ~900 dependent steps; this removes the
// per-step launch and scheduling latency that otherwise dominates.
//
// Modes: explicit dt (one step with a.dt[m]) or device-dt advance.  The
// final state is written to buffer 1 - src, so the host counts one launch
// as one buffer flip; t and the step count go to ring slot (ring + 1) % 3.
#pragma once

#include "euler_common.h"

namespace paraiso {

// Workgroups of 512 or 1024 threads, each thread holding up to
// kResidentPerThread cells: a mesh of up to 2048 cells runs on 512 threads
// (Sod 1024 FP64: 4.61-4.65 ms to t = 0.2 against 4.94 ms on 1024 and
// 6.5 ms on 256, whose waves lack the latency cover), larger ones on 1024.
constexpr int kResidentThreads = 1024;  // the largest workgroup
constexpr int kResidentPerThread = 4;
constexpr int kResidentCells = kResidentThreads * kResidentPerThread;
constexpr int resident_threads_for(int64_t cells) { return cells <= 512 * kResidentPerThread ? 512 : 1024; }

// HLLC flux of face f (between cells f-1 and f) from the primitives in LDS.
template <typename T>
__device__ __forceinline__ void resident_face(const MeshDev& M, const Gas<T>& g, int n, const T* sV, int f,
                                              T* fl) {
  const int i0 = map_index(f - 2, n, M.bc[0]), i1 = map_index(f - 1, n, M.bc[0]);
  const int i2 = map_index(f, n, M.bc[0]), i3 = map_index(f + 1, n, M.bc[0]);
  T vl[3], vr[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const T* y = sV + q * n;
    face_states(y[i0], y[i1], y[i2], y[i3], vl[q], vr[q]);
  }
  hllc<T, 1, 0>(vl, vr, fl, g);
}

// Primitives of this thread's cells into LDS (the first phase of a stage).
template <typename T, int NT>
__device__ __forceinline__ void resident_prims(int n, const Gas<T>& g, const T (*uin)[3], T* sV) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int r = 0; r < kResidentPerThread; ++r) {
    const int i = tid + r * NT;
    if (i < n) {
      T v[3];
      prim_of_cons<T, 1>(uin[r], v, g);
#pragma unroll
      for (int q = 0; q < 3; ++q) sV[q * n + i] = v[q];
    }
  }
}

// The rest of a stage, after the barrier that publishes sV: faces f = 0..n
// (thread t takes t, t + NT, ...; a wave with a lane that holds two faces in
// one round evaluates both in one pass, two independent chains, so the
// (n + 1)-th face of a mesh of a multiple of NT cells does not cost a round
// of its own), one barrier, the update.  No
// barrier at the end: the next stage first writes sV, which every thread has
// finished reading at the barrier after the flux phase, and writes sF only
// after its own first barrier.
template <typename T, int NT>
__device__ __forceinline__ void resident_flux_update(const MeshDev& M, const Gas<T>& g, int n, T coef,
                                                     const T (*ubase)[3], T (*uout)[3], const T* sV, T* sF) {
  const int tid = threadIdx.x;
  for (int f0 = tid; f0 <= n; f0 += 2 * NT) {
    const int f1 = f0 + NT;
    T fa[3];
    if (__builtin_amdgcn_ballot_w64(f1 <= n)) {
      T fb[3];
      resident_face<T>(M, g, n, sV, f0, fa);
      resident_face<T>(M, g, n, sV, f1 <= n ? f1 : f0, fb);
      if (f1 <= n) {
#pragma unroll
        for (int q = 0; q < 3; ++q) sF[q * (n + 1) + f1] = fb[q];
      }
    } else {
      resident_face<T>(M, g, n, sV, f0, fa);
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) sF[q * (n + 1) + f0] = fa[q];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kResidentPerThread; ++r) {
    const int i = tid + r * NT;
    if (i < n) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const T* F = sF + q * (n + 1);
        uout[r][q] = ubase[r][q] + coef * (F[i] - F[i + 1]);
      }
    }
  }
}

template <typename T, int NT>
__global__ void __launch_bounds__(NT) k_resident1d(Args a, LdsGeom) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double s_red[NT / 64];
  const int m = blockIdx.x;
  const MeshDev& M = a.meshes[m];
  const int n = M.n[0];
  T* sV = reinterpret_cast<T*>(smem);  // [3][n]
  T* sF = sV + 3 * n;                   // [3][n + 1]
  const int tid = threadIdx.x;
  const Gas<T> g = gas_of<T>(M);
  const Fields<T, 1> U0 = fields<T, 1>(M.s[a.src]);
  const Fields<T, 1> Uout = fields<T, 1>(M.s[1 - a.src]);
  T u[kResidentPerThread][3], u1[kResidentPerThread][3];
#pragma unroll
  for (int r = 0; r < kResidentPerThread; ++r) {
    const int i = tid + r * NT;
#pragma unroll
    for (int q = 0; q < 3; ++q) u[r][q] = i < n ? U0.f[q][i] : T(1);
  }
  const bool explicit_dt = a.dt != nullptr;
  Ctl& c = a.ctl[m];
  double t = c.t[a.ring];
  long long steps = c.steps[a.ring];
  const long long steps0 = steps;
  double qmax = explicit_dt ? 0.0 : __longlong_as_double((long long)qbits_max(c, a.ring));
  const double t_end = explicit_dt ? 0.0 : a.prm->t_end;
  const long long max_steps = explicit_dt ? 1 : a.prm->max_steps;
  const double cfl = explicit_dt ? 0.0 : a.prm->cfl;
  // a non-physical input (flagged by the CFL reduction before the launch) is not stepped
  bool bad = !explicit_dt && c.flags[a.ring] != 0;
  // Each step opens with stage 1's primitives going to LDS; in an advance the
  // same phase reduces the CFL maximum of that state (from the second step
  // on: the first takes the reduction made before the launch), each wave
  // into s_red, so the barrier that publishes sV publishes the wave maxima
  // too, and every thread then folds them itself.  s_red is next written
  // three barriers later.  A non-physical cell counts as +inf.
  for (bool first = true;; first = false) {
    resident_prims<T, NT>(n, g, u, sV);
    const bool reduce = !explicit_dt && !first;
    if (reduce) {
      double q = 0.0;
      bool b = false;
#pragma unroll
      for (int r = 0; r < kResidentPerThread; ++r) {
        const int i = tid + r * NT;
        if (i < n) {
          cfl_fold(cfl_q<T, 1>(u[r], M.inv_dx, M.gamma), q, b);
        }
      }
      double v = b ? __builtin_huge_val() : q;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
      if ((tid & 63) == 0) s_red[tid >> 6] = v;
    }
    __syncthreads();
    if (reduce) {
      double v = s_red[0];
      for (int k = 1; k < NT / 64; ++k) v = fmax(v, s_red[k]);
      bad = !(v < __builtin_huge_val());
      qmax = v;
    }
    double dt;
    if (explicit_dt) {
      if (steps > steps0) break;
      dt = a.dt[m];
    } else {
      if (!(t < t_end) || steps >= max_steps || bad) break;
      dt = cfl / qmax;
      if (dt > t_end - t) dt = t_end - t;
    }
    const T c1 = (T)((0.5 * dt) * M.inv_dx[0]);
    const T c2 = (T)(dt * M.inv_dx[0]);
    resident_flux_update<T, NT>(M, g, n, c1, u, u1, sV, sF);
    resident_prims<T, NT>(n, g, u1, sV);
    __syncthreads();
    resident_flux_update<T, NT>(M, g, n, c2, u, u, sV, sF);
    t += dt;
    ++steps;
  }
#pragma unroll
  for (int r = 0; r < kResidentPerThread; ++r) {
    const int i = tid + r * NT;
    if (i < n) {
#pragma unroll
      for (int q = 0; q < 3; ++q) Uout.f[q][i] = u[r][q];
    }
  }
  if (m == 0 && tid < 16 && a.queue) a.queue[((a.ring + 2) % 3) * 16 + tid] = 0u;
  if (tid == 0) {
    const int nx = (a.ring + 1) % 3, nn = (a.ring + 2) % 3;
    c.t[nx] = t;
    c.steps[nx] = steps;
    c.flags[nx] = bad ? 1 : 0;
    c.flags[nn] = 0;
    if (!explicit_dt) {
      qbits_clear(c, nx);
      c.qbits[nx][0] = (unsigned long long)__double_as_longlong(qmax);
      qbits_clear(c, nn);
    }
  }
}

}  // namespace paraiso
