// Exact solutions of the convergence-test problems (analytic boundaries).
#pragma once

#include "euler_common.h"

namespace paraiso {

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

// Exact ghost cells of the 2D analytic meshes for one step: stage 1 at the
// step's time t, stage 2 at t + dt/2 (the times the stages' inputs stand
// for), as conserved values rounded once to T.  Grid: meshes along x, the
// ghost cells of a mesh spread over the blocks along y.
template <typename T>
__global__ void __launch_bounds__(256) k_analytic_ghosts(Args a) {
  const int m = blockIdx.x;
  const MeshDev& M = a.meshes[m];
  if (!M.ghost || M.an.kind == 0) return;
  bool active;
  const double dt = step_dt(a, m, active);
  if (!active) return;
  const double t0 = a.ctl[m].t[a.ring];
  const int nx = M.n[0], ny = M.n[1];
  const int S = ghost_stride(nx, ny);
  T* gh = reinterpret_cast<T*>(M.ghost);
  for (int l = blockIdx.y * blockDim.x + threadIdx.x; l < 2 * S; l += gridDim.y * blockDim.x) {
    const int st = l / S, idx = l - st * S;
    int c, r;
    if (idx < 4 * (ny + 4)) {
      const int j = idx / (ny + 4);
      r = idx - j * (ny + 4) - 2;
      c = j < 2 ? j - 2 : nx + j - 2;
    } else {
      const int i2 = idx - 4 * (ny + 4);
      const int j = i2 / (nx + 4);
      c = i2 - j * (nx + 4) - 2;
      r = j < 2 ? j - 2 : ny + j - 2;
    }
    double v[4];
    exact_prims<double, 2>(M, (c + 0.5) * M.dx[0], (r + 0.5) * M.dx[1], st == 0 ? t0 : t0 + 0.5 * dt, v);
    const double ke = v[1] * v[1] + v[2] * v[2];
    T* out = gh + (size_t)st * 4 * S + idx;
    out[0] = (T)v[0];
    out[S] = (T)(v[0] * v[1]);
    out[2 * S] = (T)(v[0] * v[2]);
    out[3 * S] = (T)(v[3] * M.inv_gm1 + 0.5 * v[0] * ke);
  }
}

}  // namespace paraiso
