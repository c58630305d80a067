// Device-side numerics of the Euler step for gfx950.
//
// Scheme (paper, "Tuning Experiments / The Target Program"): conserved
// U = (rho, m_a, E), primitive V = (rho, v_a, p), minbee piecewise-linear
// reconstruction of V along each axis, HLLC face fluxes (Toro-Spruce-Speares,
// cited there), AddFlux with the usual sign of the conservation law, and the
// two-stage midpoint Runge-Kutta marching.  dt comes from the CFL condition
// as a global max-reduction of sum_a (|v_a| + c)/dx_a in FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace paraiso {

constexpr int kMaxFields = 5;
constexpr int kPeriodic = 0;
constexpr int kOutflow = 1;
constexpr int kAnalytic = 2;  // ghosts from an exact solution (see Analytic)

// ---------------------------------------------------------------------------
// integer helpers
// ---------------------------------------------------------------------------

// Division by a run-time invariant d via a 32x32->hi multiply:
// q = umulhi(n, floor((2^32-1)/d) + 1) is exact whenever n * d < 2^32
// (Granlund-Montgomery, round-up variant).  d == 1 is handled by a mask.
struct FastDiv {
  uint32_t m;
  uint32_t mask;
  __host__ __device__ static FastDiv make(uint32_t d) {
    FastDiv f;
    if (d <= 1u) {
      f.m = 0u;
      f.mask = 0xFFFFFFFFu;
    } else {
      f.m = 0xFFFFFFFFu / d + 1u;
      f.mask = 0u;
    }
    return f;
  }
  __device__ __forceinline__ uint32_t div(uint32_t n) const { return __umulhi(n, m) + (n & mask); }
};

// A box of cells in tile-local coordinates, x fastest.
struct Box {
  int e[3];
  int count;
  FastDiv d0;   // / e[0]
  FastDiv d01;  // / (e[0]*e[1])
  __device__ __forceinline__ void coords(int l, int& i, int& j, int& k) const {
    uint32_t kk = d01.div((uint32_t)l);
    uint32_t rem = (uint32_t)l - kk * (uint32_t)(e[0] * e[1]);
    uint32_t jj = d0.div(rem);
    i = (int)(rem - jj * (uint32_t)e[0]);
    j = (int)jj;
    k = (int)kk;
  }
};

// A box built on the device (two integer divisions, once per call).
__device__ __forceinline__ Box make_box_dev(int e0, int e1, int e2) {
  Box b;
  b.e[0] = e0;
  b.e[1] = e1;
  b.e[2] = e2;
  b.count = e0 * e1 * e2;
  b.d0 = FastDiv::make((uint32_t)e0);
  b.d01 = FastDiv::make((uint32_t)(e0 * e1));
  return b;
}

// Map any cell index onto [0, n) along one axis: clamp (outflow) or wrap
// (periodic).  One add or subtract covers -n <= p < 2n; anything further out
// (tiles wider than the mesh) takes the remainder.
__device__ __forceinline__ int map_index(int p, int n, int bc) {
  if (bc == kOutflow) return p < 0 ? 0 : (p >= n ? n - 1 : p);
  p += (p < 0) ? n : 0;
  p -= (p >= n) ? n : 0;
  if ((unsigned)p >= (unsigned)n) {
    const int r = p % n;
    p = r < 0 ? r + n : r;
  }
  return p;
}

// ---------------------------------------------------------------------------
// floating-point helpers
// ---------------------------------------------------------------------------
template <typename T>
struct Fp;

template <>
struct Fp<float> {
  // hardware reciprocal and square root (1 ulp); the FP32 path is held to a
  // relative error budget, not to correct rounding
  static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
  static __device__ __forceinline__ float div(float a, float b) { return a * rcp(b); }
  // sqrt(a / b) for a, b > 0 with a single transcendental: a * rsqrt(a b)
  static __device__ __forceinline__ float sqrt_ratio(float a, float b) { return a * __builtin_amdgcn_rsqf(a * b); }
  // median of (a, b, 0): zero unless a and b share a sign, else the smaller magnitude
  static __device__ __forceinline__ float med0(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, 0.0f); }
};

template <>
struct Fp<double> {
  // The hardware seeds (v_rcp_f64, v_rsq_f64) refined by one third-order
  // step each, which cubes the relative error e of the seed: with
  // r = (1/x)(1 - e), 1 - x r = e and r (1 + e + e^2) = (1/x)(1 - e^3); with
  // y = x^-1/2 (1 - e), d = 1 - x y^2 and y (1 + d/2 + 3 d^2 / 8) =
  // x^-1/2 (1 - 5/2 e^3 + O(e^4)) (the series of (1 - d)^-1/2 to second
  // order).  From seeds good to about 2^-22 that leaves a result within a
  // few ulp, in fewer and shorter-chained operations than two Newton-Raphson
  // steps.  The FP64 path is held to a relative error budget of 1e-12 per
  // step, not to correct rounding.  Arguments are positive normal numbers on
  // physical states; anything else yields a non-finite value, which the CFL
  // check reports.
  static __device__ __forceinline__ double rcp(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, r, 1.0);
    return fma(r, fma(e, e, e), r);
  }
  static __device__ __forceinline__ double rsqrt(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double d = fma(-x * y, y, 1.0);
    return fma(y, d * fma(d, 0.375, 0.5), y);
  }
  static __device__ __forceinline__ double div(double a, double b) { return a * rcp(b); }
  // sqrt(a / b) for a, b > 0: a * rsqrt(a b)
  static __device__ __forceinline__ double sqrt_ratio(double a, double b) { return a * rsqrt(a * b); }
  static __device__ __forceinline__ double med0(double a, double b) {
    return fmax(fmin(a, b), fmin(fmax(a, b), 0.0));
  }
};

// Constants of the gas, each computed in FP64 on the host and rounded once.
template <typename T>
struct Gas {
  T gamma;
  T gm1;      // gamma - 1
  T inv_gm1;  // 1 / (gamma - 1)
};

// Limited slope of the Interpolate equation: 0 when the one-sided
// differences differ in sign (or one is zero), otherwise the one of smaller
// magnitude.  That is exactly the median of (a, b, 0), one v_med3_f32 in FP32:
// no product is formed, so FP32 underflow cannot zero a valid slope, and a
// tie returns a value equal to either difference.
template <typename T>
__device__ __forceinline__ T minmod(T a, T b) {
  return Fp<T>::med0(a, b);
}

// V(U): rho, v_a = m_a / rho, p = (gamma-1)(E - rho v^2/2).
template <typename T, int D>
__device__ __forceinline__ void prim_of_cons(const T* u, T* v, const Gas<T>& g) {
  const T rho = u[0];
  const T ir = Fp<T>::rcp(rho);
  T ke = T(0);
  v[0] = rho;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const T va = u[1 + a] * ir;
    v[1 + a] = va;
    ke += va * u[1 + a];
  }
  v[D + 1] = g.gm1 * (u[D + 1] - T(0.5) * ke);
}

// Reconstructed face states at the face between cells y1 and y2 of the
// four-cell stencil y0 y1 | y2 y3 along the face normal.
template <typename T>
__device__ __forceinline__ void face_states(T y0, T y1, T y2, T y3, T& left, T& right) {
  const T d12 = y2 - y1;
  left = y1 + T(0.5) * minmod(y1 - y0, d12);
  right = y2 - T(0.5) * minmod(d12, y3 - y2);
}

// HLLC flux across a face normal to axis AX.  vl / vr: primitive states on
// the left / right of the face; f: conserved-ordered flux.
//   c_K = sqrt(gamma p_K / rho_K); S_L = min(u_L - c_L, u_R - c_R),
//   S_R = max(u_L + c_L, u_R + c_R) (Davis);
//   S* = (p_R - p_L + rho_L u_L (S_L - u_L) - rho_R u_R (S_R - u_R))
//        / (rho_L (S_L - u_L) - rho_R (S_R - u_R));
//   F = F_L if 0 <= S_L; F_R if S_R <= 0; else F_K + S_K (U*_K - U_K) with
//   K = L if 0 <= S*, else R, and
//   U*_K = rho_K (S_K - u_K)/(S_K - S*) (1, S*, v_t, E_K/rho_K
//          + (S* - u_K)(S* + p_K / (rho_K (S_K - u_K)))).
// The side is selected first so that one physical flux and one star state
// are evaluated; E*_K is formed as
//   [(S_K - u_K) E_K + (S* - u_K)(rho_K (S_K - u_K) S* + p_K)] / (S_K - S*).
template <typename T, int D, int AX>
__device__ __forceinline__ void hllc(const T* vl, const T* vr, T* f, const Gas<T>& g) {
  const T rl = vl[0], rr = vr[0];
  const T ul = vl[1 + AX], ur = vr[1 + AX];
  const T pl = vl[D + 1], pr = vr[D + 1];
  const T cl = Fp<T>::sqrt_ratio(g.gamma * pl, rl);
  const T cr = Fp<T>::sqrt_ratio(g.gamma * pr, rr);
  const T sl = fmin(ul - cl, ur - cr);
  const T sr = fmax(ul + cl, ur + cr);
  const T al = rl * (sl - ul);
  const T ar = rr * (sr - ur);
  // S* = num / den with den = al - ar < 0 for positive densities and sound
  // speeds, so 0 <= S* exactly when num <= 0
  const T num = pr - pl + al * ul - ar * ur;
  const T den = al - ar;

  const bool left_sup = (T(0) <= sl);
  const bool right_sup = (sr <= T(0));
  const bool use_l = left_sup || (!right_sup && (num <= T(0)));

  T vk[D + 2];
#pragma unroll
  for (int q = 0; q < D + 2; ++q) vk[q] = use_l ? vl[q] : vr[q];
  const T sk = use_l ? sl : sr;
  const T ak = use_l ? al : ar;
  const T rk = vk[0], uk = vk[1 + AX], pk = vk[D + 1];

  T v2 = T(0);
#pragma unroll
  for (int b = 0; b < D; ++b) v2 += vk[1 + b] * vk[1 + b];
  const T ek = pk * g.inv_gm1 + T(0.5) * rk * v2;

  // one reciprocal gives both S* = num/den and 1/(S_K - S*) = den/(S_K den - num).
  // The weight of the star correction is zero on supersonic faces; e = 1
  // there keeps the (unused) star terms finite, so 0 * (U*_K - U_K) is 0.
  const bool sup = left_sup || right_sup;
  const T e = sup ? T(1) : sk * den - num;
  const T r = Fp<T>::rcp(den * e);
  const T w = sup ? T(0) : sk;
  const T sstar = num * e * r;
  const T inv = den * den * r;
  const T rstar = ak * inv;
  const T estar = inv * ((sk - uk) * ek + (sstar - uk) * (ak * sstar + pk));

  // F_K + w (U*_K - U_K).  Every transverse component is v_t times the mass
  // component: rho u v_t + w (chi v_t - rho v_t) = v_t (rho u + w (chi - rho)).
  const T mk = rk * uk;
  f[0] = mk + w * (rstar - rk);
#pragma unroll
  for (int b = 0; b < D; ++b) {
    if (b == AX)
      f[1 + b] = mk * uk + pk + w * (rstar * sstar - mk);
    else
      f[1 + b] = vk[1 + b] * f[0];
  }
  f[D + 1] = uk * (ek + pk) + w * (estar - ek);
}

// CFL quantity sum_a (|v_a| + c)/dx_a of one cell, in FP64.  Evaluated as
// (sum_a (|m_a| + rho c)/dx_a) / rho with (rho c)^2 = gamma rho p and
// rho p = (gamma - 1)(rho E - |m|^2/2), so the reciprocal of rho and the
// reciprocal square root of gamma rho p are independent chains.  The result
// is positive and finite exactly when the state is physical (rho > 0,
// p > 0, every component finite): p <= 0, a NaN or an infinite component,
// or rho = 0 make gamma rho p zero, negative, infinite or NaN, and q NaN on
// its way through the reciprocal square root (0 * inf, inf * 0, or the root
// of a negative number); rho < 0 with gamma rho p > 0 leaves q < 0; a
// subnormal rho, whose reciprocal overflows, makes the refined reciprocal
// NaN.  So the one class test of cfl_fold flags every non-physical cell.
template <typename T, int D>
__device__ __forceinline__ double cfl_q(const T* u, const double* inv_dx, double gamma) {
  double ud[D + 2];
#pragma unroll
  for (int q = 0; q < D + 2; ++q) ud[q] = (double)u[q];
  const double rho = ud[0];
  const double ir = Fp<double>::rcp(rho);
  double m2 = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) m2 = fma(ud[1 + a], ud[1 + a], m2);
  const double grp = gamma * (gamma - 1.0) * fma(rho, ud[D + 1], -0.5 * m2);  // gamma rho p
  const double rc = grp * Fp<double>::rsqrt(grp);                            // rho c
  double q = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) q = fma(fabs(ud[1 + a]) + rc, inv_dx[a], q);
  return q * ir;
}

// Floating-point class mask of everything but a positive finite number:
// signalling and quiet NaN, -inf, negative normal and subnormal, -0, +0, +inf.
constexpr int kNotPositiveFinite = 0x27F;

// Fold one cell's CFL quantity into a lane's running maximum and its
// non-physical flag: one class test and one maximum, which passes over NaN
// and never prefers a non-positive value to a positive one.
__device__ __forceinline__ void cfl_fold(double q, double& qmax, bool& bad) {
  bad |= __builtin_amdgcn_class(q, kNotPositiveFinite);
  qmax = fmax(qmax, q);
}

// The same for a wave whose lanes all evaluate q together, outside any
// branch on which cells count (`valid`: a mask of those lanes): the flag is
// a mask of lanes held in scalar registers, and the maximum runs on every
// lane, so the caller drops the lanes outside `valid` when it commits.  The
// one-stage 3D march runs faster this way (about 1% at 512^3); the 2D and
// fused 3D marches run faster with cfl_fold inside their store branches.
__device__ __forceinline__ void cfl_fold_wave(double q, unsigned long long valid, double& qmax,
                                              unsigned long long& bad) {
  bad |= __builtin_amdgcn_ballot_w64(__builtin_amdgcn_class(q, kNotPositiveFinite)) & valid;
  qmax = fmax(qmax, q);
}

}  // namespace paraiso
