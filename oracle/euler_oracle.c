/*
 * FP64 CPU oracle for one explicit step of the ideal-gas Euler equations.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant with the
 * HIP path.
 *
 * What it follows (paper: "Tuning Experiments / The Target Program"):
 *   - primitive V = (rho, v_a, p), conserved U = (rho, m_a, E),
 *     m_a = rho v_a, E = p/(gamma-1) + rho v^2 / 2  (state-vector equations);
 *   - the conservation law dU/dt + d_a F_a = 0 with
 *     F_a = (rho v_a, v_a m_b + p delta_ab, v_a (E + p))  (flux equation;
 *     the sign printed in the paper is read as the usual one, which is the
 *     one its AddFlux update implements);
 *   - piecewise-linear reconstruction of every primitive, axis by axis, with
 *     the minbee (minmod) limiter (Interpolate equation); or, as the order-1
 *     branch of the paper's interpolation listing, piecewise constant: the
 *     face takes the values of the two cells beside it;
 *   - the HLLC approximate Riemann flux of Toro, Spruce and Speares (1994),
 *     which the paper cites but does not print: Davis wave-speed estimates
 *     and the conserved star state (reading stated in the design notes);
 *   - AddFlux: U_out = U_base + sum_a (dt/dr_a)(F_a[i-1/2] - F_a[i+1/2]),
 *     accumulated a = 0..d-1 and then added to U_base;
 *   - the two-stage midpoint time marching
 *       F0 = Flux(U0); U1 = AddFlux(dt/2, F0, U0);
 *       F1 = Flux(U1); U2 = AddFlux(dt,   F1, U0);
 *   - dt from the CFL condition (form not printed; read as
 *     dt = C / max_i sum_a (|v_a| + c)/dr_a, c = sqrt(gamma p / rho),
 *     evaluated once per step on U0) and the OM "Reduce Min" semantics for
 *     a global reduction.
 *
 * Structure is deliberately plain: every stage fills a ghost-padded copy of
 * the primitive field (2 ghost cells per side on every active axis; periodic
 * wrap, outflow copy of the edge cell, or the analytic solution of the
 * problem at the cell centre and the stage's time), then makes whole-array
 * passes: faces of axis 0, faces of axis 1, ..., then the update.
 *
 * Analytic boundaries follow the paper's convergence tests: on the unit
 * square the analytic solution is substituted outside the solved domain.
 * A stage reads its ghosts at the time its input state stands for: t for
 * stage 1 (U0) and t + dt/2 for stage 2 (U1, the midpoint state).
 *
 * Layout of a state array: (d+2) fields, each a contiguous block of
 * nx*ny*nz doubles with x fastest: U[f*N + (k*ny + j)*nx + i].
 * Field order: rho, m_0, ..., m_{d-1}, E.  Primitive order:
 * rho, v_0, ..., v_{d-1}, p.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Built with -fopenmp, the per-cell and per-face loops below run on all host
 * cores.  Every iteration writes its own cells or faces, the stage sums are
 * formed per cell in the same order as serially, and the CFL maximum does not
 * depend on the order of the fold: results are bitwise those of the serial
 * build (the totals stay serial: their compensated sum is order-dependent). */
#ifdef _OPENMP
#include <omp.h>
#define ORC_PARALLEL_CELLS _Pragma("omp parallel for collapse(3) schedule(static)")
#define ORC_PARALLEL_FLAT _Pragma("omp parallel for schedule(static)")
#define ORC_PARALLEL_MAX _Pragma("omp parallel for schedule(static) reduction(max: qmax) reduction(|: bad)")
#define ORC_ATOMIC_WRITE _Pragma("omp atomic write")
#else
#define ORC_PARALLEL_CELLS
#define ORC_PARALLEL_FLAT
#define ORC_PARALLEL_MAX
#define ORC_ATOMIC_WRITE
#endif

/* Threads the loops above use (1 in the serial build). */
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

#define ORC_OK 0
#define ORC_BAD_ARG (-1)
#define ORC_NONFINITE (-4)
#define ORC_NOMEM (-6)

#define ORC_PERIODIC 0
#define ORC_OUTFLOW 1
#define ORC_ANALYTIC 2

/* Problems of the convergence tests (paper: entropy wave, sound wave, Sod's
 * shock tube).  Each is a function of s = (x - 1/2) cos(th) + (y - 1/2)
 * sin(th) + 1/2, the coordinate along n = (cos th, sin th) ("coaxial": th =
 * 0; "oblique": the initial condition rotated about the centre of the unit
 * square by th), with the velocity along n. */
#define ORC_ENTROPY_WAVE 1
#define ORC_SOUND_WAVE 2
#define ORC_SHOCK_TUBE 3

typedef struct {
  int32_t kind;
  int32_t pad_;
  double angle;     /* th, radians */
  double amplitude; /* A of the sound wave */
} orc_analytic;

#define NGHOST 2

typedef struct {
  int32_t ndim;
  int32_t order; /* reconstruction: 2 piecewise linear with minbee (default), 1 piecewise constant */
  int64_t n[3];
  double dx[3];
  double gamma;
  int32_t bc[3];
  int32_t pad2_;
} orc_mesh;

static int check_mesh(const orc_mesh* m) {
  if (!m) return ORC_BAD_ARG;
  if (m->ndim < 1 || m->ndim > 3) return ORC_BAD_ARG;
  if (m->order != 1 && m->order != 2) return ORC_BAD_ARG;
  if (!(m->gamma > 1.0) || !isfinite(m->gamma)) return ORC_BAD_ARG;
  for (int a = 0; a < 3; ++a) {
    if (m->n[a] < 1) return ORC_BAD_ARG;
    if (a >= m->ndim) {
      if (m->n[a] != 1) return ORC_BAD_ARG;
      continue;
    }
    if (!(m->dx[a] > 0.0) || !isfinite(m->dx[a])) return ORC_BAD_ARG;
    if (m->bc[a] != ORC_PERIODIC && m->bc[a] != ORC_OUTFLOW && m->bc[a] != ORC_ANALYTIC) return ORC_BAD_ARG;
  }
  return ORC_OK;
}

static int64_t ncells(const orc_mesh* m) { return m->n[0] * m->n[1] * m->n[2]; }

/* ---------------------------------------------------------------------- */
/* Single-cell relations (state-vector equations).                         */
/* ---------------------------------------------------------------------- */

/* V(U): rho, v_a = m_a / rho, p = (gamma-1)(E - rho v^2 / 2). */
void orc_prim_of_cons(int ndim, double gamma, const double* u, double* v) {
  double rho = u[0];
  double ke = 0.0;
  v[0] = rho;
  for (int a = 0; a < ndim; ++a) {
    double va = u[1 + a] / rho;
    v[1 + a] = va;
    ke += va * u[1 + a];
  }
  v[ndim + 1] = (gamma - 1.0) * (u[ndim + 1] - 0.5 * ke);
}

/* U(V): rho, m_a = rho v_a, E = p/(gamma-1) + rho v^2 / 2. */
void orc_cons_of_prim(int ndim, double gamma, const double* v, double* u) {
  double rho = v[0];
  double v2 = 0.0;
  u[0] = rho;
  for (int a = 0; a < ndim; ++a) {
    u[1 + a] = rho * v[1 + a];
    v2 += v[1 + a] * v[1 + a];
  }
  u[ndim + 1] = v[ndim + 1] / (gamma - 1.0) + 0.5 * rho * v2;
}

/* Physical flux along axis `ax` from a primitive vector. */
static void phys_flux(int ndim, double gamma, int ax, const double* v, double* f) {
  double u[5];
  orc_cons_of_prim(ndim, gamma, v, u);
  double vn = v[1 + ax];
  double p = v[ndim + 1];
  f[0] = vn * u[0];
  for (int b = 0; b < ndim; ++b) f[1 + b] = vn * u[1 + b] + (b == ax ? p : 0.0);
  f[ndim + 1] = vn * (u[ndim + 1] + p);
}

/* ---------------------------------------------------------------------- */
/* Reconstruction (Interpolate equation, minbee limiter).                  */
/* ---------------------------------------------------------------------- */

/* Limited slope.  dy = 0 when the one-sided differences have opposite
 * signs (or either is zero); otherwise the one of smaller magnitude, and
 * dy12 on a tie.  The sign test compares signs instead of forming the
 * product, which is the same predicate in exact arithmetic. */
double orc_minmod(double dy01, double dy12) {
  int opposite = (dy01 > 0.0 && dy12 < 0.0) || (dy01 < 0.0 && dy12 > 0.0);
  if (opposite) return 0.0;
  if (dy01 == 0.0 || dy12 == 0.0) return 0.0;
  if (fabs(dy01) < fabs(dy12)) return dy01;
  return dy12;
}

/* Interpolate(y0, y1, y2) = (y1 - dy/2, y1 + dy/2): the values of the
 * cell-1 profile on its lower and upper faces. */
void orc_interpolate(double y0, double y1, double y2, double* lower, double* upper) {
  double dy = orc_minmod(y1 - y0, y2 - y1);
  *lower = y1 - 0.5 * dy;
  *upper = y1 + 0.5 * dy;
}

/* ---------------------------------------------------------------------- */
/* HLLC flux across a face normal to axis `ax` (Toro, Spruce, Speares).    */
/* vl: primitive state on the left of the face, vr: on the right.          */
/* ---------------------------------------------------------------------- */
void orc_hllc(int ndim, double gamma, int ax, const double* vl, const double* vr, double* f) {
  const int nf = ndim + 2;
  double rl = vl[0], rr = vr[0];
  double ul = vl[1 + ax], ur = vr[1 + ax];
  double pl = vl[ndim + 1], pr = vr[ndim + 1];
  double cl = sqrt(gamma * pl / rl);
  double cr = sqrt(gamma * pr / rr);

  /* Davis estimates of the slowest and fastest signal speeds. */
  double sl = fmin(ul - cl, ur - cr);
  double sr = fmax(ul + cl, ur + cr);

  /* Contact (middle-wave) speed from the jump conditions. */
  double sstar = (pr - pl + rl * ul * (sl - ul) - rr * ur * (sr - ur)) /
                 (rl * (sl - ul) - rr * (sr - ur));

  double fl[5], fr[5], uL[5], uR[5];
  phys_flux(ndim, gamma, ax, vl, fl);
  phys_flux(ndim, gamma, ax, vr, fr);
  orc_cons_of_prim(ndim, gamma, vl, uL);
  orc_cons_of_prim(ndim, gamma, vr, uR);

  if (0.0 <= sl) {
    for (int q = 0; q < nf; ++q) f[q] = fl[q];
    return;
  }
  if (sr <= 0.0) {
    for (int q = 0; q < nf; ++q) f[q] = fr[q];
    return;
  }
  /* Star state on the side the contact leaves behind. */
  const double* vk;
  const double* uk;
  const double* fk;
  double sk;
  if (0.0 <= sstar) {
    vk = vl; uk = uL; fk = fl; sk = sl;
  } else {
    vk = vr; uk = uR; fk = fr; sk = sr;
  }
  double rk = vk[0], uk_n = vk[1 + ax], pk = vk[ndim + 1];
  double fac = rk * (sk - uk_n) / (sk - sstar);
  double ustar[5];
  ustar[0] = fac;
  for (int b = 0; b < ndim; ++b) ustar[1 + b] = fac * (b == ax ? sstar : vk[1 + b]);
  ustar[ndim + 1] =
      fac * (uk[ndim + 1] / rk + (sstar - uk_n) * (sstar + pk / (rk * (sk - uk_n))));
  for (int q = 0; q < nf; ++q) f[q] = fk[q] + sk * (ustar[q] - uk[q]);
}

#ifndef ORC_COUNTING
/* ---------------------------------------------------------------------- */
/* Exact solutions of the convergence-test problems.                       */
/* ---------------------------------------------------------------------- */

/* Exact Riemann problem for the ideal gas (Toro, Riemann Solvers and
 * Numerical Methods for Fluid Dynamics, ch. 4).  States are (rho, u, p)
 * along the normal.  f_K(p) is the velocity change across the K wave: a
 * shock for p > p_K, a rarefaction otherwise; p* solves
 * f_L(p) + f_R(p) + u_R - u_L = 0 (Newton from the two-rarefaction guess),
 * u* = (u_L + u_R)/2 + (f_R(p*) - f_L(p*))/2. */
static double wave_fn(double p, const double* k, double gamma, double* dfdp) {
  const double rk = k[0], pk = k[2];
  const double ck = sqrt(gamma * pk / rk);
  if (p > pk) {
    const double a = 2.0 / ((gamma + 1.0) * rk), b = (gamma - 1.0) / (gamma + 1.0) * pk;
    const double q = sqrt(a / (p + b));
    *dfdp = q * (1.0 - 0.5 * (p - pk) / (p + b));
    return (p - pk) * q;
  }
  const double e = (gamma - 1.0) / (2.0 * gamma);
  const double r = pow(p / pk, e);
  *dfdp = r / (rk * ck * (p / pk));
  return 2.0 * ck / (gamma - 1.0) * (r - 1.0);
}

int orc_riemann_star(double gamma, const double* L, const double* R, double* ps, double* us) {
  const double cl = sqrt(gamma * L[2] / L[0]), cr = sqrt(gamma * R[2] / R[0]);
  const double e = (gamma - 1.0) / (2.0 * gamma);
  const double du = R[1] - L[1];
  if (2.0 * (cl + cr) / (gamma - 1.0) <= du) return ORC_BAD_ARG; /* vacuum forms */
  double p = pow((cl + cr - 0.5 * (gamma - 1.0) * du) / (cl / pow(L[2], e) + cr / pow(R[2], e)), 1.0 / e);
  for (int it = 0; it < 100; ++it) {
    double dl, dr;
    const double g = wave_fn(p, L, gamma, &dl) + wave_fn(p, R, gamma, &dr) + du;
    double pn = p - g / (dl + dr);
    if (pn < 1e-300) pn = 1e-300;
    const double change = fabs(pn - p) / (0.5 * (pn + p));
    p = pn;
    if (change < 1e-15) break;
  }
  double dl, dr;
  *ps = p;
  *us = 0.5 * (L[1] + R[1]) + 0.5 * (wave_fn(p, R, gamma, &dr) - wave_fn(p, L, gamma, &dl));
  return ORC_OK;
}

/* The solution at x/t = xi: the left state, the left fan, the left star
 * state, the right star state, the right fan or the right state. */
void orc_riemann_sample(double gamma, const double* L, const double* R, double ps, double us, double xi,
                        double* out) {
  const double g1 = (gamma - 1.0) / (gamma + 1.0);
  if (xi <= us) {
    const double rk = L[0], uk = L[1], pk = L[2], ck = sqrt(gamma * pk / rk);
    if (ps > pk) {
      const double sk = uk - ck * sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pk + (gamma - 1.0) / (2.0 * gamma));
      if (xi <= sk) {
        out[0] = rk; out[1] = uk; out[2] = pk;
      } else {
        out[0] = rk * (ps / pk + g1) / (g1 * ps / pk + 1.0); out[1] = us; out[2] = ps;
      }
    } else {
      const double head = uk - ck, cs = ck * pow(ps / pk, (gamma - 1.0) / (2.0 * gamma)), tail = us - cs;
      if (xi <= head) {
        out[0] = rk; out[1] = uk; out[2] = pk;
      } else if (xi > tail) {
        out[0] = rk * pow(ps / pk, 1.0 / gamma); out[1] = us; out[2] = ps;
      } else {
        const double c = 2.0 / (gamma + 1.0) * (ck + 0.5 * (gamma - 1.0) * (uk - xi));
        out[0] = rk * pow(c / ck, 2.0 / (gamma - 1.0));
        out[1] = 2.0 / (gamma + 1.0) * (ck + 0.5 * (gamma - 1.0) * uk + xi);
        out[2] = pk * pow(c / ck, 2.0 * gamma / (gamma - 1.0));
      }
    }
  } else {
    const double rk = R[0], uk = R[1], pk = R[2], ck = sqrt(gamma * pk / rk);
    if (ps > pk) {
      const double sk = uk + ck * sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pk + (gamma - 1.0) / (2.0 * gamma));
      if (xi >= sk) {
        out[0] = rk; out[1] = uk; out[2] = pk;
      } else {
        out[0] = rk * (ps / pk + g1) / (g1 * ps / pk + 1.0); out[1] = us; out[2] = ps;
      }
    } else {
      const double head = uk + ck, cs = ck * pow(ps / pk, (gamma - 1.0) / (2.0 * gamma)), tail = us + cs;
      if (xi >= head) {
        out[0] = rk; out[1] = uk; out[2] = pk;
      } else if (xi < tail) {
        out[0] = rk * pow(ps / pk, 1.0 / gamma); out[1] = us; out[2] = ps;
      } else {
        const double c = 2.0 / (gamma + 1.0) * (ck - 0.5 * (gamma - 1.0) * (uk - xi));
        out[0] = rk * pow(c / ck, 2.0 / (gamma - 1.0));
        out[1] = 2.0 / (gamma + 1.0) * (-ck + 0.5 * (gamma - 1.0) * uk + xi);
        out[2] = pk * pow(c / ck, 2.0 * gamma / (gamma - 1.0));
      }
    }
  }
}

/* Primitive state of problem `an` at point x (x[0..ndim-1]) and time t. */
int orc_exact_prims(const orc_mesh* m, const orc_analytic* an, const double* x, double t, double* v) {
  if (!m || !an) return ORC_BAD_ARG;
  const int d = m->ndim;
  const double gamma = m->gamma;
  const double cth = d > 1 ? cos(an->angle) : 1.0, sth = d > 1 ? sin(an->angle) : 0.0;
  if (d == 1 && an->angle != 0.0) return ORC_BAD_ARG;
  const double s = (x[0] - 0.5) * cth + (d > 1 ? (x[1] - 0.5) * sth : 0.0) + 0.5;
  double rho, vn, p;
  const double pi = 3.14159265358979323846;
  if (an->kind == ORC_ENTROPY_WAVE) {
    /* rho = 2 + sin(2 pi x), v = 1, p = 1: carried unchanged at speed 1 */
    rho = 2.0 + sin(2.0 * pi * (s - t));
    vn = 1.0;
    p = 1.0;
  } else if (an->kind == ORC_SOUND_WAVE) {
    /* rho = gamma (1 + A sin 2 pi x), v = A sin 2 pi x, p = 1 + gamma A sin 2 pi x:
     * a right-going acoustic wave on rho = gamma, p = 1 (sound speed 1),
     * exact to first order in A */
    const double w = an->amplitude * sin(2.0 * pi * (s - t));
    rho = gamma * (1.0 + w);
    vn = w;
    p = 1.0 + gamma * w;
  } else if (an->kind == ORC_SHOCK_TUBE) {
    const double L[3] = {1.0, 0.0, 1.0}, R[3] = {0.125, 0.0, 0.1};
    if (!(t > 0.0)) {
      const double* k = s < 0.5 ? L : R;
      rho = k[0]; vn = k[1]; p = k[2];
    } else {
      double ps, us, out[3];
      int rc = orc_riemann_star(gamma, L, R, &ps, &us);
      if (rc) return rc;
      orc_riemann_sample(gamma, L, R, ps, us, (s - 0.5) / t, out);
      rho = out[0]; vn = out[1]; p = out[2];
    }
  } else {
    return ORC_BAD_ARG;
  }
  v[0] = rho;
  v[1] = vn * cth;
  if (d > 1) v[2] = vn * sth;
  if (d > 2) v[3] = 0.0;
  v[d + 1] = p;
  return ORC_OK;
}

/* The conserved state of problem `an` at every cell centre at time t. */
int orc_exact_state(const orc_mesh* m, const orc_analytic* an, double t, double* U) {
  int rc = check_mesh(m);
  if (rc) return rc;
  const int d = m->ndim, nf = d + 2;
  const int64_t N = ncells(m);
  for (int64_t k = 0; k < m->n[2]; ++k)
    for (int64_t j = 0; j < m->n[1]; ++j)
      for (int64_t i = 0; i < m->n[0]; ++i) {
        const int64_t g[3] = {i, j, k};
        double x[3], v[5], u[5];
        for (int a = 0; a < d; ++a) x[a] = ((double)g[a] + 0.5) * m->dx[a];
        rc = orc_exact_prims(m, an, x, t, v);
        if (rc) return rc;
        orc_cons_of_prim(d, m->gamma, v, u);
        const int64_t c = (k * m->n[1] + j) * m->n[0] + i;
        for (int q = 0; q < nf; ++q) U[q * N + c] = u[q];
      }
  return ORC_OK;
}
#endif

/* ---------------------------------------------------------------------- */
/* Ghost-padded primitive field.                                           */
/* ---------------------------------------------------------------------- */

typedef struct {
  int ndim, nf;
  int64_t n[3];  /* interior extents */
  int64_t p[3];  /* padded extents (n + 2*NGHOST on active axes) */
  int64_t np;    /* padded cell count */
  double* v;     /* nf blocks of np doubles */
} padded;

static int64_t map_index(int64_t g, int64_t n, int bc) {
  /* g: interior index, may be in [-NGHOST, n + NGHOST). */
  if (bc == ORC_PERIODIC) {
    int64_t r = g % n;
    if (r < 0) r += n;
    return r;
  }
  if (g < 0) return 0;
  if (g >= n) return n - 1;
  return g;
}

static int pad_prims(const orc_mesh* m, const orc_analytic* an, double t, const double* U, padded* P) {
  const int d = m->ndim, nf = d + 2;
  const int64_t N = ncells(m);
  int analytic = 0;
  for (int a = 0; a < d; ++a) analytic |= (m->bc[a] == ORC_ANALYTIC);
#ifdef ORC_COUNTING
  if (analytic) return ORC_BAD_ARG;
#else
  if (analytic && !an) return ORC_BAD_ARG;
#endif
  P->ndim = d;
  P->nf = nf;
  for (int a = 0; a < 3; ++a) {
    P->n[a] = m->n[a];
    P->p[a] = (a < d) ? m->n[a] + 2 * NGHOST : 1;
  }
  P->np = P->p[0] * P->p[1] * P->p[2];
  P->v = (double*)malloc(sizeof(double) * (size_t)nf * (size_t)P->np);
  if (!P->v) return ORC_NOMEM;
  const int64_t off[3] = {d > 0 ? NGHOST : 0, d > 1 ? NGHOST : 0, d > 2 ? NGHOST : 0};
  int err = ORC_OK;
  ORC_PARALLEL_CELLS
  for (int64_t k = 0; k < P->p[2]; ++k)
    for (int64_t j = 0; j < P->p[1]; ++j)
      for (int64_t i = 0; i < P->p[0]; ++i) {
        const int64_t g[3] = {i - off[0], j - off[1], k - off[2]};
        int64_t dst = (k * P->p[1] + j) * P->p[0] + i;
        double v[5];
        int outside = 0;
        for (int a = 0; a < d; ++a)
          outside |= (m->bc[a] == ORC_ANALYTIC && (g[a] < 0 || g[a] >= m->n[a]));
#ifndef ORC_COUNTING
        if (outside) {
          /* analytic boundary: the solution at the ghost cell's centre */
          double x[3];
          for (int a = 0; a < d; ++a) x[a] = ((double)g[a] + 0.5) * m->dx[a];
          int rc = orc_exact_prims(m, an, x, t, v);
          if (rc) {
            ORC_ATOMIC_WRITE
            err = rc;
            continue;
          }
          for (int q = 0; q < nf; ++q) P->v[q * P->np + dst] = v[q];
          continue;
        }
#endif
        int64_t si = map_index(g[0], m->n[0], m->bc[0]);
        int64_t sj = (d > 1) ? map_index(g[1], m->n[1], m->bc[1]) : 0;
        int64_t sk = (d > 2) ? map_index(g[2], m->n[2], m->bc[2]) : 0;
        int64_t src = (sk * m->n[1] + sj) * m->n[0] + si;
        double u[5];
        for (int q = 0; q < nf; ++q) u[q] = U[q * N + src];
        orc_prim_of_cons(d, m->gamma, u, v);
        for (int q = 0; q < nf; ++q) P->v[q * P->np + dst] = v[q];
      }
  if (err) {
    free(P->v);
    return err;
  }
  return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* One stage: U_out = U_base + sum_a (cdt/dr_a)(F_a[i-1/2] - F_a[i+1/2]),   */
/* fluxes from U_in.                                                       */
/* ---------------------------------------------------------------------- */
int orc_stage_t(const orc_mesh* m, const orc_analytic* an, double t, const double* Uin,
                const double* Ubase, double cdt, double* Uout) {
  int rc = check_mesh(m);
  if (rc) return rc;
  if (!Uin || !Ubase || !Uout) return ORC_BAD_ARG;
  const int d = m->ndim, nf = d + 2;
  const int64_t N = ncells(m);
  padded P;
  rc = pad_prims(m, an, t, Uin, &P);
  if (rc) return rc;

  double* acc = (double*)calloc((size_t)nf * (size_t)N, sizeof(double));
  if (!acc) {
    free(P.v);
    return ORC_NOMEM;
  }
  const int64_t off[3] = {d > 0 ? NGHOST : 0, d > 1 ? NGHOST : 0, d > 2 ? NGHOST : 0};

  for (int ax = 0; ax < d; ++ax) {
    /* Faces of axis ax: index f in [0, n_ax] is the face between interior
     * cells f-1 and f, i.e. face (f - 1/2). */
    int64_t fe[3] = {m->n[0], m->n[1], m->n[2]};
    fe[ax] += 1;
    const int64_t nfaces = fe[0] * fe[1] * fe[2];
    double* F = (double*)malloc(sizeof(double) * (size_t)nf * (size_t)nfaces);
    if (!F) {
      free(acc);
      free(P.v);
      return ORC_NOMEM;
    }
    int64_t stride = 1;
    for (int b = 0; b < ax; ++b) stride *= P.p[b];
    ORC_PARALLEL_CELLS
    for (int64_t k = 0; k < fe[2]; ++k)
      for (int64_t j = 0; j < fe[1]; ++j)
        for (int64_t i = 0; i < fe[0]; ++i) {
          /* padded index of the cell on the right of the face */
          int64_t c = ((k + off[2]) * P.p[1] + (j + off[1])) * P.p[0] + (i + off[0]);
          double vl[5], vr[5];
          for (int q = 0; q < nf; ++q) {
            const double* y = P.v + q * P.np;
            if (m->order == 1) {
              /* piecewise constant: the two cells' own values */
              vl[q] = y[c - stride];
              vr[q] = y[c];
              continue;
            }
            double lo, hi;
            /* left cell (c - stride): its upper-face value */
            orc_interpolate(y[c - 2 * stride], y[c - stride], y[c], &lo, &hi);
            vl[q] = hi;
            /* right cell c: its lower-face value */
            orc_interpolate(y[c - stride], y[c], y[c + stride], &lo, &hi);
            vr[q] = lo;
          }
          double f[5];
          orc_hllc(d, m->gamma, ax, vl, vr, f);
          int64_t fi = (k * fe[1] + j) * fe[0] + i;
          for (int q = 0; q < nf; ++q) F[q * nfaces + fi] = f[q];
        }
    const double coef = cdt / m->dx[ax];
    int64_t fstride = 1;
    for (int b = 0; b < ax; ++b) fstride *= fe[b];
    ORC_PARALLEL_CELLS
    for (int64_t k = 0; k < m->n[2]; ++k)
      for (int64_t j = 0; j < m->n[1]; ++j)
        for (int64_t i = 0; i < m->n[0]; ++i) {
          int64_t cell = (k * m->n[1] + j) * m->n[0] + i;
          int64_t fm = (k * fe[1] + j) * fe[0] + i; /* face i - 1/2 along ax */
          int64_t fp = fm + fstride;                /* face i + 1/2 along ax */
          for (int q = 0; q < nf; ++q)
            acc[q * N + cell] += coef * (F[q * nfaces + fm] - F[q * nfaces + fp]);
        }
    free(F);
  }
  ORC_PARALLEL_FLAT
  for (int64_t e = 0; e < (int64_t)nf * N; ++e) Uout[e] = Ubase[e] + acc[e];
  free(acc);
  free(P.v);
  return ORC_OK;
}

int orc_stage(const orc_mesh* m, const double* Uin, const double* Ubase, double cdt, double* Uout) {
  return orc_stage_t(m, 0, 0.0, Uin, Ubase, cdt, Uout);
}

/* One midpoint Runge-Kutta step with a given dt from time t (t only
 * matters for analytic boundaries: stage 1 at t, stage 2 at t + dt/2). */
int orc_step_t(const orc_mesh* m, const orc_analytic* an, double t, const double* U0, double dt,
               double* U2) {
  int rc = check_mesh(m);
  if (rc) return rc;
  if (!(dt >= 0.0) || !isfinite(dt)) return ORC_BAD_ARG;
  const int64_t total = (int64_t)(m->ndim + 2) * ncells(m);
  double* U1 = (double*)malloc(sizeof(double) * (size_t)total);
  if (!U1) return ORC_NOMEM;
  rc = orc_stage_t(m, an, t, U0, U0, 0.5 * dt, U1);
  if (!rc) rc = orc_stage_t(m, an, t + 0.5 * dt, U1, U0, dt, U2);
  free(U1);
  return rc;
}

int orc_step(const orc_mesh* m, const double* U0, double dt, double* U2) {
  return orc_step_t(m, 0, 0.0, U0, dt, U2);
}

/* ---------------------------------------------------------------------- */
/* CFL time step: dt = C / max_i q_i, q_i = sum_a (|v_a| + c)/dr_a.         */
/* Returns ORC_NONFINITE if any cell has rho <= 0, p <= 0 or a non-finite  */
/* value.  The maximum is taken like the OM Reduce: start from cell 0 and  */
/* fold over the cells in storage order.                                   */
/* ---------------------------------------------------------------------- */
int orc_cfl_qmax(const orc_mesh* m, const double* U, double* qmax_out) {
  int rc = check_mesh(m);
  if (rc) return rc;
  const int d = m->ndim, nf = d + 2;
  const int64_t N = ncells(m);
  /* Every cell is checked; a bad cell anywhere makes the result NONFINITE.
   * The maximum of the positive terms does not depend on the fold order. */
  double qmax = 0.0;
  int bad = 0;
  ORC_PARALLEL_MAX
  for (int64_t c = 0; c < N; ++c) {
    double u[5], v[5];
    for (int q = 0; q < nf; ++q) u[q] = U[q * N + c];
    orc_prim_of_cons(d, m->gamma, u, v);
    double rho = v[0], p = v[d + 1];
    if (!(rho > 0.0) || !(p > 0.0) || !isfinite(rho) || !isfinite(p) ||
        !isfinite(u[d + 1])) {
      bad = 1;
      continue;
    }
    double cs = sqrt(m->gamma * p / rho);
    double q = 0.0;
    for (int a = 0; a < d; ++a) {
      if (!isfinite(v[1 + a])) bad = 1;
      q += (fabs(v[1 + a]) + cs) / m->dx[a];
    }
    qmax = fmax(qmax, q);
  }
  if (bad) return ORC_NONFINITE;
  *qmax_out = qmax;
  return ORC_OK;
}

int orc_cfl_dt(const orc_mesh* m, const double* U, double cfl, double* dt_out) {
  if (!(cfl > 0.0 && cfl <= 1.0)) return ORC_BAD_ARG;
  double qmax;
  int rc = orc_cfl_qmax(m, U, &qmax);
  if (rc) return rc;
  *dt_out = cfl / qmax;
  return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* Conserved totals: sum over cells of each field times the cell volume,   */
/* with Neumaier-compensated summation in storage order.                   */
/* ---------------------------------------------------------------------- */
int orc_totals(const orc_mesh* m, const double* U, double* out) {
  int rc = check_mesh(m);
  if (rc) return rc;
  const int d = m->ndim, nf = d + 2;
  const int64_t N = ncells(m);
  double vol = 1.0;
  for (int a = 0; a < d; ++a) vol *= m->dx[a];
  for (int q = 0; q < nf; ++q) {
    double s = 0.0, comp = 0.0;
    for (int64_t c = 0; c < N; ++c) {
      double x = U[q * N + c];
      double t = s + x;
      if (fabs(s) >= fabs(x))
        comp += (s - t) + x;
      else
        comp += (x - t) + s;
      s = t;
    }
    out[q] = (s + comp) * vol;
  }
  return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* Advance to t_end with the CFL step clamped to the remaining time.       */
/* ---------------------------------------------------------------------- */
int orc_advance_t(const orc_mesh* m, const orc_analytic* an, double* U, double cfl, double t_end,
                  int64_t max_steps, double* t_inout, int64_t* steps_out) {
  int rc = check_mesh(m);
  if (rc) return rc;
  const int64_t total = (int64_t)(m->ndim + 2) * ncells(m);
  double* W = (double*)malloc(sizeof(double) * (size_t)total);
  if (!W) return ORC_NOMEM;
  double t = *t_inout;
  int64_t steps = 0;
  while (t < t_end && steps < max_steps) {
    double dt;
    rc = orc_cfl_dt(m, U, cfl, &dt);
    if (rc) break;
    if (dt > t_end - t) dt = t_end - t;
    rc = orc_step_t(m, an, t, U, dt, W);
    if (rc) break;
    memcpy(U, W, sizeof(double) * (size_t)total);
    t += dt;
    ++steps;
  }
  free(W);
  *t_inout = t;
  *steps_out = steps;
  return rc;
}

int orc_advance(const orc_mesh* m, double* U, double cfl, double t_end, int64_t max_steps,
                double* t_inout, int64_t* steps_out) {
  return orc_advance_t(m, 0, U, cfl, t_end, max_steps, t_inout, steps_out);
}
