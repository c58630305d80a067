/* Drives every entry point of the FP64 oracle (oracle/euler_oracle.c) on
 * small meshes of every dimension, boundary and reconstruction order, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer (tests only).
 * Exits non-zero on a failed status or a non-finite result; the sanitizers
 * abort on any out-of-bounds access, leak or undefined operation. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
  int32_t kind, pad_;
  double angle, amplitude;
} orc_analytic;
typedef struct {
  int32_t ndim, order;
  int64_t n[3];
  double dx[3];
  double gamma;
  int32_t bc[3];
  int32_t pad2_;
} orc_mesh;

int orc_exact_state(const orc_mesh* m, const orc_analytic* an, double t, double* U);
int orc_step_t(const orc_mesh* m, const orc_analytic* an, double t, const double* U0, double dt, double* U2);
int orc_cfl_dt(const orc_mesh* m, const double* U, double cfl, double* dt_out);
int orc_totals(const orc_mesh* m, const double* U, double* out);
int orc_advance_t(const orc_mesh* m, const orc_analytic* an, double* U, double cfl, double t_end, int64_t max_steps,
                  double* t_out, int64_t* steps_out);
int orc_riemann_star(double gamma, const double* L, const double* R, double* ps, double* us);

static int check(const char* what, int rc) {
  if (rc) {
    fprintf(stderr, "%s: status %d\n", what, rc);
    exit(2);
  }
  return rc;
}

static void finite(const char* what, const double* a, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!isfinite(a[i])) {
      fprintf(stderr, "%s: non-finite at %lld\n", what, (long long)i);
      exit(3);
    }
}

int main(void) {
  const int64_t sizes[3][3] = {{13, 1, 1}, {9, 7, 1}, {6, 5, 4}};
  int cases = 0;
  for (int d = 1; d <= 3; ++d)
    for (int bc = 0; bc <= 2; ++bc)
      for (int order = 1; order <= 2; ++order)
        for (int kind = 1; kind <= 3; ++kind) {
          orc_mesh m = {0};
          m.ndim = d;
          m.order = order;
          m.gamma = 1.4;
          for (int a = 0; a < 3; ++a) {
            m.n[a] = sizes[d - 1][a];
            m.dx[a] = a < d ? 1.0 / (double)m.n[a] : 1.0;
            m.bc[a] = a < d ? bc : 0;
          }
          orc_analytic an = {kind, 0, d > 1 ? 1.0471975511965976 : 0.0, 1e-5};
          const int64_t cells = m.n[0] * m.n[1] * m.n[2];
          const int64_t total = (d + 2) * cells;
          double* U = malloc(sizeof(double) * total);
          double* V = malloc(sizeof(double) * total);
          double tot[5], dt, t;
          int64_t steps;
          check("exact_state", orc_exact_state(&m, &an, 0.03, U));
          finite("exact_state", U, total);
          check("cfl_dt", orc_cfl_dt(&m, U, 0.5, &dt));
          check("step_t", orc_step_t(&m, bc == 2 ? &an : NULL, 0.03, U, dt, V));
          finite("step_t", V, total);
          check("totals", orc_totals(&m, V, tot));
          finite("totals", tot, d + 2);
          t = 0.03;
          check("advance_t", orc_advance_t(&m, bc == 2 ? &an : NULL, U, 0.5, 0.06, 5, &t, &steps));
          finite("advance_t", U, total);
          free(U);
          free(V);
          ++cases;
        }
  const double L[3] = {1.0, 0.0, 1.0}, R[3] = {0.125, 0.0, 0.1};
  double ps, us;
  check("riemann_star", orc_riemann_star(1.4, L, R, &ps, &us));
  printf("ok %d cases, p* = %.6f\n", cases, ps);
  return 0;
}
