/*
 * A C program that uses the library through include/paraiso.h alone (no
 * Python): device buffers from hipMalloc, a 256 x 192 periodic shear layer
 * in FP64, ten device-dt steps of paraiso_advance, FP64 totals before and
 * after.  Usage: c_abi_consumer OUT.bin -- writes the final state (4 fields
 * of nx * ny doubles, x fastest) to OUT.bin and prints
 *   steps t mass0 mx0 my0 E0 mass1 mx1 my1 E1
 * on one line.  Exit status 0 on success, 1 with a message on any error.
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "paraiso.h"

#define CHECK_HIP(x)                                                   \
  do {                                                                 \
    hipError_t e_ = (x);                                               \
    if (e_ != hipSuccess) {                                            \
      fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));          \
      return 1;                                                        \
    }                                                                  \
  } while (0)
#define CHECK_P(x)                                                     \
  do {                                                                 \
    int32_t r_ = (x);                                                  \
    if (r_ != PARAISO_OK) {                                            \
      fprintf(stderr, "%s: %d %s\n", #x, r_, paraiso_last_error());    \
      return 1;                                                        \
    }                                                                  \
  } while (0)

int main(int argc, char** argv) {
  if (argc != 2) {
    fprintf(stderr, "usage: %s OUT.bin\n", argv[0]);
    return 1;
  }
  const int nx = 256, ny = 192;
  const size_t n = (size_t)nx * ny;
  const double gamma = 1.4;
  double* h = (double*)malloc(4 * n * sizeof(double));
  if (!h) return 1;
  /* rho = 2, v_x = 0.5 in the middle band, rho = 1, v_x = -0.5 outside;
   * v_y a rational ripple (exact in every arithmetic); p = 2.5 */
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const size_t k = (size_t)j * nx + i;
      const double y = (j + 0.5) / ny;
      const int mid = y >= 0.25 && y < 0.75;
      const double rho = mid ? 2.0 : 1.0, vx = mid ? 0.5 : -0.5;
      const double vy = 0.01 * ((i % 7) - 3) / 3.0, p = 2.5;
      h[k] = rho;
      h[n + k] = rho * vx;
      h[2 * n + k] = rho * vy;
      h[3 * n + k] = p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy);
    }
  void* d[2];
  CHECK_HIP(hipMalloc(&d[0], 4 * n * sizeof(double)));
  CHECK_HIP(hipMalloc(&d[1], 4 * n * sizeof(double)));
  CHECK_HIP(hipMemcpy(d[0], h, 4 * n * sizeof(double), hipMemcpyHostToDevice));

  paraiso_mesh m = {0};
  m.ndim = 2;
  m.dtype = PARAISO_F64;
  m.n[0] = nx;
  m.n[1] = ny;
  m.n[2] = 1;
  m.dx[0] = 1.0 / nx;
  m.dx[1] = 1.0 / ny;
  m.dx[2] = 1.0;
  m.gamma = gamma;
  m.bc[0] = m.bc[1] = m.bc[2] = PARAISO_PERIODIC;
  for (int b = 0; b < 2; ++b)
    for (int q = 0; q < 4; ++q) m.state[b][q] = (char*)d[b] + q * n * sizeof(double);

  size_t ws = 0;
  CHECK_P(paraiso_workspace_bytes(&m, 1, &ws));
  void* w = NULL;
  CHECK_HIP(hipMalloc(&w, ws > 0 ? ws : 256));
  paraiso_ctx* ctx = NULL;
  CHECK_P(paraiso_init(&m, 1, w, ws, NULL, &ctx));

  double tot0[4], tot1[4], t = 0.0;
  int64_t steps = 0;
  CHECK_P(paraiso_totals(ctx, tot0));
  CHECK_P(paraiso_advance(ctx, 1.0, 0.5, 10, &t, &steps));
  CHECK_P(paraiso_totals(ctx, tot1));
  int32_t cur = 0;
  CHECK_P(paraiso_current(ctx, &cur));
  CHECK_HIP(hipMemcpy(h, d[cur], 4 * n * sizeof(double), hipMemcpyDeviceToHost));
  FILE* f = fopen(argv[1], "wb");
  if (!f || fwrite(h, sizeof(double), 4 * n, f) != 4 * n) {
    fprintf(stderr, "cannot write %s\n", argv[1]);
    return 1;
  }
  fclose(f);
  printf("%lld %.17g %.17g %.17g %.17g %.17g %.17g %.17g %.17g %.17g\n", (long long)steps, t, tot0[0], tot0[1],
         tot0[2], tot0[3], tot1[0], tot1[1], tot1[2], tot1[3]);
  CHECK_P(paraiso_destroy(ctx));
  CHECK_HIP(hipFree(w));
  CHECK_HIP(hipFree(d[0]));
  CHECK_HIP(hipFree(d[1]));
  free(h);
  return 0;
}
