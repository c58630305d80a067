/*
 * paraiso.h — C ABI of the MI355X (gfx950) explicit Euler-step library.
 *
 * The library advances the ideal-gas Euler equations on uniform 1D/2D/3D
 * meshes with the scheme of Paraiso (arXiv:1204.4779, section "Tuning
 * Experiments / The Target Program"):
 *   - primitive V = (rho, v_a, p) and conserved U = (rho, m_a, E) with
 *     m_a = rho v_a and E = p/(gamma-1) + rho v^2/2 (state-vector equations);
 *   - minbee (minmod) piecewise-linear reconstruction of V along each axis
 *     (Interpolate equation);
 *   - HLLC face fluxes (Toro, Spruce, Speares 1994, as cited there);
 *   - AddFlux U_out = U_base + sum_a (dt/dr_a)(F_a[i-1/2] - F_a[i+1/2]);
 *   - the two-stage midpoint time marching
 *       U1 = AddFlux(dt/2, Flux(U0), U0),  U2 = AddFlux(dt, Flux(U1), U0);
 *   - dt from the CFL condition, dt = C / max_i sum_a (|v_a| + c)/dr_a with
 *     c = sqrt(gamma p / rho), taken as a global min-reduction over cells
 *     (the Orthotope Machine's Reduce Min).
 *
 * Memory ownership: the caller allocates every device buffer (state fields
 * and the workspace), keeps them alive for the lifetime of the context, and
 * frees them after paraiso_destroy.  The library never allocates or frees
 * device memory.  It never aborts: every entry point returns a status code
 * and, on failure, leaves a message for paraiso_last_error().  A HIP call of
 * the library that fails is reported as PARAISO_ERR_HIP and taken off HIP's
 * per-thread error record (hipGetLastError), so the caller's next HIP call
 * does not report it again.
 *
 * Streams: a context is bound to the HIP stream given at init and is not
 * thread-safe; calls on one context must come from one thread at a time.
 * Asynchronous calls (paraiso_step) return after enqueueing work on that
 * stream.  Synchronous calls (cfl_dt, advance, totals) return after the
 * work they enqueued has finished.
 *
 * Layout of a state buffer: d+2 separate device arrays (rho, m_0..m_{d-1},
 * E), each holding n[0]*n[1]*n[2] reals in x-fastest order:
 * field[(k*n[1] + j)*n[0] + i].  Element type float (PARAISO_F32) or double
 * (PARAISO_F64); arrays must be 16-byte aligned.
 */
#ifndef PARAISO_H
#define PARAISO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define PARAISO_OK 0
#define PARAISO_ERR_INVALID_ARG (-1)     /* a pointer, size or value is outside its documented range */
#define PARAISO_ERR_UNSUPPORTED (-2)     /* valid request that this build cannot run (variant, size) */
#define PARAISO_ERR_HIP (-3)             /* a HIP runtime call failed; message holds the HIP error */
#define PARAISO_ERR_NONFINITE (-4)       /* a cell has rho <= 0, p <= 0 or a non-finite value */
#define PARAISO_ERR_WORKSPACE (-5)       /* workspace smaller than paraiso_workspace_bytes reports */

/* boundary conditions per axis */
#define PARAISO_PERIODIC 0               /* wrap-around */
#define PARAISO_OUTFLOW 1                /* zero-gradient: ghost cells copy the edge cell's U */
#define PARAISO_ANALYTIC 2               /* ghost cells hold an exact solution (paraiso_set_analytic) */

/* exact solutions for PARAISO_ANALYTIC boundaries (paraiso_analytic.kind) */
#define PARAISO_ENTROPY_WAVE 1
#define PARAISO_SOUND_WAVE 2
#define PARAISO_SHOCK_TUBE 3

/* element types */
#define PARAISO_F32 0
#define PARAISO_F64 1

/*
 * One mesh.  n[a] >= 1 cells along axis a (n[a] == 1 for a >= ndim),
 * dx[a] > 0 the cell size (ignored for a >= ndim), gamma > 1 the ratio of
 * specific heats.  state[b][q] is field q of buffer b (q < ndim+2), a
 * device pointer; the two buffers must not overlap.  The library reads the
 * current state from one buffer and writes the next state to the other
 * (paraiso_current says which holds the current state).
 * order selects the reconstruction of the Interpolate equation: 2 (or 0)
 * piecewise linear with the minbee limiter, 1 piecewise constant (each face
 * takes the values of the two cells beside it: the order-1 branch of the
 * paper's interpolation listing, section "Annotating By Hand"; runs on the
 * LDS-tile kernels, and all meshes of a batch share it).
 * Limits: n[0]*n[1]*n[2] < 2^31.
 */
typedef struct paraiso_mesh {
  int32_t ndim;
  int32_t dtype;
  int64_t n[3];
  double dx[3];
  double gamma;
  int32_t bc[3];
  int32_t order;
  void* state[2][5];
} paraiso_mesh;

/*
 * Kernel variant (the tuning space).  These choices change speed, never
 * results beyond floating-point rounding.
 *   tile[a]      cells per workgroup tile along axis a (1 for unused axes);
 *   lds          staging of the stencil:
 *                0: every cell computes its own 2d face fluxes from global
 *                   memory;
 *                1: LDS tiles, each face flux computed once per tile;
 *                2: register march (2D and 3D): a wave per strip of 64
 *                   columns (tile[0] = 64) marching along the last axis,
 *                   x-neighbours by lane shifts; 2D: tile[1] rows per wave,
 *                   threads / 64 waves per block; the fused 2D form needs
 *                   periodic boundaries, and with at least 2 waves of at
 *                   least 6 rows its waves share stage-1 rows through LDS
 *                   (a block then covers waves * rows - 2 rows); 3D:
 *                   tile[2] planes per block; one stage per launch
 *                   (fuse = 0): tile[1] = 4 or 8 rows (= waves) per
 *                   block; fused (fuse = 1, periodic meshes): tile[1] =
 *                   6..12 stage-1 rows (= waves) per block, of which
 *                   tile[1] - 4 are output rows (FP64: 6, the LDS limit);
 *                3: resident (1D, at most 4096 cells per mesh in FP32 and
 *                   3407 in FP64, the LDS of one workgroup holding
 *                   8 * (6n + 3) bytes): one workgroup per mesh runs a
 *                   whole paraiso_advance in one launch;
 *   fuse         1: both Runge-Kutta stages in one launch, stage 1
 *                recomputed on a halo of 2 cells; 0: one launch per stage,
 *                stage-1 state kept in the workspace;
 *   waves_per_eu 0 (compiler's choice, at most 256 VGPRs), 3, 4 or 5:
 *                minimum waves per SIMD the kernel is compiled for, which
 *                caps registers per lane at 168, 128 or 100;
 *   threads      workgroup size, a multiple of 64 in [64, 512], or 0 for
 *                the default of the chosen kernel (the 3D register march:
 *                64 * tile[1], up to 768 when fused; the resident kernel:
 *                512 or 1024, each thread holding up to 4 cells, and 0
 *                picks 512 for meshes of at most 2048 cells, else 1024);
 *   manifest     what an LDS tile (lds = 1) keeps between the phases of an
 *                axis, the paper's Manifest/Delayed choice for the results
 *                of the interpolation and of the Riemann solver (section
 *                "Annotating By Hand"):
 *                0: face fluxes, each face's states formed where its flux is
 *                   computed (interpolation delayed, Riemann manifest);
 *                1: face states; each cell solves both of its faces
 *                   (interpolation manifest, Riemann delayed);
 *                2: face states, then face fluxes (both manifest).
 *                lds = 0 delays both.  Nonzero only with lds = 1 on
 *                second-order meshes without analytic boundaries.
 */
typedef struct paraiso_variant {
  int32_t tile[3];
  int32_t lds;
  int32_t fuse;
  int32_t waves_per_eu;
  int32_t threads;
  int32_t persistent;  /* 1: grid of a few workgroups per CU pulling tiles from a queue;
                          0: one workgroup per tile (the default, also for batches),
                          unless that grid would pass 2^32 work-items (rows of
                          very few rows, tiny tiles): then the queue, and
                          paraiso_get_variant reports 1 */
  int32_t manifest;
} paraiso_variant;

typedef struct paraiso_ctx paraiso_ctx;

/*
 * Bytes of device workspace needed for `count` meshes (stage-1 state for
 * the unfused variants, per-mesh time-stepping control, reduction partials,
 * mesh table, work queue).  The figure covers every variant, so
 * paraiso_set_variant never needs a larger workspace.
 * Errors: INVALID_ARG for a null pointer or an invalid mesh.
 */
int32_t paraiso_workspace_bytes(const paraiso_mesh* meshes, int32_t count, size_t* bytes);

/*
 * Create a context over `count` meshes (count > 1: a batch of independent
 * meshes that are stepped together; all must share ndim and dtype).
 * `workspace` is a device buffer of at least paraiso_workspace_bytes bytes,
 * 256-byte aligned, borrowed for the context's lifetime.  `hip_stream` is a
 * hipStream_t (NULL = the default stream).  The mesh descriptors are copied;
 * buffer 0 holds the initial state.
 * Errors: INVALID_ARG (null pointers, ndim not in 1..3, n < 1, gamma <= 1,
 * dx <= 0 or non-finite, bc not PERIODIC/OUTFLOW/ANALYTIC, order not 0/1/2,
 * overlapping buffers, mixed ndim/dtype/order in a batch), UNSUPPORTED (too many cells),
 * WORKSPACE (workspace too small), HIP.
 */
int32_t paraiso_init(const paraiso_mesh* meshes, int32_t count, void* workspace,
                     size_t workspace_bytes, void* hip_stream, paraiso_ctx** out);

/* Select the kernel variant.  UNSUPPORTED if the variant does not fit the
 * hardware limits (LDS bytes, threads, registers) or the mesh. */
int32_t paraiso_set_variant(paraiso_ctx* ctx, const paraiso_variant* v);
int32_t paraiso_get_variant(const paraiso_ctx* ctx, paraiso_variant* v);

/* The default variant the library picks for these meshes (and applies in
 * paraiso_init): 1D the resident kernel when every mesh fits one
 * workgroup, else LDS tiles; 2D the fused register march when every mesh is
 * periodic on both axes, else LDS tiles; 3D the register march.  Any mesh
 * with an analytic axis: in 2D the one-stage register march, else unfused
 * LDS tiles; first order: LDS tiles.  One workgroup per tile (persistent =
 * 0), batches included. */
int32_t paraiso_default_variant(const paraiso_mesh* meshes, int32_t count, paraiso_variant* v);

/*
 * CFL time step of the current state of every mesh:
 * dt_out[m] = cfl / max_i sum_a (|v_a| + c)/dx_a, computed in FP64 whatever
 * the state's element type.  Synchronous.  0 < cfl <= 1.
 * Defined by: the time step of the two-stage marching is set by the CFL
 * condition (section "Tuning Experiments / The Target Program", the sentence
 * before the time-marching equations; the paper does not print the formula,
 * this is the reading every kernel and the oracle share), taken over the mesh
 * as the Orthotope Machine's Reduce with the Min operator (section "Outline of
 * The Orthotope Machine", paragraph Reduce): a global value folded from every
 * cell's local value; here the maximum of the signal-speed term, whose
 * reciprocal is the minimum time step.
 * Errors: INVALID_ARG, NONFINITE (any cell with rho <= 0, p <= 0 or a
 * non-finite value; dt_out is then unspecified), HIP.
 */
int32_t paraiso_cfl_dt(paraiso_ctx* ctx, double cfl, double* dt_out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the CFL
 * time step of paraiso_cfl_dt without a context or workspace.  The call
 * returns dt to the host, so it synchronizes and is not itself recorded
 * into a graph; it allocates nothing, and clears its control blocks with a
 * kernel rather than a memset.
 * dt_out[m] = cfl / max_i sum_a (|v_a| + c)/dx_a over the state in buffer
 * `buffer` (0 or 1) of meshes[m], in FP64, for 1 <= count <=
 * PARAISO_STATIC_MESHES meshes that share ndim and dtype; it reads ndim,
 * dtype, n, dx, gamma and state[buffer] of each descriptor (bc and order do
 * not enter the CFL term).  Results equal paraiso_cfl_dt's bit for bit (same
 * reduction kernel).  The mesh table and the reduction's control blocks live
 * in a fixed device array of the library (at most 48 KiB per device, held
 * until the process ends); nothing is allocated on the host or the device.
 * Every call on a device shares that device's array, so calls that overlap
 * on one device (other threads, other streams) race.  Synchronous on
 * `hip_stream`, which must belong to the current device.
 * Errors: INVALID_ARG (null pointers, count < 1, buffer not 0/1, cfl outside
 * (0, 1], an invalid descriptor), UNSUPPORTED (count > PARAISO_STATIC_MESHES,
 * more than 2^31 - 1 cells, device index > 63), NONFINITE, HIP.
 */
#define PARAISO_STATIC_MESHES 64
int32_t paraiso_cfl_dt_static(const paraiso_mesh* meshes, int32_t count, int32_t buffer, double cfl,
                              double* dt_out, void* hip_stream);

/*
 * One midpoint-RK2 step of every mesh with the caller's time steps
 * dt[m] >= 0 (finite): F0 = Flux(U0), U1 = AddFlux(dt/2, F0, U0),
 * F1 = Flux(U1), U2 = AddFlux(dt, F1, U0) (section "Tuning Experiments / The
 * Target Program", the time-marching equations and the AddFlux equation).  It
 * is the generated solver class's proceed() of the paper (section "Tuning
 * Targets", the generated code listing): a call that advances the class's
 * static state arrays in place; here the state moves between the two buffers.  Reads the current buffer, writes the other one and
 * makes it current; the device-held time advances by dt[m].  Asynchronous
 * on the context's stream.
 * Errors: INVALID_ARG (also: an analytic mesh without a problem set), HIP.
 */
int32_t paraiso_step(paraiso_ctx* ctx, const double* dt);

/*
 * Advance every mesh from t_inout[m] towards t_end with dt = CFL step
 * clamped so that no step passes t_end, for at most max_steps steps per
 * mesh: repeated proceed() calls of the generated class (section "Tuning
 * Targets") with the time step of each from the CFL reduction of its input
 * (paraiso_cfl_dt), as the target program's time marching prescribes
 * (section "Tuning Experiments / The Target Program").  The time step, the time and the step count stay on the device;
 * step sequences are replayed from captured HIP graphs.  On return
 * t_inout[m] and steps_out[m] hold each mesh's time and steps taken.
 * Synchronous.  0 < cfl <= 1, max_steps >= 0, t_end finite.
 * Errors: INVALID_ARG, NONFINITE (a mesh's state became non-physical, as
 * the CFL reduction of each new state detects: that mesh takes no further
 * step, its current buffer holds the offending step's output and
 * t_inout[m] and steps_out[m] that step's time and count; the other meshes
 * of a batch have advanced to where the call stopped), HIP.
 */
int32_t paraiso_advance(paraiso_ctx* ctx, double t_end, double cfl, int64_t max_steps,
                        double* t_inout, int64_t* steps_out);

/*
 * Analytic boundaries: the convergence tests of section "Tuning Experiments
 * / Automated Tuning" (the convergence-test figure and the initial
 * conditions given with it).  Cell i of axis a has its centre at
 * x_a = (i + 1/2) dx[a] (the tests use the unit square, dx[a] = 1/n[a]).  On
 * each axis whose bc is PARAISO_ANALYTIC, cells outside the mesh take the
 * exact solution at their centres, evaluated in FP64 at the time the
 * stage's input stands for:
 * stage 1 at the step's time t, stage 2 at t + dt/2 (the midpoint state).
 * With s = (x - 1/2) cos(angle) + (y - 1/2) sin(angle) + 1/2 and the
 * velocity along n = (cos(angle), sin(angle), 0):
 *   PARAISO_ENTROPY_WAVE  rho = 2 + sin 2 pi (s - t), |v| = 1, p = 1;
 *   PARAISO_SOUND_WAVE    w = amplitude sin 2 pi (s - t): rho = gamma (1 + w),
 *                         v_n = w, p = 1 + gamma w (sound speed 1; exact to
 *                         first order in the amplitude);
 *   PARAISO_SHOCK_TUBE    Sod's tube (1, 0, 1) | (0.125, 0, 0.1) split at
 *                         s = 1/2, the exact Riemann solution at (s - 1/2)/t
 *                         (the star state solved on the host in FP64).
 * angle must be 0 in 1D ("coaxial"; the "oblique" tests use pi/3).
 * Meshes with an analytic axis run on the unfused LDS-tile kernel (variant
 * lds = 1, fuse = 0) or, in 2D, the one-stage register march (lds = 2,
 * fuse = 0, the default), which reads its ghost cells from arrays in the
 * workspace that a small kernel fills before every step.
 */
typedef struct paraiso_analytic {
  int32_t kind;      /* PARAISO_ENTROPY_WAVE, PARAISO_SOUND_WAVE or PARAISO_SHOCK_TUBE */
  int32_t reserved;  /* 0 */
  double angle;      /* radians; finite, 0 in 1D */
  double amplitude;  /* sound wave: finite, |amplitude| < 1; ignored otherwise */
} paraiso_analytic;

/*
 * Set the exact solution of mesh `mesh`, which must have a PARAISO_ANALYTIC
 * axis.  Stepping a context with an analytic mesh whose problem is not set
 * fails with INVALID_ARG.  Synchronous (uploads the mesh table).
 * Errors: INVALID_ARG (null pointer, mesh out of range or without an
 * analytic axis, kind, angle or amplitude out of range), HIP.
 */
int32_t paraiso_set_analytic(paraiso_ctx* ctx, int32_t mesh, const paraiso_analytic* an);

/*
 * Write the exact conserved state of mesh `mesh`'s problem at time t
 * (finite) at every cell centre into its state buffer `buffer` (0 or 1):
 * initial conditions and reference solutions of the convergence tests.
 * Evaluated in FP64, rounded once to the element type.  Asynchronous on the
 * context's stream.
 * Errors: INVALID_ARG (null context, mesh or buffer out of range, no
 * problem set), HIP.
 */
int32_t paraiso_exact_state(paraiso_ctx* ctx, int32_t mesh, double t, int32_t buffer);

/*
 * Simulation time of every mesh, t[m] (finite), kept on the device and
 * advanced by paraiso_step and paraiso_advance; the analytic ghosts read it.
 * paraiso_init starts it at 0; paraiso_advance starts it from t_inout.
 * Synchronous.  Errors: INVALID_ARG, HIP.
 */
int32_t paraiso_set_time(paraiso_ctx* ctx, const double* t);
int32_t paraiso_get_time(paraiso_ctx* ctx, double* t_out);

/* Index (0 or 1) of the buffer holding the current state. */
int32_t paraiso_current(const paraiso_ctx* ctx, int32_t* idx);

/*
 * Conserved totals of the current state: out[m*(ndim+2) + q] = cell volume
 * times the sum over cells of field q of mesh m, accumulated in FP64 in a
 * fixed order (bitwise reproducible for a given variant).  Synchronous.
 * Defined by: the Reduce of the Orthotope Machine with the Sum operator
 * (section "Outline of The Orthotope Machine", paragraph Reduce), which the
 * paper's linear-wave example applies to audit its discrete energy (section
 * "An Example of Orthotope Machine Data-Flow Graph"); here the audited
 * quantities are the conserved mass, momenta and energy of the Euler state.
 * Errors: INVALID_ARG (null pointer), HIP.
 */
int32_t paraiso_totals(paraiso_ctx* ctx, double* out);

/*
 * The linear-wave example (section "An Example of Orthotope Machine
 * Data-Flow Graph"): f_t = g, g_t = c^2 f_xx on a periodic line of n cells,
 * advanced by the paper's two-level scheme
 *   f^{k+1}[i] = f^k[i] + dt g^k[i],
 *   g^{k+1}[i] = g^k[i] + (c^2 dt / dx^2)(f^{k+1}[i+1] + f^{k+1}[i-1] - 2 f^{k+1}[i]),
 * and, after every step, the discrete energy in the form of the paper's
 * source listing
 *   E^{k+1} = sum_i (c^2 ((f^{k+1}[i+1] - f^{k+1}[i-1]) / (2 dx))^2
 *                    + ((g^k[i] + g^{k+1}[i]) / 2)^2) dx / 2,
 * which at dt = dx / c is an exact invariant of the scheme (the paper finds
 * it constant to about 1e-13 in FP64).  FP64 throughout.
 *
 * One line: n cells, 3 <= n <= PARAISO_WAVE_MAX_CELLS; c >= 0 and dt >= 0
 * finite, dx > 0 finite; f and g device arrays of n doubles, read at the
 * start and overwritten with the final state; energy a device array of
 * `steps` doubles (E after each step) or NULL.  Arrays 8-byte aligned,
 * owned by the caller, not overlapping.
 */
#define PARAISO_WAVE_MAX_CELLS 4096
typedef struct paraiso_wave {
  int64_t n;
  double c;
  double dx;
  double dt;
  double* f;
  double* g;
  double* energy;
} paraiso_wave;

/* Bytes of device workspace paraiso_wave_advance needs for `count` lines
 * (the device copy of the line table).  Errors: INVALID_ARG. */
int32_t paraiso_wave_workspace_bytes(int32_t count, size_t* bytes);

/*
 * Validate `count` lines and copy their table into `workspace`, a device
 * buffer of at least paraiso_wave_workspace_bytes(count) bytes, 256-byte
 * aligned (synchronous on `hip_stream`).
 * Errors: INVALID_ARG (null pointers, count < 1, a line out of range: the
 * message names it), WORKSPACE, HIP.
 */
int32_t paraiso_wave_prepare(const paraiso_wave* lines, int32_t count, void* workspace, size_t workspace_bytes,
                             void* hip_stream);

/*
 * Advance the `count` lines prepared in `workspace` by `steps` steps each,
 * one workgroup per line, enqueued on `hip_stream` (asynchronous).
 * `max_cells` is the largest n among the prepared lines: it selects the
 * kernel's cells per thread (ceil(max_cells / 256), rounded up to 1, 2, 3,
 * 4, 6, 8, 12 or 16); a line longer than that allows is left untouched.
 * Each line's energy array receives E after each of these steps (from
 * index 0).  The energy sums are taken in a fixed order: results are
 * bitwise reproducible.  Errors: INVALID_ARG (null workspace, count < 1,
 * steps < 0, max_cells outside [3, PARAISO_WAVE_MAX_CELLS], misaligned
 * workspace), HIP.
 */
int32_t paraiso_wave_run(const void* workspace, int32_t count, int64_t steps, int64_t max_cells,
                         void* hip_stream);

/* paraiso_wave_prepare, then paraiso_wave_run. */
int32_t paraiso_wave_advance(const paraiso_wave* lines, int32_t count, int64_t steps, void* workspace,
                             size_t workspace_bytes, void* hip_stream);

/* Release the context (never the caller's buffers).  NULL is a no-op. */
int32_t paraiso_destroy(paraiso_ctx* ctx);

/* Message of the last failed call on this thread ("" if none). */
const char* paraiso_last_error(void);

/* Library version string. */
const char* paraiso_version(void);

/* ------------------------------------------------------------------------
 * Cost model of the kernel tuner: a multilayer perceptron in -> H -> H -> 1
 * with ReLU hidden layers, trained with mean-squared error and Adam.  It
 * predicts a variant's benchmark score from its features before the variant
 * is benchmarked (the paper lists such prediction as future work for its
 * tuner, section "Conclusion and Discussion").
 *
 * Parameters: one packed FP32 device array W1[in][H], b1[H], W2[H][H],
 * b2[H], w3[H], b3 (row-major, input index first).  X is a device array
 * [batch][in] (row-major).  All pointers are device pointers owned by the
 * caller; the workspace holds activations.  Calls are asynchronous on
 * `hip_stream` and bitwise reproducible (fixed-order reductions).
 * Errors: INVALID_ARG (null pointer, batch/in/H < 1, in > 4096, H > 1024),
 * WORKSPACE, HIP.
 * ---------------------------------------------------------------------- */

/* Number of parameters and workspace bytes for a batch size. */
int32_t paraiso_mlp_sizes(int32_t in_dim, int32_t hidden, int32_t batch, int64_t* n_params,
                          size_t* workspace_bytes);

/* y[b] = network output for X[b]. */
int32_t paraiso_mlp_forward(const float* X, int32_t batch, int32_t in_dim, int32_t hidden,
                            const float* params, float* y, void* workspace, size_t workspace_bytes,
                            void* hip_stream);

/* loss = mean_b (y[b] - target[b])^2 (device scalar; may be NULL) and its
 * gradient with respect to every parameter, packed like the parameters. */
int32_t paraiso_mlp_loss_grad(const float* X, const float* target, int32_t batch, int32_t in_dim,
                              int32_t hidden, const float* params, float* grad, float* loss,
                              void* workspace, size_t workspace_bytes, void* hip_stream);

/* One Adam update (Kingma & Ba) of n parameters in place; step >= 1 is the
 * 1-based update count used for bias correction; m and v are the moment
 * buffers (zero before the first step). */
int32_t paraiso_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t n, float lr,
                         float beta1, float beta2, float eps, int32_t step, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* PARAISO_H */
