/*
 * lx.h - C ABI of an MI355X (gfx950) library for the action of phi functions
 * of a matrix-free stencil operator, phi_l(hA)v, by Newton interpolation at
 * scaled and shifted Leja points.
 *
 * Method (Deka, Moriggl, Einkemmer, "LeXInt: GPU-accelerated Exponential
 * Integrators package", SoftwareX; arXiv 2310.08344):
 *   - phi functions: Sec. 1, phi_0 = exp, phi_{l+1}(z) = (phi_l(z) - 1/l!)/z;
 *   - Leja points of [-2, 2] and the Newton recurrence: Sec. 2.1, Eq. (2):
 *       p_0 = d_0 y_0,  y_{m+1} = ((A - c)/gamma - xi_m) y_m,
 *       p_{m+1} = p_m + d_{m+1} y_{m+1},
 *     d_j the divided differences of sigma*phi_l(alpha*h*(c + gamma*xi));
 *   - stop rule: Sec. 2.2 (text with Listing 2): error estimate at most
 *     rtol*||p|| + atol, l2 norms divided by sqrt(N); the estimate used here
 *     is |d_{m+1}| * ||y_{m+1}|| / sqrt(N);
 *   - shift and scale from power iteration: Sec. 2 and Listing 7,
 *     lambda = -safety*rho_hat, c = lambda/2, gamma = -lambda/4;
 *   - several phi outputs from one Newton basis ("vertical" interpolation):
 *     Sec. 2.3, Listing 11;
 *   - exponential Rosenbrock steps with the nonlinear remainder
 *     N(w) = f(w) - J(u_n) w: Sec. 2.3 (Listings 12 and 13).
 *
 * Conventions shared by every entry point
 *   Grids are periodic nx x ny, stored row-major [ny][nx] (x fastest),
 *   contiguous, FP64, in device memory owned by the caller (Sec. 2.2, the
 *   caller allocates input and output arrays, Listing 4).  The library owns
 *   only its context workspaces, allocated once by lx_create (Sec. 2.3,
 *   Listing 10: allocate once per object, free in the destructor).
 *   All device work is enqueued on the stream given to lx_create; every call
 *   that returns host values waits for that stream once, at its end, except
 *   that a Leja loop returns as soon as it has read its final state: the few
 *   launches it enqueued past the end then still run on the stream (they
 *   read the loop state and return; every output is final on return).
 *   A context is not thread-safe: one host thread at a time per context.
 *   Every call returns an lx_status; on an error other than LX_ENOTCONV the
 *   outputs are unspecified and lx_last_error() holds a message.
 */
#ifndef LX_H
#define LX_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LX_K_MAX 4          /* most phi outputs per Newton basis            */
#define LX_MAX_ITERS 1000   /* most Leja iterations (operator applications) */

typedef struct lx_ctx lx_ctx;

typedef enum {
    LX_OK = 0,
    LX_EINVAL = 1,      /* bad argument: sizes, null pointers, c > 0, gamma <= 0, ... */
    LX_ENOMEM = 2,      /* device or pinned host allocation failed                    */
    LX_ENOTCONV = 3,    /* max_iters reached; outputs hold the last polynomial        */
    LX_ENONFINITE = 4,  /* a norm became NaN or Inf; outputs unspecified              */
    LX_EDEVICE = 5      /* a HIP call failed                                           */
} lx_status;

typedef enum {
    /* A y = D*lap(y) + vx*Ux(y) + vy*Uy(y): centred 5-point Laplacian and a
     * first-order upwind difference on the side that keeps Re(sigma(A)) <= 0
     * (v > 0 forward, v < 0 backward); Sec. 3, Eq. (3).                     */
    LX_OP_DIFFADV2D = 1,
    /* F(u) = nu*lap(u) - (1/2)(d_x + d_y)(u^2), centred differences, and its
     * Jacobian J(u) w = nu*lap(w) - (d_x + d_y)(u w); Sec. 3, Eq. (5).       */
    LX_OP_BURGERS2D = 2,
    /* A y = D*lap(y) + vx*Dx(y) + vy*Dy(y) with the paper's third-order
     * upwind gradient (Sec. 3): per axis the four-point upwind-biased
     * difference, exact for cubics, on points i-1..i+2 for v >= 0,
     *   Dx y = (-y_{i+2} + 6 y_{i+1} - 3 y_i - 2 y_{i-1}) / (6 dx),
     * and mirrored (points i-2..i+1) for v < 0; a radius-2 stencil.  Grids
     * need sides >= 4.  Not accepted by the batched and learned calls.     */
    LX_OP_DIFFADV2D_UP3 = 3
} lx_op_kind;

typedef enum {
    LX_FP64 = 0,        /* basis vectors, stencil arithmetic and accumulation in FP64 */
    LX_FP32_SWEEP = 1   /* basis vectors and stencil arithmetic in FP32 once the
                           terms are small (see lx_leja_opts.fp32_switch); Leja
                           points, divided differences, norms and the polynomial
                           stay FP64                                               */
} lx_prec;

typedef struct {
    int kind;           /* lx_op_kind                                 */
    int nx, ny;         /* grid, each >= 3                            */
    double dx, dy;      /* spacings, > 0                              */
    double D;           /* LX_OP_DIFFADV2D: diffusion coefficient >= 0 */
    double vx, vy;      /* LX_OP_DIFFADV2D: advection velocity        */
    double nu;          /* LX_OP_BURGERS2D: viscosity >= 0            */
    int prec;           /* lx_prec                                    */
} lx_operator;

typedef struct {
    double rtol, atol;  /* stop when |d_{m+1}| ||y_{m+1}|| <= rtol ||p|| + atol (rms norms) */
    int max_iters;      /* 1 .. LX_MAX_ITERS                                              */
    /* LX_FP32_SWEEP only: FP32 sweeps start after the first iteration at which
     * every unconverged output has |d_{m+1}| ||y_{m+1}|| <=
     * fp32_switch * (rtol ||p|| + atol).  0 means FP32 from the first sweep.  */
    double fp32_switch;
    /* Substeps s (not in the paper): the Leja loop loses accuracy once
     * alpha*h*gamma is large (it diverges near 800 on the diffusion-
     * advection operators), so each output may be computed over s substeps
     * of tau = alpha*h/s: exp(alpha h A) v = exp(tau A)^s v, and for l >= 1
     * by phi-function time stepping (Niesen and Wright 2012): with
     * u(t) = t^l phi_l(tA) v,
     *   u(t + tau) = e^{tau A} u(t) + sum_{i=1..l} tau^i t^{l-i}/(l-i)! phi_i(tau A) v,
     * phi_1..phi_l(tau A) v from one Newton basis, one exp action per
     * substep, each call with its own stop rule.
     * 0: automatic, s = ceil(max_k alpha_k * h * gamma / 300);
     * 1 .. LX_MAX_SUBSTEPS: that many.  Batched calls ignore it.            */
    int substeps;
} lx_leja_opts;

#define LX_MAX_SUBSTEPS 1000

/* Per-call record, filled by every lx_spectrum / lx_phi_leja / lx_exprb_step. */
typedef struct {
    int status;             /* lx_status of the call                          */
    int n_apply;            /* operator applications made                     */
    int n_fp32;             /* of which in FP32 (LX_FP32_SWEEP)               */
    int iters[LX_K_MAX];    /* per output: sweeps until it passed the test    */
    double err[LX_K_MAX];   /* per output: last error estimate                */
    double pnorm[LX_K_MAX]; /* per output: rms norm of the result             */
    double rho_hat;         /* lx_spectrum: spectral estimate                 */
    double plan_ms;         /* host planner time (Leja table, coefficients)   */
    double loop_ms;         /* device loop, first to last sweep (timing on)   */
    double sweep_ms;        /* sum of the working sweeps' durations (timing)  */
    double first_sweep_ms;  /* duration of sweep 0 (timing on)                */
    double bytes;           /* algorithmic HBM bytes of the working sweeps    */
    int n_launch;           /* Leja-loop launches that did work               */
    int depth;              /* Leja iterations per launch: 1, 2, 3, 4, 6 or 8
                               (lx_spectrum: power sweeps per launch)        */
    double step_err;        /* lx_exprb_step with LX_EXPRB32: embedded error  */
    int substeps;           /* substeps taken (lx_leja_opts.substeps)         */
    int marching;           /* 1: the windows (lx_spectrum: the power sweeps)
                               ran by register marching, 0 otherwise         */
    int batch_graph;        /* lx_phi_leja_batched: 1 when the call replayed a
                               captured pipeline (lx_set_batch_graphs)       */
} lx_stats;

/* ---- context ---------------------------------------------------------- */

/* Creates a context for grids of at most n_max points and at most k_max
 * (<= LX_K_MAX) outputs per basis; allocates every device workspace once
 * (Listing 10).  stream is a hipStream_t (NULL = the null stream).  The
 * current HIP device at this call is the context's device.
 * Errors: LX_EINVAL (n_max < 9, k_max out of range), LX_ENOMEM, LX_EDEVICE. */
lx_status lx_create(lx_ctx** ctx, size_t n_max, int k_max, void* stream);

/* Frees every workspace (Listing 10, destructor) and destroys the
 * predictors created on this context, whose handles become invalid.
 * NULL is a no-op. */
void lx_destroy(lx_ctx* ctx);

/* Changes the stream later calls enqueue on, after waiting for the one
 * before.  Errors: LX_EDEVICE (that wait failed). */
lx_status lx_set_stream(lx_ctx* ctx, void* stream);

/* on != 0: record HIP events around every sweep so that lx_stats carries
 * loop_ms, sweep_ms and first_sweep_ms.  Off by default. */
lx_status lx_set_timing(lx_ctx* ctx, int on);

/* Last error message of this context (static storage, valid until the next
 * call on it). */
const char* lx_last_error(const lx_ctx* ctx);
const char* lx_status_string(int status);

/* Copies the record of the last call. */
lx_status lx_get_stats(const lx_ctx* ctx, lx_stats* out);

/* ---- spectral bound --------------------------------------------------- */

/* Power iteration for the dominant eigenvalue modulus of A (LX_OP_DIFFADV2D)
 * or of the Jacobian J(u) (LX_OP_BURGERS2D, d_u = the state), then the Leja
 * shift and scale of Listing 7:
 *   w_0 = x0;  w_{k+1} = A w_k / ||w_k||;  rho_hat = ||w_iters||
 *   lambda = -safety * rho_hat;  c = lambda / 2;  gamma = -lambda / 4.
 * d_x0: start vector (nx*ny FP64, device, not modified); NULL = the library
 * fills one with splitmix64 values in [-1, 1) (seed 0).  A constant start
 * vector is invalid: it lies in the null space of the periodic operators.
 * iters >= 1 applications of the operator (20 is customary).
 * rho_hat, c, gamma: host outputs, each may be NULL.
 * Errors: LX_EINVAL (op invalid, size > n_max, d_u missing for Burgers,
 * iters < 1, safety <= 0), LX_ENONFINITE (zero or non-finite norm). */
lx_status lx_spectrum(lx_ctx* ctx, const lx_operator* op, const double* d_u,
                      const double* d_x0, int iters, double safety,
                      double* rho_hat, double* c, double* gamma);

/* ---- phi actions ------------------------------------------------------ */

/* For k = 0..K-1:  d_out[k] = sigma[k] * phi_{l[k]}(alpha[k] * h * A) d_v,
 * all K outputs from one Newton basis (Sec. 2.1 Eq. (2); vertical outputs,
 * Listing 11).  Covers real_Leja_exp (K = 1, l = 0) and real_Leja_phi_nl /
 * real_Leja_phi (l >= 1) of Listings 2, 3, 8, 9 and 11.
 *   op      operator; LX_OP_BURGERS2D uses the Jacobian J(d_u)
 *   d_u     device state for the Jacobian (Burgers), else NULL
 *   d_v     device input vector (nx*ny), not modified
 *   K       1 .. k_max outputs;  l[k] in 0..8;  alpha[k] > 0 (NULL = all 1);
 *           sigma[k] (NULL = all 1)
 *   d_out   K device output vectors, distinct, none equal to d_v or d_u
 *   h > 0 step; c <= 0 and gamma > 0 from lx_spectrum (the Leja interval
 *           [-2, 2] maps onto [c - 2 gamma, c + 2 gamma])
 *   o       tolerances, iteration cap and substeps (NULL = rtol 1e-8,
 *           atol 0, 500, automatic substeps)
 *   iters   host [K] or NULL: sweeps until each output passed (with
 *           substeps: the sweeps of its phi_l call plus its exp calls)
 *   err     host [K] or NULL: each output's last error estimate
 * Each output freezes once it passes; the call ends when all have passed,
 * or with LX_ENOTCONV after max_iters sweeps (outputs then hold the last
 * polynomial; with substeps, of the call that did not converge), or with
 * LX_ENONFINITE.  With more than one substep the call allocates, on first
 * use, up to 10 workspace vectors of the context's n_max. */
lx_status lx_phi_leja(lx_ctx* ctx, const lx_operator* op, const double* d_u,
                      const double* d_v, int K, const int* l, const double* alpha,
                      const double* sigma, double* const* d_out, double h,
                      double c, double gamma, const lx_leja_opts* o,
                      int* iters, double* err);

/* For callers that cannot allocate device memory (code in serving loops
 * or harnesses that forbid allocation after set-up): lx_phi_leja with every
 * device buffer its kernels use beyond the inputs, the outputs and the
 * context's fixed workspaces (the Newton basis pair, the windows' second
 * output buffers, the partial sums) taken from the library's static device
 * scratch instead of the context, so the call allocates no device memory,
 * also on its first use (lx_phi_leja grows its workspaces on demand).  The
 * scratch is a file-scope device array of (2 + LX_K_MAX) * 2^18 + 327680
 * doubles (about 15 MB) that every GPU the library runs on holds until the
 * process ends; its address on a device is looked up on the first call on
 * that device.  Arguments, results, errors and launch shapes as
 * lx_phi_leja, with these limits (LX_EINVAL beyond them): nx * ny <= 2^18
 * points (the context's n_max does not apply), FP64 sweeps, no substeps
 * (lx_leja_opts.substeps 0 must resolve to one), and timing (lx_set_timing)
 * is not recorded.  Every call on a GPU shares that GPU's scratch, which
 * keeps the last call's contents (no buffer needs to start at zero: every
 * launch writes what the next one reads): calls that overlap on one GPU,
 * on any streams or contexts, race and must be serialised by the caller.
 * The host planner (Leja points, divided differences) keeps its own
 * bounded host tables. */
lx_status lx_phi_leja_static(lx_ctx* ctx, const lx_operator* op, const double* d_u,
                             const double* d_v, int K, const int* l, const double* alpha,
                             const double* sigma, double* const* d_out, double h,
                             double c, double gamma, const lx_leja_opts* o,
                             int* iters, double* err);

/* ---- exponential integrator steps ------------------------------------- */

/* In all three, J = J(u) and N(w) = F(w) - J w (Sec. 2.3); every phi
 * action is a Leja pass of its own, whose stop rule measures that action
 * alone, and the stages are summed afterwards. */
typedef enum {
    /* exponential Rosenbrock-Euler, second order (Sec. 2.3):
     *   u+ = u + h phi_1(h J) F(u)                                            */
    LX_ROS_EULER = 2,
    /* EXPRB32, third order with an embedded second-order solution (Sec. 2.3):
     *   a  = u + h phi_1(h J) F(u)
     *   u+ = a + 2 h phi_3(h J) [N(a) - N(u)];
     * lx_stats.step_err receives the rms norm (l2 / sqrt(N)) of the
     * correction u+ - a, the embedded error estimate.                        */
    LX_EXPRB32 = 32,
    /* two-stage fourth-order exponential Rosenbrock method (named in Sec. 1;
     * formula of the published method, c_2 = 3/4):
     *   U2  = u + (3/4) h phi_1((3/4) h J) F(u)
     *   u+  = u + h phi_1(h J) F(u) + (32/9) h phi_3(h J) [N(U2) - N(u)];
     * both phi_1 actions come from one Newton basis.                         */
    LX_EXPRB42 = 42
} lx_scheme;

/* One step u -> d_u_out of u_t = F(u) for LX_OP_BURGERS2D (Sec. 2.3: the
 * integrator entry point of the exponential Rosenbrock listings).  c and
 * gamma describe the spectrum of J(d_u) (lx_spectrum with d_u).
 *   d_u, d_u_out  device, nx*ny, caller-owned; d_u_out must differ from d_u.
 *   d_u_low       device, nx*ny, or NULL.  LX_EXPRB32 only (the one scheme
 *                 with an embedded method): receives the embedded
 *                 second-order solution a = u + h phi_1(h J) F(u).  Must
 *                 differ from d_u and d_u_out; LX_EINVAL for another scheme.
 *   err           host, or NULL: LX_EXPRB32's embedded error estimate, the
 *                 rms norm (l2 / sqrt(N)) of u+ - a (the EXPRB32 listing's
 *                 `error`); 0 for the other schemes, which have none.
 *   iters         host [3], or NULL: iterations of every phi action of the
 *                 step in the order taken, each with its own stop rule:
 *                 LX_ROS_EULER {phi_1, 0, 0}; LX_EXPRB32 {phi_1, phi_3, 0};
 *                 LX_EXPRB42 {(3/4) phi_1((3/4) h J), phi_1(h J), phi_3}
 *                 (the first two from one Newton basis).
 * Three workspace vectors of the context's n_max are allocated on the first
 * call.  Errors as lx_phi_leja; LX_EINVAL for another operator or scheme,
 * or LX_EXPRB42 on a context with k_max < 2. */
lx_status lx_exprb_step(lx_ctx* ctx, const lx_operator* op, int scheme,
                        const double* d_u, double* d_u_out, double* d_u_low,
                        double* err, double h, double c, double gamma,
                        const lx_leja_opts* o, int* iters);

/* One step of the linear problem u_t = A u + S (Sec. 3, Problems I and
 * II) for LX_OP_DIFFADV2D or LX_OP_DIFFADV2D_UP3:
 *   d_src == NULL:  u+ = exp(h A) u                       (Problem I)
 *   otherwise:      u+ = u + h phi_1(h A) (A u + S)       (Problem II)
 * d_src: device, nx*ny, the time-independent source, or NULL.  c and gamma
 * describe the spectrum of A (lx_spectrum).  The phi action's stop rule
 * measures that action alone (Problem II) or exp(h A) u (Problem I).
 * iters: host, or NULL: iterations taken.  d_u_out must differ from d_u
 * and d_src.  The first call with a source allocates one workspace vector
 * of the context's n_max.  Errors as lx_phi_leja (after LX_ENOTCONV,
 * d_u_out holds the step taken with the last polynomial); LX_EINVAL for
 * another operator kind. */
lx_status lx_linear_step(lx_ctx* ctx, const lx_operator* op, const double* d_u,
                         const double* d_src, double* d_u_out, double h,
                         double c, double gamma, const lx_leja_opts* o,
                         int* iters);

/* ---- batches of independent problems ---------------------------------- */

/* One problem of a batch: out = phi_l(h A) v for its own operator and data
 * (Sec. 2.1, Eq. (2); one output per instance). */
typedef struct {
    lx_operator op;         /* grid and operator (prec must be LX_FP64)            */
    const double* d_u;      /* Burgers state, else NULL                             */
    const double* d_v;      /* input vector (device, op.nx*op.ny), not modified     */
    double* d_out;          /* output vector (device), distinct from d_v            */
    const double* d_x0;     /* power-iteration start vector, or NULL: the library's
                               splitmix64 vector seeded by the instance index        */
    int l;                  /* phi order 0..8                                       */
    double h;               /* step > 0                                             */
    double c, gamma;        /* shift and scale when the batch runs no power
                               iteration (c <= 0, gamma > 0); ignored otherwise       */
    int budget;             /* most sweeps for this instance, 1..max_iters;
                               0 = the batch's max_iters                             */
} lx_instance;

typedef struct {
    int status;             /* LX_OK, LX_ENOTCONV (budget reached), LX_ENONFINITE   */
    int iters;              /* sweeps until the stop rule passed                    */
    double err;             /* last error estimate                                  */
    double pnorm;           /* rms norm of the output                               */
    double rho_hat;         /* power-iteration estimate (0 when none ran)           */
    double c, gamma;        /* shift and scale that were used                       */
    int fallback;           /* lx_phi_leja_learned: solved again by the plain method */
} lx_instance_result;

/* Computes every instance of a batch with one launch per window of
 * iterations (or per one or two iterations) for the whole batch: all
 * instances advance together, each with its own stop decision and budget
 * (Sec. 2.2), and finished instances cost nothing more.  Launch shape: the
 * one lx_tune_batched or lx_set_batch_shape chose for the batch's class,
 * else windows of four when every side allows them (8-row tiles with a
 * Burgers instance, 16 otherwise; 16384 points per workgroup), else two
 * iterations per launch, else one.  The device pipeline (power iteration,
 * coefficients, windows) of a layout is captured in a hipGraph after its
 * first call and replayed by later calls with the same layout (the same
 * instance count, sizes, shape and workspaces), with as many window
 * launches as the last call needed; a replay that needs more goes on with
 * launches from the host, one look at the device per chunk
 * (lx_set_batch_graphs; not with timing on).  With
 * power_iters > 0, each instance's spectral bound first comes from
 * power_iters power-iteration sweeps, and c, gamma follow from safety as in
 * lx_spectrum (Listing 7); otherwise the instances' c and gamma are used.
 * The Newton coefficients are computed on the device.  Instances may have
 * different sizes, operators, data, orders and steps; the caller owns all
 * vectors.  n: 1..65536 instances.  res: host array of n results.
 * Returns LX_OK when every instance converged, LX_ENOTCONV when at least
 * one reached its budget (its output holds the last polynomial),
 * LX_ENONFINITE when one became non-finite; LX_EINVAL for a bad argument
 * (naming the instance), LX_ENOMEM when workspaces cannot grow. */
lx_status lx_phi_leja_batched(lx_ctx* ctx, int n, const lx_instance* inst, int power_iters, double safety,
                              const lx_leja_opts* o, lx_instance_result* res);

/* The autotuner of batch launch shapes (not in the paper).  Runs the batch
 * itself (every instance's d_out is written) 1 + repeats times under each
 * candidate: windows of four, two and one iterations per launch x tile rows
 * 8, 16 (windows with a Burgers instance: 8) x 4096, 8192, 16384, 32768
 * points per workgroup; keeps the shape with the lowest median wall time
 * for the batch's class (whether any instance is a Burgers Jacobian, and
 * the set of distinct grid sides) in the context, appended to the file
 * LX_TUNE_CACHE names when set.  report: host text, or NULL: one line per
 * candidate, "depth th points_per_workgroup median_ms".  repeats: 1..50.
 * Errors as lx_phi_leja_batched (the shape is then not kept). */
lx_status lx_tune_batched(lx_ctx* ctx, int n, const lx_instance* inst, int power_iters, double safety,
                          const lx_leja_opts* o, int repeats, char* report, size_t report_len);

/* Sets the launch shape of the class of this batch (see lx_tune_batched):
 * depth 0 (the default rule), 1, 2 or 4; th 0 (default), 8 or 16; ppw 0
 * (default) or the points per workgroup, at most 2^22.  All three 0
 * forgets the class's shape.  Sides too short for windows, odd sides or
 * unaligned vectors still take fewer iterations per launch; windows with a
 * Burgers instance still take 8-row tiles.  Errors: LX_EINVAL. */
lx_status lx_set_batch_shape(lx_ctx* ctx, int n, const lx_instance* inst, int depth, int th, int ppw);

/* Capture and replay of batch pipelines (lx_phi_leja_batched): on = 1 (the
 * default) or 0, which also frees the captured graphs. */
lx_status lx_set_batch_graphs(lx_ctx* ctx, int on);

/* ---- learned spectral bound and sweep budget ------------------------- */

/* A small MLP (8 -> 64 -> 64 -> 2, ReLU, float32 weights, bfloat16 hidden
 * activations) predicting, from 8 features of an instance, the scaled
 * spectral bound log(safety * rho_hat) and the sweep count log(iters) of the
 * plain method.  Trained on records the plain method produces (power
 * iteration and batched Leja runs); a prediction is accepted only when the
 * Leja loop converges within the predicted budget, and power iteration is
 * the fallback.  The paper has no learned component.
 * Features (lx_instance_features): log D, log(|v| + 1e-3), atan2(vy, vx),
 * log dx, log h, log rms(u), log max|u|, l, where u is the input vector of a
 * diffusion-advection instance and the state of a Burgers instance, for
 * which D := nu, |v| := sqrt(2) max|u| and the angle is pi/4.
 * State vector (get/set/save/load): parameters W1[64][8], b1[64],
 * W2[64][64], b2[64], W3[2][64], b3[2], then the Adam moments m and v in
 * the same layout, the standardisation (mean_x[8], std_x[8], mean_y[2],
 * std_y[2]) and the Adam step count: LX_MLP_STATE floats. */
#define LX_MLP_PARAMS 4866
#define LX_MLP_STATE (3 * LX_MLP_PARAMS + 21)

typedef struct lx_predictor lx_predictor;

/* Creates a predictor on the context's device and stream: He-uniform weights
 * from a splitmix64 stream of the given seed, zero biases and moments,
 * identity standardisation. */
lx_status lx_predictor_create(lx_ctx* ctx, unsigned long long seed, lx_predictor** out);
/* Frees a predictor; call it before lx_destroy of its context, or not at
 * all (lx_destroy frees the context's remaining predictors). */
void lx_predictor_destroy(lx_predictor* p);
int lx_predictor_state_size(void);

/* Input and target standardisation, x_std = (x - mean)/std (host arrays of
 * 8, 8, 2, 2 floats; std > 0). */
lx_status lx_predictor_set_scaling(lx_predictor* p, const float* mean_x, const float* std_x,
                                   const float* mean_y, const float* std_y);

/* Host copies of the whole state, and the same as a binary file (an 8-byte
 * tag, the float count, the floats): checkpoint and resume. */
lx_status lx_predictor_get_state(const lx_predictor* p, float* state);
lx_status lx_predictor_set_state(lx_predictor* p, const float* state);
lx_status lx_predictor_save(const lx_predictor* p, const char* path);
lx_status lx_predictor_load(lx_predictor* p, const char* path);

/* Mean squared error over n samples and both outputs of the standardised
 * targets, and its gradient (host, LX_MLP_PARAMS floats; NULL to skip).
 * d_x: device [n][8] raw features, d_y: device [n][2] raw targets. */
lx_status lx_predictor_gradient(lx_predictor* p, const float* d_x, const float* d_y, int n, float* grad,
                                double* loss);

/* steps Adam steps (learning rate lr, beta 0.9/0.999, eps 1e-8) on
 * minibatches of `batch` samples: the host array order (steps * batch
 * indices) when given, else epochs of a splitmix64-driven shuffle of seed.
 * final_loss: the last minibatch's loss (host, may be NULL). */
lx_status lx_predictor_train(lx_predictor* p, const float* d_x, const float* d_y, int n, int steps, int batch,
                             float lr, unsigned long long seed, const int* order, double* final_loss);

/* d_y[n][2] = raw predictions for the raw features d_x[n][8] (device),
 * enqueued on the context's stream. */
lx_status lx_predictor_infer(lx_predictor* p, const float* d_x, int n, float* d_y);

/* The 8 features of each instance into d_x[n][8] (device), enqueued on the
 * context's stream. */
lx_status lx_instance_features(lx_ctx* ctx, int n, const lx_instance* inst, float* d_x);

/* The learned form of lx_phi_leja_batched.  The predictor maps each
 * instance's features to (a, b) ~ (log(safety * rho_hat), log(sweeps)); the
 * instance then runs without power iteration, with lambda = -exp(a +
 * margin_log_rho), c = lambda/2, gamma = -lambda/4 and a budget of
 * ceil(exp(b + margin_log_sweeps)) + 1 sweeps (at most o->max_iters; the
 * instance's own c, gamma and budget fields are ignored).  The prediction
 * is accepted when the Leja loop converges within that budget; every other
 * instance (and any with a non-finite prediction) is solved again by the
 * plain method: power_iters (>= 1) power-iteration sweeps with the given
 * safety factor, then the loop with o->max_iters.  res[i].fallback says
 * which; res[i].rho_hat is 0 for accepted instances.  The predictor must
 * belong to ctx.  fallbacks (host, may be NULL) receives their number.
 * Statuses as for lx_phi_leja_batched, after the fallback. */
lx_status lx_phi_leja_learned(lx_ctx* ctx, lx_predictor* p, int n, const lx_instance* inst, double margin_log_rho,
                              double margin_log_sweeps, int power_iters, double safety, const lx_leja_opts* o,
                              lx_instance_result* res, int* fallbacks);

/* ---- launch shapes and measurement ------------------------------------ */

/* Times every candidate launch shape of the Leja loop for this operator,
 * grid, output count K and precision on the context's stream (about
 * `sweeps` timed iterations per candidate, after two warm-up launches, on
 * scratch vectors the call allocates and frees): the one-sweep shapes
 * (tx, ty, ry, vec, workgroups) and, for FP64 with even nx, the shapes of
 * two iterations per launch and (diffusion-advection operators) of windows
 * of three, four and six (tile rows th, workgroups).  It keeps the fastest
 * one-sweep shape (used by the one-sweep power iteration, the right-hand
 * side of lx_linear_step and depth-1 loops) and the fastest multi-iteration
 * shape with its depth, and of the two the one with the lower time per
 * iteration: later calls with the same (kind, nx, ny, K, prec) use them
 * (the window kernel needs a second buffer per output, which this call
 * allocates and keeps in the context).  When the
 * environment variable LX_TUNE_CACHE names a file, the winners are
 * appended to it as one JSON object per line, and lx_create loads the
 * file's entries.
 * report: host buffer of report_len chars, or NULL; receives one line per
 * candidate: "depth tx ty rows vec workgroups microseconds_per_iteration",
 * rows being ry for depth 1, th for LDS-tile depths 2..6 (whose workgroups
 * are 64 x 4) and the number of bands for register-marching windows, which
 * report depth as 100 + D.
 * Errors: LX_EINVAL (op invalid, K out of range, sweeps outside 1..200),
 * LX_ENOMEM. */
lx_status lx_tune(lx_ctx* ctx, const lx_operator* op, int K, int sweeps, char* report, size_t report_len);

/* Forces the launch shape of later sweeps: tx lanes along x times ty
 * thread-rows (tx * ty = 256), each lane owning vec (1 or 2) columns and
 * marching ry (1, 2, 4 or 8) rows; nb workgroups loop over the tiles
 * (0 = one workgroup per tile).  tx = 0 restores the automatic choice
 * (tuned entry, else the built-in rule).  vec = 2 needs an even nx and
 * 16-byte aligned vectors; otherwise vec 1 is used. */
lx_status lx_set_tile(lx_ctx* ctx, int tx, int ty, int ry, int vec, int nb);

/* Leja iterations per launch of later lx_phi_leja / lx_exprb_step loops:
 * depth 1 runs one fused sweep per launch (the shape of lx_set_tile);
 * depth 2 runs two iterations per launch on LDS-resident tiles of 128
 * columns by th (8, 16 or 32) rows with nb workgroups (0 = automatic),
 * reading the basis once per two iterations; depths 3, 4, 6 and 8 run
 * windows of that many iterations whose terms are added speculatively, and
 * re-execute a window in which an output stopped (they also use one more
 * buffer per output, allocated on first use).  Windows run either on LDS
 * tiles (th 8 or 16; larger th is taken as 16; depths 3, 4, 6) or by
 * register marching (lx_set_window_kernel; depths 4, 6, 8); depth 0
 * restores the automatic choice (the tuned entry, else 2).
 * Depths 2..8 apply to grids with even nx and 16-byte aligned vectors; on
 * LDS tiles (FP64 sweeps) 3 and 4 to the diffusion-advection operators and
 * the Burgers Jacobian, 6 to LX_OP_DIFFADV2D (others fall back to 4, then
 * 2), each with sides of at least depth times the stencil radius; register
 * marching to LX_OP_DIFFADV2D (FP64: depth 4 for K <= 4, 6 and 8 for
 * K <= 3) and LX_OP_BURGERS2D (depth 4 for K <= 2, 6 for K = 1), and to
 * FP32 sweeps of both for K <= 2 at depth 4 and K = 1 at 6 (windows switch
 * to FP32 levels on the device); depth 8 otherwise falls back to 6; other
 * calls use depth 1 (FP32 sweeps: one per launch).
 * Results agree with depth 1 to rounding (the outputs take the same terms
 * in the same order; only the order of the norm reductions differs).
 * Errors: LX_EINVAL (depth not 0..4, 6 or 8, th not 0, 8, 16 or 32, nb < 0). */
lx_status lx_set_depth(lx_ctx* ctx, int depth, int th, int nb);

/* Which kernel later windows (depth >= 3) and power iterations run on:
 * kind 0 = automatic (windows as the tuned entry says, else LDS tiles;
 * power iteration by register marching where it applies), 1 = LDS tiles
 * for both (leja_block, power_block), 2 = register marching where it
 * applies (leja_stream: the five-point operators, FP64 or FP32 sweeps, at
 * the depths lx_set_depth lists; power_stream: LX_OP_DIFFADV2D; even nx,
 * sides >= depth, 16-byte aligned vectors of at most 2^30 bytes).
 * Register marching gives every wavefront a strip of 128 columns (its
 * output columns and depth columns on each side) and a band of rows, which
 * it walks from top to bottom forming all levels of the window in
 * registers; for LX_OP_DIFFADV2D at depths 4, 6 and 8 every level also passes
 * through a small ring in LDS, from which each output row takes its terms
 * depth rows later.  bands: bands of rows (0 = one resident round of wavefronts);
 * nb: workgroups of four wavefronts (0 = automatic).  Results are the same
 * as with LDS tiles up to the order of the norm reductions.
 * Errors: LX_EINVAL (kind not 0..2, bands < 0, nb < 0). */
lx_status lx_set_window_kernel(lx_ctx* ctx, int kind, int bands, int nb);

/* Practical HBM bandwidth of plain streaming HIP kernels, the calibration
 * of Sec. 3: kind 0 copies y = x (16 bytes per element), kind 1 computes
 * z = a x + b y (24 bytes per element).  n FP64 elements (even, >= 2),
 * reps timed repetitions after one warm-up, on vectors the call allocates
 * and frees.  gbs: host output, bytes moved / time in GB/s. */
lx_status lx_bandwidth_probe(lx_ctx* ctx, int kind, size_t n, int reps, double* gbs);

/* ---- host-only planner (no device needed) ------------------------------ */

/* First M (1 .. LX_MAX_ITERS+1) Leja points of [-2, 2] (Sec. 2.1): xi_0 = 2,
 * each next point maximises the product of distances to the earlier ones,
 * exact ties to the larger point.  xi: host array of M doubles. */
lx_status lx_leja_points(int M, double* xi);

/* phi_l(z) for real z (Sec. 1), FP64. */
double lx_phi_scalar(int l, double z);

/* Newton coefficients d_0..d_{M-1} (divided differences) of
 * f(xi) = sigma * phi_l(alpha * h * (c + gamma * xi)) at the first M Leja
 * points, as the device loop uses them.  d: host array of M doubles. */
lx_status lx_newton_coeffs(int l, double alpha, double sigma, double h,
                           double c, double gamma, int M, double* d);

#ifdef __cplusplus
}
#endif

#endif /* LX_H */
