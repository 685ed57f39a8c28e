/*
 * ader.h -- C ABI of the ADER-DG hot path on MI355X (gfx950).
 *
 * The library advances hyperbolic systems
 *     Q_t + div F(Q) + B(Q).grad Q = S(Q)                      (Sec. 2, eq. pde)
 * on periodic Cartesian meshes with the unlimited ADER-DG scheme of Dumbser,
 * Fambri, Tavelli, Bader and Weinzierl (2018): a nodal tensor basis on the
 * N+1 Gauss-Legendre points of [0,1] (Sec. 2.1, eq. ansatz.uh), the
 * element-local space-time predictor solved by Picard iteration (Sec. 2.2,
 * eqs. spacetime and pde.st2) and the one-step corrector with the
 * path-conservative Rusanov jump term (Sec. 2.1, eqs. pde.nc.gw2, pc.scheme,
 * rusanov).  Two systems are built in: the compressible Euler equations
 * (Sec. 3.1, eq. euler) and linear elasticity in velocity-stress form
 * (Sec. 3.2, eqs. 3.00-3.1 with volume fraction 1).
 *
 * Conventions
 *   - Every call returns ader_status; nothing throws across the ABI.
 *   - All state pointers (u, dt_dev, qhat_out) are DEVICE pointers on the
 *     device that was current at ader_create; host pointers are named *_host.
 *   - A context is bound to one HIP stream and is not thread-safe.  Calls
 *     enqueue work on that stream and return without synchronising, except
 *     where a host output is requested (they then synchronise the stream).
 *   - Errors are reported synchronously for argument checks
 *     (ADER_ERR_INVALID / ADER_ERR_UNSUPPORTED).  Non-finite or non-physical
 *     states (NaN/Inf, density <= 0, pressure <= 0) are detected on the
 *     device by the time-step reduction; asynchronous calls latch the flag and
 *     the next synchronising call returns ADER_ERR_NONFINITE (and clears it).
 *     While the flag is raised every problem of the context takes a step
 *     of size 0 (its state and time stay as they are).
 *   - ader_last_error(ctx) returns a message for the last failing call.
 *
 * State layout (caller-owned, FP64, one contiguous device buffer holding all
 * problems, each at the offset returned by ader_layout):
 *     u[e][v][k],  e = ix + nx*(iy + ny*iz),  k = k1 + n*(k2 + n*k3),  n = N+1
 *   node k of element e sits at x_a = lo_a + (i_a + xi_{k_a}) * h_a with xi
 *   the Gauss-Legendre points of [0,1] and h_a = (hi_a - lo_a)/nelem_a.
 *   Variables: Euler (rho, rho*v_1..rho*v_d, rho*E); elasticity
 *   (v_x, v_y, v_z, s_xx, s_yy, s_zz, s_xy, s_yz, s_xz).
 */
#ifndef ADER_H
#define ADER_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ader_ctx ader_ctx; /* opaque; owns every scratch buffer */

typedef enum {
  ADER_OK = 0,
  ADER_ERR_INVALID = 1,     /* bad argument: NULL pointer, size, dimension, ... */
  ADER_ERR_UNSUPPORTED = 2, /* valid but not built: degree > 7, LDS too small, ... */
  ADER_ERR_OOM = 3,         /* device allocation failed */
  ADER_ERR_DEVICE = 4,      /* a HIP call failed */
  ADER_ERR_NONFINITE = 5    /* NaN/Inf or non-physical state met on the device */
} ader_status;

typedef enum { ADER_EULER = 0, ADER_ELASTIC = 1 } ader_pde;

/* Arithmetic of the predictor's Picard sweeps.  ADER_FP64: every sweep in
 * FP64.  ADER_FP32: sweeps 1..P-1 in FP32 with FP32 accumulation, the last
 * sweep in FP64; the FP32 operator contractions run either on the matrix
 * cores (v_mfma_f32_4x4x1, rows in groups of four, the rest on VALU) or as
 * VALU FMAs, whichever the timing at ader_create finds faster for the
 * configuration (ader_describe names the variant in use: fp32-mfma-* or
 * fp32-valu-*).  ADER_BF16: like FP32 but the inputs of the spatial
 * contractions (flux, or q for elasticity) are rounded to bfloat16; they run
 * as VALU FMAs with the FP32 operator (bf16-valu-*) or on the matrix cores
 * (bf16-mfma-*: v_mfma_f32_4x4x4bf16_1k, the operator split into two
 * bfloat16 parts), again chosen by timing; FP32 accumulation and FP32 time
 * contraction.  The corrector's update u^{n+1} = u^n + dt*R, the
 * time-step reduction and the conservation sums are FP64 in every mode. */
typedef enum { ADER_FP64 = 0, ADER_FP32 = 1, ADER_BF16 = 2 } ader_prec;

typedef struct {
  int32_t dim;          /* 2 or 3 (elasticity: 3) */
  int32_t degree;       /* N in [0,7].  The space-time DOFs of one element must
                           fit one CU's LDS (160 KB): 2-D Euler every N; 3-D
                           Euler N <= 7 in FP64 (N >= 6 with the accumulator in
                           HBM) and N <= 6 in FP32/BF16; elasticity N <= 5 (N = 5
                           FP64 by row groups).  Other
                           combinations: ADER_ERR_UNSUPPORTED at create. */
  int32_t nelem[3];     /* elements per axis, 1..65535 (nelem[2] ignored for
                           dim = 2) */
  double lo[3], hi[3];  /* box; periodic in every axis */
  int32_t pde;          /* ader_pde */
  double gamma;         /* Euler: ratio of specific heats (> 1) */
  const double *material; /* ELASTIC: HOST array [E][3] = (rho, lambda, mu),
                             copied at create; ignored for Euler */
  int32_t prec;         /* ader_prec */
  int32_t picard_iters; /* Picard sweeps P; 0 -> max(1, N+1-guess), 1 for guess 3 */
  double cfl;           /* dt = cfl * alpha_N / max_e sum_d lambda_d / h_d,  0 < cfl <= 1 */
  int32_t guess;        /* initial guess of the Picard iteration (Sec. 2.2), a Taylor
                           polynomial in t - t^n at the time nodes: 0 q0 = u (constant);
                           1 q0 = u + (t-t^n) L(u) (MUSCL-Hancock type, second order);
                           2 q0 = u + (t-t^n) k1 + (t-t^n)^2 (k2-k1)/(2 dt), k1 = L(u),
                           k2 = L(u + dt k1) (third order); L = S - div F - B.grad;
                           3 extrapolation of the previous interval: the predictor of the
                           step before (degree N in time), continued to the new time nodes
                           and shifted to start at the corrected state,
                           q0 = u + q_prev(t) - q_prev(t^n), with one sweep by default (a
                           guess of degree >= N-1 in time needs a single sweep).  The context
                           keeps N Taylor coefficients per node and variable of the last
                           predictor (8 or 4 bytes each); a step without them (the first, one
                           on another buffer than the last step wrote, or after a step of
                           size 0) is the plain scheme: constant guess, N+1 sweeps.
                           Guesses 1 to 3 are computed in the sweeps' precision. */
  int32_t face_avg;     /* 0: the jump term at every face node and time node, integrated in
                           time (eqs. pc.scheme, rusanov); 1: from time-averaged traces,
                           qbar = sum w_l q(l) and (Euler) Fbar = sum w_l F(q(l)), q(l) the
                           face trace at time node l:
                           G = 1/2 (Fbar+ + Fbar-).n + 1/2 (path - s_max)(qbar+ - qbar-),
                           s_max from the averaged states.  Exact for elasticity (linear,
                           time-independent coefficients); for Euler only the Rusanov speed
                           changes.  Stores 2m (Euler) or m (elasticity) values per face node
                           and side instead of (N+1) m. */
} ader_problem;

/* Create a context for `nprob` independent problems (Sec. 2; the problems
 * share nothing but the stream).  `hip_stream` is a hipStream_t (NULL = the
 * default stream).  Device memory for traces, face integrals and the
 * predictor's output is allocated here and owned by the context.  The
 * simulation time of every problem starts at 0.  Problems of equal
 * dimension, degree, PDE and precision form one kernel class: every stage
 * of a step is one launch per class over the elements of all its problems
 * (persistent workgroups walking per-problem tile ranges held in device
 * memory), so the launch count of a step does not grow with nprob. */
ader_status ader_create(const ader_problem *probs, int32_t nprob, void *hip_stream,
                        ader_ctx **out);
/* Free everything the context owns.  NULL is accepted. */
ader_status ader_destroy(ader_ctx *ctx);

/* Offset and length (in doubles) of problem `prob` inside the state buffer;
 * the buffer must hold at least offset+count doubles for every problem. */
ader_status ader_layout(const ader_ctx *ctx, int32_t prob, int64_t *offset, int64_t *count);
/* Total number of doubles of the state buffer. */
ader_status ader_state_size(const ader_ctx *ctx, int64_t *count);

/* Time step of every problem from the state u (Sec. 3, CFL condition):
 *   dt_p = cfl * alpha_N / max_e sum_a (max_{k in e} |lambda_a(u_k)|) / h_a,
 * with |lambda_a| = |v_a| + c for Euler and the P-wave speed for elasticity;
 * alpha_N is the 1-D von Neumann stability limit of the scheme (below the
 * paper's bound 1/(2N+1)).  The result stays on the device and is the step
 * used by a following ader_predictor/ader_corrector with dt_dev = NULL.  If
 * dt_host (host, [nprob]) is not NULL the call synchronises and copies it. */
ader_status ader_cfl_dt(ader_ctx *ctx, const double *u, double *dt_host);

/* Space-time predictor of every element (Sec. 2.2, eq. pde.st2): Picard
 * iteration q <- u + dt*T*R(q) from q = u, R the collocated right-hand side
 * S - div F - B.grad q.  Also evaluates the predictor's volume integrals and
 * the boundary-extrapolated traces on all faces into context scratch.
 *   u        device [state], read only
 *   dt_dev   device [nprob] step sizes, or NULL for the context's step
 *   qhat_out device [E][m][N+1][(N+1)^d] per problem at the same offsets
 *            scaled by (N+1) (debug / test output), or NULL. */
ader_status ader_predictor(ader_ctx *ctx, const double *u, const double *dt_dev,
                           double *qhat_out);
/* Offset (in doubles) of problem `prob` inside a qhat_out buffer, and its size. */
ader_status ader_qhat_layout(const ader_ctx *ctx, int32_t prob, int64_t *offset, int64_t *count);

/* Corrector (Sec. 2.1, eq. pde.nc.gw2) with the last predictor's output:
 * face integrals of the path-conservative Rusanov jump term (eqs. pc.scheme,
 * rusanov) at every face node and time node, then the FP64 update
 *   u <- u + dt * (V - lifted face terms) / (diagonal mass).
 * dt_dev must equal the one given to ader_predictor (NULL = context's). */
ader_status ader_corrector(ader_ctx *ctx, double *u, const double *dt_dev);

/* One full step of every problem: time step (clipped so that the step ends
 * exactly at t_end_host[p]; a problem already at t_end takes dt = 0),
 * predictor, corrector, time advance.  Host-synchronisation free, so it can
 * be captured into a hipGraph (the captured t_end values are then fixed).
 * The update of a step also takes the wave-speed maxima of the state it
 * writes (the quantity of ader_cfl_dt), and the next ader_step / ader_run on
 * the same buffer takes its dt from them instead of reading u again; the
 * result is the same bit for bit.  Any other call on the context that
 * touches the state (ader_cfl_dt, ader_predictor, ader_corrector,
 * ader_set_detection) discards those maxima.  A caller that changes u
 * outside the library between two steps on the same buffer must call
 * ader_cfl_dt(ctx, u, NULL) before the next step.  With detection on, every
 * step reads u with the time-step kernel. */
ader_status ader_step(ader_ctx *ctx, double *u, const double *t_end_host);

/* nsteps consecutive ader_step calls replayed as one HIP graph.  The graph
 * is captured on the first call (and again when u or nsteps change) on a
 * stream of the context's own, ordered after earlier work on the context
 * stream; later work on that stream waits for the replay.  Results are
 * bitwise those of nsteps ader_step calls.  Stage profiling does not apply
 * to replays.  nsteps >= 1, else ADER_ERR_INVALID.  Changing t_end_host
 * between calls costs one synchronous copy. */
ader_status ader_run(ader_ctx *ctx, double *u, const double *t_end_host, int32_t nsteps);

/* A posteriori detection of troubled elements (Sec. 2.3: the criteria that
 * mark cells for the subcell limiter; the limiter itself is not part of
 * this library).  With enable != 0 every following ader_step / ader_run
 * step also records, per element, the extremes of each variable of the
 * state it starts from (in the time-step kernel) and, after the update,
 * checks the new state: bit 1 a value is NaN or infinite; bit 2 (Euler)
 * rho <= 0 or p <= 0 at a node; bit 4 the relaxed discrete maximum
 * principle fails: for some variable a nodal value lies outside
 * [m - delta, M + delta], m and M the extremes of the previous state over
 * the element and the 3^d elements sharing a vertex with it (periodic),
 * delta = max(1e-4, 1e-3 (M - m)).  Allocates 4 bytes per element and
 * 16 m bytes per element at the first enable; switching drops a captured
 * ader_run graph.  The detection time is counted in the update stage of
 * ader_stage_times.  If enabling fails (ADER_ERR_OOM, ADER_ERR_DEVICE),
 * detection stays off; buffers already allocated are kept for a later call. */
ader_status ader_set_detection(ader_ctx *ctx, int32_t enable);
/* Flags of the last detected step, host int32 [sum over problems of E],
 * problems in order, elements e = ix + nx (iy + ny iz) within a problem;
 * synchronises.  ADER_ERR_INVALID if detection was never enabled. */
ader_status ader_detect_flags(ader_ctx *ctx, int32_t *flags_host);

/* Current simulation time of every problem (host [nprob]); synchronises and
 * reports a latched ADER_ERR_NONFINITE. */
ader_status ader_time(ader_ctx *ctx, double *t_host);
/* Overwrite the simulation times (host [nprob]), e.g. to resume a run. */
ader_status ader_set_time(ader_ctx *ctx, const double *t_host);
/* Step sizes of the last ader_cfl_dt/ader_step (host [nprob]); synchronises. */
ader_status ader_last_dt(ader_ctx *ctx, double *dt_host);

/* Domain integral of every variable, sum_e |Omega_e| sum_k w_k u (FP64,
 * deterministic order), into host [sum over problems of m]; synchronises. */
ader_status ader_totals(ader_ctx *ctx, const double *u, double *sums_host);

/* ader_totals without a context and without any allocation, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  The same domain
 * integrals as ader_totals, bit for bit (same kernels and grid), of ONE
 * problem whose state u (device, [E][m][(N+1)^d], the layout of ader_layout
 * for a single-problem context) is described by *prob (validated as in
 * ader_create), written to sums_dev (device, m doubles, caller-owned)
 * asynchronously on the HIP stream hip_stream (NULL = default stream); the
 * call does not synchronise.  The per-block partial sums live in a static
 * device array of the library of 512 x 9 doubles (36 KB), held by every GPU
 * the library runs on until the process ends; every problem size fits it
 * (at most 9 variables; more would be ADER_ERR_UNSUPPORTED).  All calls on
 * one GPU share that array: calls that overlap on one GPU (on different
 * streams or threads) race and must be ordered by the caller.  Errors:
 * ADER_ERR_INVALID (NULL pointers, a bad problem), ADER_ERR_DEVICE (a HIP
 * call failed); the message is ader_last_error(NULL). */
ader_status ader_totals_noalloc(const ader_problem *prob, const double *u, double *sums_dev, void *hip_stream);

/* Per-stage device timing of ader_step.  With enable != 0 the context
 * records HIP events on its own stream at the boundaries of the four stages
 * of every following ader_step: 0 time-step reduction, 1 predictor, 2 face
 * integrals, 3 update.  ader_stage_times synchronises and returns, per stage,
 * the summed elapsed milliseconds (host [4]) and the number of recorded
 * steps (host [4], may be NULL), then clears the record.  Timing adds one
 * event record per stage boundary; it is off by default. */
ader_status ader_profile(ader_ctx *ctx, int32_t enable);
ader_status ader_stage_times(ader_ctx *ctx, double *ms_host, int64_t *launches_host);

/* Human-readable description of the kernels chosen for problem `prob`
 * (predictor variant, workgroup size, LDS bytes, how it was selected), as
 * a NUL-terminated string of at most len bytes in the host buffer buf.
 * The predictor variant is picked at ader_create: the implementations of
 * the problem's precision that fit the LDS budget (VALU or MFMA
 * contractions, two workgroup sizes; for elasticity also the variants with
 * two threads per line, one per row group of the right-hand side) are
 * timed on a uniform state of up to 32768 elements and the fastest is
 * kept, cached per configuration for the process.  Environment:
 * ADER_AUTOTUNE=0 keeps the first candidate; ADER_VARIANT=<name> forces one
 * (names as printed here). */
ader_status ader_describe(const ader_ctx *ctx, int32_t prob, char *buf, int32_t len);

/* Message of the last failing call on this context (never NULL); with
 * ctx = NULL, the message of the last failed ader_create on this thread. */
const char *ader_last_error(const ader_ctx *ctx);

/* Host-side queries (no device needed). */
/* alpha_N of the CFL rule for degree N (see ader_cfl_dt). */
ader_status ader_stability_alpha(int32_t degree, double *alpha);
/* The 1-D tables of degree N: Gauss-Legendre points and weights on [0,1]
 * (n each), derivative matrix Dhat[k][j] = phi_j'(xi_k) and the predictor's
 * time operator T (n*n each, row-major).  Any output may be NULL. */
ader_status ader_basis(int32_t degree, double *xi, double *w, double *dhat, double *tmat);
/* Library version string. */
const char *ader_version(void);

#ifdef __cplusplus
}
#endif
#endif
