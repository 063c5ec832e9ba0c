/*
 * pint.h -- C ABI of the MI355X (gfx950) all-at-once space-time solver for
 * the fourth-order problems of Garai & Mandal, "Diagonalization based
 * parallel-in-time method for a class of fourth order time dependent PDEs"
 * (arXiv:2304.14021).
 *
 * Problems (homogeneous Neumann conditions, unit interval or unit square):
 *   biharmonic heat   u_t = -Lap^2 u                          (Section 2, eq. modelproblem1a)
 *   linearized CH     u_t = -beta^2 Lap u - eps^2 Lap^2 u      (Section 3, eq. modelproblem2a)
 *   nonlinear CH      u_t = Lap(u^3 - u) - eps^2 Lap^2 u       (Section 4, eq. modelproblem3)
 * discretized by the cell-centred Neumann Laplacian (N cells, h = L/N,
 * x_j = (j + 1/2) h) and the theta-method / backward Euler / Eyre splitting in
 * time (eqs. linear-theta1, fully-dis_CH, fully-dis_CH_WR_Eyre).
 *
 * The solve is the paper's waveform-relaxation / quasi-Newton iteration with
 * the periodic-like initial condition u(0) = alpha u(T) - alpha u^{k-1}(T) + u0
 * (eqs. modelproblem1a_wr, modelproblem3_wr), written in correction form
 * U <- U + P_alpha^{-1} r(U), where r is the alpha = 0 all-at-once residual
 * evaluated in FP64 and P_alpha is the Strang-type alpha-circulant space-time
 * matrix, inverted by the three steps of eq. pintiter1 / pintiter_CH:
 * time transform (F Gamma_alpha (x) I), N_t independent shifted spatial solves
 * (diagonalized by the 2D DCT-II), inverse time transform.
 *
 * Conventions for every entry point
 *  - All functions return int: PINT_OK (0) or a negative PINT_E* code.  No C++
 *    exception crosses the ABI.  pint_status_string() names a code;
 *    pint_plan_last_error() gives the message of the last failing call on a
 *    plan, pint_last_error() that of the last failing call on this thread.
 *  - "d_" pointers are device memory on the current HIP device, owned by the
 *    caller, never freed by the library.  "h_" pointers are host memory.
 *  - Space-time arrays are FP64, layout [N_t][N_y][N_x] row-major (x fastest),
 *    holding u_1 .. u_{N_t}; the datum u_0 is a separate [N_y][N_x] array.
 *    In 1D, N_y = 1.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls enqueue work on it and return; pint_solve() synchronizes with the
 *    stream to read its convergence control (see there).
 *  - A plan may be used by one host thread at a time.  Calls on different
 *    plans are independent.
 *  - Sizes: N (cells per dimension) a power of two in [8, 512]; N_t a power of
 *    two in [4, 1024].  Other sizes return PINT_EINVAL.
 */
#ifndef PINT_H
#define PINT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
#define PINT_OK            0
#define PINT_EINVAL       (-1)  /* invalid argument or unsupported size       */
#define PINT_ENOCONV      (-2)  /* max_iter reached before the stop rule held  */
#define PINT_EDIVERGED    (-3)  /* NaN/Inf or growing updates detected         */
#define PINT_ENOMEM       (-4)  /* workspace/pool too small                    */
#define PINT_EHIP         (-5)  /* a HIP runtime call failed                   */
#define PINT_ETIMEDOUT    (-6)  /* server wait timed out                       */
#define PINT_ECANCELED    (-7)  /* server request cancelled                    */
#define PINT_ENOTFOUND    (-8)  /* unknown server ticket                       */

/* ------------------------------------------------------------- operators */
#define PINT_OP_BIHARMONIC 0    /* A = Lap_h^2                                 */
#define PINT_OP_LINEAR_CH  1    /* A = beta^2 Lap_h + eps^2 Lap_h^2            */
#define PINT_OP_CH         2    /* nonlinear CH, fully implicit BE (PinT-I)    */
#define PINT_OP_CH_EYRE    3    /* nonlinear CH, Eyre splitting (PinT-II)      */

/* ------------------------------------------------------------- precision */
#define PINT_PREC_FP64          0  /* every stage in FP64                      */
#define PINT_PREC_FP32_REFINE   1  /* transforms/divide FP32, residual+update FP64 */
#define PINT_PREC_FP32_NOREFINE 2  /* residual and update in FP32 too          */
#define PINT_PREC_BF16_REFINE   3  /* dense time contraction with BF16 operands,
                                      FP32 accumulate (time path AUTO or DENSE);
                                      forward spatial DCT FP64 as for MIXED,
                                      inverse FP32; residual+update FP64      */
#define PINT_PREC_BF16_NOREFINE 5  /* the unrefined FP32 loop of FP32_NOREFINE
                                      with the BF16 dense time contraction (time
                                      path AUTO or DENSE); stops on its plateau */
#define PINT_PREC_MIXED         4  /* forward spatial DCT in FP64 (its rounding
                                      would be amplified by the stiffness ratio
                                      of the shifted spatial solves), time solve
                                      and inverse DCT in FP32; residual+update
                                      FP64                                     */

/* ------------------------------------------------------------- time path */
#define PINT_TIME_AUTO  0          /* FFT over time (alpha-circulant); the
                                      dense path for PINT_PREC_BF16_REFINE    */
#define PINT_TIME_FFT   1          /* batched FFT over the time index          */
#define PINT_TIME_DENSE 2          /* dense contraction over the time index on
                                      the matrix cores: FP32 MFMA for
                                      FP32_REFINE / MIXED, BF16 MFMA for
                                      BF16_REFINE; FP32 accumulation.  Needs
                                      N_t >= 32 and N_s a multiple of
                                      max(32, 4096 / N_t); not for FP64       */

/* ----------------------------------------------------------------- flags */
#define PINT_FLAG_INIT_BROADCAST_U0 0x1u /* fill d_U with u0 before iterating */
#define PINT_FLAG_STAGE_TIMING      0x2u /* fill pint_report.ms_stage (adds syncs) */
#define PINT_FLAG_SOLVE_GRAPH       0x8u /* pint_solve on a non-NULL stream: capture
                                            the init and the predicted iterations
                                            as one HIP graph, replayed by later
                                            solves with the same buffers, stream
                                            and iteration count (ignored with
                                            PINT_FLAG_STAGE_TIMING)            */
#define PINT_FLAG_BF16_SPLIT        0x4u /* PINT_PREC_BF16_REFINE: two-term BF16
                                            split of both operands, three
                                            products (hi*hi + hi*lo + lo*hi) */
#define PINT_FLAG_INVARIANTS       0x10u /* pint_solve: after the last iteration,
                                            fill pint_report.mass_drift and
                                            energy_monotone (one more read of
                                            U and two small kernels)           */
#define PINT_FLAG_FIELD_JACOBIAN   0x20u /* PINT_OP_CH: the quasi-Newton step uses
                                            the averaged Jacobian as Section 4.1
                                            defines it (eq. approx_jacobian),
                                            J~ = diag((1/N_t) sum_n 3 u_n^2),
                                            varying in space, so that Step-(2)
                                            of eq. pintiter_CH is no longer
                                            diagonal in the cosine basis; each
                                            step solves G~'(U) delta = r(U) by
                                            BiCGStab on the space-time vectors,
                                            preconditioned by the scalar-c_bar
                                            solve (inner residual reduced by
                                            1e-3, at most 30 inner iterations;
                                            pint_report.inner_iterations).  The
                                            fixed point is unchanged.  Needs
                                            8 more FP64 space-time vectors of
                                            workspace; synchronizes with the
                                            stream several times per inner
                                            iteration; not with
                                            PINT_FLAG_SOLVE_GRAPH or
                                            PINT_FLAG_STAGE_TIMING             */

#define PINT_HIST 64

/* Statement of one problem (plain data, versioned by struct_size). */
typedef struct pint_problem {
  size_t struct_size;  /* sizeof(pint_problem)                                 */
  int op;              /* PINT_OP_*                                            */
  int dim;             /* 1 or 2                                               */
  int nx, ny;          /* cells per dimension (ny = 1 in 1D; nx == ny in 2D)   */
  int nt;              /* number of unknown time levels; T = nt * dt           */
  double lx, ly;       /* domain lengths (h = lx / nx); 0 means 1.0            */
  double dt;           /* time step > 0                                        */
  double theta;        /* 1 (backward Euler) or 0.5 (trapezoidal); linear ops  */
  double eps;          /* interface parameter epsilon > 0 (ignored: biharmonic)*/
  double beta;         /* linearized CH parameter (ignored unless LINEAR_CH)   */
  double alpha;        /* PinT parameter in (0, 1); 0 = choose automatically   */
  int precision;       /* PINT_PREC_*                                          */
  int time_path;       /* PINT_TIME_*                                          */
  double rtol;         /* target relative error (L^inf(L^2)); 0 = 1e-10        */
  int max_iter;        /* cap on outer iterations (<= PINT_HIST); 0 = 30       */
  unsigned flags;      /* PINT_FLAG_*                                          */
  /* Nonuniform time steps (Section 1, direct diagonalization with variable
   * steps): NULL for the uniform step dt; else nt positive, pairwise distinct
   * steps dt_1..dt_nt (host memory, copied by pint_plan_create; dt is then
   * ignored and T = sum dt_n).  The time-step pencil of the theta-method,
   * B = diag(1/dt_n)(I - S), C = theta I + (1 - theta) S (S the down-shift),
   * is no longer alpha-circulant: the plan diagonalizes it directly,
   * B V = C V D, in FP64 on the GPU (one eigenpair per thread, by forward and
   * backward substitution in the bidiagonal pencil), and the time solve is
   * the dense contraction x -> V (D + shift_k)^{-1} V^{-1} C^{-1} x per spatial
   * mode (FP32 MFMA for FP32_REFINE and MIXED, FP64 for FP64), wrapped in the
   * same FP64 residual refinement.  alpha is not used.  Operators: the linear
   * ones (theta 1 or 1/2) and PINT_OP_CH (backward Euler); time path AUTO or
   * DENSE; precision FP64, FP32_REFINE or MIXED.  N_t >= 32 (the contraction
   * tile), and the time-step pencil's eigenvector matrix V grows
   * ill-conditioned as neighbouring steps approach each other: the refinement
   * then needs more iterations or stops converging (PINT_ENOCONV). */
  const double* dts;
} pint_problem;

/* Outcome of one solve (filled by the library when a pointer is passed). */
typedef struct pint_report {
  size_t struct_size;          /* sizeof(pint_report), set by the caller       */
  int status;                  /* same as the return code of pint_solve         */
  int iterations;              /* outer iterations performed                    */
  double alpha_used;           /* alpha actually used                           */
  double c_bar;                /* final scalar averaged Jacobian (CH ops)        */
  double est_rel_err;          /* error estimate rho/(1-rho) * |dU|/|U|          */
  double res_hist[PINT_HIST];  /* max_n ||r_n||_2 of the iterate entering step k */
  double upd_hist[PINT_HIST];  /* max_n ||delta_n||_2 / max_n ||u_n||_2, step k */
  double ms_stage[8];          /* summed over iterations (FLAG_STAGE_TIMING only):
                                  [0] residual + x-DCT-II, [1] y-DCT-II,
                                  [2] time solve, [3] y-DCT-III,
                                  [4] x-DCT-III + update, [5] control; rest 0  */
  double ms_total;             /* wall time of the solve call (host clock)      */
  /* Invariants of the returned iterate (PINT_FLAG_INVARIANTS; Section 1: the
   * CH flow conserves mass and does not increase the Ginzburg-Landau energy,
   * and the backward-Euler scheme inherits both for small dt):
   *   mass_drift = max_n |M(u_n) - M(u_0)| / (h^d sum_j |u_0,j|),
   *                M(u) = h^d sum_j u_j (NaN when not computed, or when u_0 = 0);
   *   energy_monotone = 1 if E(u_n) <= E(u_{n-1}) + 1e-13 |E(u_{n-1})| for
   *                n = 1..N_t, with E the discrete Ginzburg-Landau energy
   *                h^d [sum (u^2-1)^2/4 + eps^2/2 sum_faces ((u'-u)/h)^2];
   *                0 if some level violates it; -1 for the linear operators
   *                (whose flow has no such energy) or when not computed.   */
  double mass_drift;
  int energy_monotone;
  int inner_iterations;        /* BiCGStab iterations over the whole solve
                                  (PINT_FLAG_FIELD_JACOBIAN), else 0          */
} pint_report;

typedef struct pint_plan pint_plan;

/* Returns a static string naming a status code. */
const char* pint_status_string(int status);
/* Message of the last failing call on this host thread ("" if none). */
const char* pint_last_error(void);
/* Library version string. */
const char* pint_version(void);

/*
 * Validate a problem and build its plan: FP64 constant tables (a = alpha^(1/N_t),
 * a^j, the time eigenvalues lambda_{1,l} = (1 - a w^l)/dt and
 * lambda_{2,l} = theta + (1 - theta) a w^l with w = exp(-2 pi i / N_t)
 * (Section 2.1, Lemma and eq. pintiter1), the 1D Laplacian spectrum
 * (2/h^2)(cos(k pi/N) - 1), FFT twiddles), copied to the current device.
 * alpha == 0 selects alpha automatically (1e-3, reduced until
 * alpha * R^{N_t} <= 0.1 with R^{N_t} = (1 + dt mu_min)^{-N_t}, the
 * admissibility of thm3/thm6); an explicit alpha with alpha * R^{N_t} >= 1/2
 * is rejected with PINT_EINVAL.  The plan owns its device tables (< 1 MB,
 * plus 8 N_t^2 bytes for the dense time path's matrices); bulk memory is the
 * caller's workspace.  *out receives the plan.
 */
int pint_plan_create(const pint_problem* p, pint_plan** out);
/* Free a plan and its device tables.  NULL is accepted. */
int pint_plan_destroy(pint_plan* plan);
/* Message of the last failing call on this plan. */
const char* pint_plan_last_error(const pint_plan* plan);
/* Bytes of device workspace pint_solve and the stage calls need: the
 * spectral array in the working type (N_t N_s values), a second one for 2D
 * plans on the FFT time path whose time-solve tile is narrower than a 128-byte
 * line (N_t >= 512: the iteration keeps that copy in panels of 32 modes, 16
 * for FP64 and the mixed precision, level-major within a panel), an FP64 copy
 * for the mixed precision, and the per-level partial sums and control record. */
int pint_plan_workspace_size(const pint_plan* plan, size_t* bytes);
/* alpha the plan uses (after automatic choice). */
int pint_plan_alpha(const pint_plan* plan, double* alpha);

/*
 * Full solve: runs the outer iteration (residual, forward DCT-II, time
 * transform + shifted divide + inverse, inverse DCT + FP64 update, reductions
 * and stop rule) until the estimated relative error is below rtol (and the
 * FP64 residual norm has not grown over the last sweep) or max_iter is
 * reached.
 *   d_u0    [N_y][N_x] FP64 initial datum u_0.
 *   d_U     [N_t][N_y][N_x] FP64, initial guess on entry (or filled from u0
 *           with PINT_FLAG_INIT_BROADCAST_U0), solution on exit.  Also written
 *           when PINT_ENOCONV / PINT_EDIVERGED are returned.
 *   d_work  device workspace of >= pint_plan_workspace_size bytes, 256-byte
 *           aligned; contents on entry are ignored.
 *   rep     optional report (NULL allowed); rep->struct_size must be set.
 * The call enqueues on `stream` as many iterations as the previous solve of
 * the plan needed (kernels return at once after the device stop flag is set),
 * synchronizes, and then once per further iteration; the control kernel
 * writes its status to pinned host memory, so no copy is needed.  It returns
 * after the last iteration has completed on the device.  A non-NULL stream is
 * faster than the legacy default stream.
 */
int pint_solve(pint_plan* plan, const double* d_u0, double* d_U, void* d_work, size_t work_bytes,
               void* stream, pint_report* rep);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): pint_solve
 * with the library's own static device workspace instead of d_work.  It
 * allocates nothing (no hipMalloc / hipFree, no allocating library call).
 *   - Workspace: a file-scope device array of PINT_NOALLOC_WORKSPACE_BYTES
 *     (64 MiB) that every device running the library holds until the process
 *     ends; a problem whose pint_plan_workspace_size exceeds it returns
 *     PINT_ENOMEM (e.g. FP64 up to 128^2 x 256, mixed up to 128^2 x 128).
 *   - The plan is created beforehand with pint_plan_create (which does
 *     allocate its small table block); d_u0 and d_U are as for pint_solve.
 *   - PINT_FLAG_SOLVE_GRAPH and PINT_FLAG_STAGE_TIMING are rejected
 *     (PINT_EINVAL): both create runtime objects.
 *   - Every call on one device shares that device's workspace, so calls that
 *     overlap on one GPU (other host threads or streams) race; serialize
 *     them.  Nothing in the workspace needs to start at zero: the solve
 *     initializes what it reads.
 * Returns as pint_solve.
 */
#define PINT_NOALLOC_WORKSPACE_BYTES (64u << 20)
int pint_solve_noalloc(pint_plan* plan, const double* d_u0, double* d_U, void* stream, pint_report* rep);

/* ---- stage entry points (same kernels as pint_solve; used for per-stage parity) ----
 * Working precision W: double for PINT_PREC_FP64, float otherwise (for
 * PINT_PREC_MIXED the forward transform inside pint_solve and
 * pint_precond_apply is FP64, the stage DCT and time solve are FP32).  d_work must
 * be a workspace as for pint_solve.  All are asynchronous on `stream`.
 */

/* a1 (+ a2): true alpha = 0 all-at-once residual r = b_0 - K(U) of the plan's
 * operator (eqs. all-at-once1 / nonlinear_G / nonlinear_Q with alpha = 0),
 * FP64 arithmetic, written as FP64 [N_t][N_y][N_x] into d_r (no transform). */
int pint_residual(pint_plan* plan, const double* d_u0, const double* d_U, double* d_r,
                  void* d_work, size_t work_bytes, void* stream);

/* a2: orthonormal 2D (1D if dim = 1) DCT-II of each of the N_t slices of
 * d_in (type W, [N_t][N_y][N_x]) into d_out (type W, [N_t][k_y][k_x]);
 * d_in == d_out allowed.  inverse != 0 applies the inverse (DCT-III).  Both
 * buffers must be 16-byte aligned (PINT_EINVAL otherwise). */
int pint_dct(pint_plan* plan, const void* d_in, void* d_out, int inverse, void* stream);

/* a3-a5: for each spatial cosine mode k, y = Gamma^{-1} F^{-1} D^{-1} F Gamma x
 * over the time index: the alpha-circulant space-time solve in the DCT basis
 * (Section 2.1, eq. pintiter1 Steps 1-3; CH: eq. pintiter_CH), in place on
 * d_S (type W, [N_t][k_y][k_x]).  c_bar is the scalar averaged Jacobian used
 * by the CH operators (ignored for linear ones).  d_S must be 16-byte aligned
 * (PINT_EINVAL otherwise). */
int pint_time_solve(pint_plan* plan, void* d_S, double c_bar, void* stream);

/* a2-a6 without the update: d_delta = P_alpha^{-1} d_r for an FP64 residual
 * d_r [N_t][N_y][N_x] (read) into FP64 d_delta (written), through the
 * working-precision DCT and time solve. */
int pint_precond_apply(pint_plan* plan, const double* d_r, double* d_delta, double c_bar,
                       void* d_work, size_t work_bytes, void* stream);

/* The inner solve of PINT_FLAG_FIELD_JACOBIAN as a stage: delta = G~'(U)^{-1} r
 * with G~'(U) = C1^(alpha) (x) I - I (x) Lap_h J~(U) + I (x) Lap_h
 * + eps^2 I (x) Lap_h^2 and J~(U) = diag((1/N_t) sum_n 3 u_n^2) (Section 4.1,
 * eq. approx_jacobian), by BiCGStab preconditioned with the scalar-c_bar
 * solve (c_bar the mean of J~) until the residual norm has dropped by
 * inner_rtol or after inner_max iterations.  d_U, d_r, d_delta:
 * [N_t][N_y][N_x] FP64 device arrays (d_r is not modified); d_u0 as for
 * pint_solve (not read by the operator).  The plan must carry
 * PINT_FLAG_FIELD_JACOBIAN; d_work as for pint_solve.  Synchronizes.
 * *inner_iterations (nullable) receives the iterations taken. */
int pint_field_jacobian_solve(pint_plan* plan, const double* d_u0, const double* d_U, const double* d_r,
                              double* d_delta, double inner_rtol, int inner_max, void* d_work, size_t work_bytes,
                              void* stream, int* inner_iterations);

/* The FP64 eigendecomposition of the time-step pencil of a plan with
 * nonuniform steps (pint_problem.dts; Section 1): h_V [N_t][N_t] with the
 * unit-norm right eigenvectors as columns, h_W [N_t][N_t] with the left ones
 * as rows, scaled so that W C V = I, and h_d [N_t] the eigenvalues
 * d_j = 1/(theta dt_j), so that B V = C V diag(d).  Host buffers, caller-owned;
 * the call copies from the plan's device tables and synchronizes the device.
 * PINT_EINVAL for a plan with uniform steps. */
int pint_time_eig(pint_plan* plan, double* h_V, double* h_W, double* h_d);

/* Diagnostics of a space-time state: per-level discrete mass h^d sum u and
 * Ginzburg-Landau energy h^d [sum (u^2-1)^2/4 + eps^2/2 sum_faces ((u'-u)/h)^2]
 * (Section 1), FP64, written to device arrays d_mass[N_t], d_energy[N_t]. */
int pint_diagnostics(pint_plan* plan, const double* d_U, double* d_mass, double* d_energy,
                     void* stream);

/* ------------------------------------------------------------- serving ----
 * A persistent request loop (one worker thread per server) for streams of
 * solves of uneven size.  Requests are admitted first come, first served as
 * soon as a slot (a HIP stream) is free and their whole device footprint
 * (plan tables + u0 + U + workspace) fits in the caller's pool.  Active
 * requests advance one outer iteration at a time on their own streams, so
 * their work overlaps on the device; a request retires as soon as its own
 * stop rule holds and its slot and memory go to the next one (continuous
 * batching).  Iterations after the first replay a HIP graph of one outer
 * iteration, captured and instantiated once per request on its slot (an
 * executable graph is never re-targeted to another request).  Results do not
 * depend on what else is running: every request's kernels read and write only
 * its own memory, in a fixed order.
 */
#define PINT_SERVER_NO_GRAPHS 0x1u  /* launch every iteration without graphs */

typedef struct pint_server pint_server;

typedef struct pint_server_config {
  size_t struct_size;   /* sizeof(pint_server_config)                           */
  void* d_pool;         /* caller-owned device memory, 256-byte aligned; the
                           server sub-allocates every request's state from it   */
  size_t pool_bytes;    /* >= 4096                                              */
  int max_active;       /* requests in flight at once (HIP streams); 1..64, 0 = 8 */
  unsigned flags;       /* PINT_SERVER_*                                        */
  size_t host_pool_bytes; /* pinned host memory for finished results of
                             host-buffer requests awaiting pint_server_wait;
                             0 = 1 GiB.  Allocated by the server.             */
} pint_server_config;

typedef struct pint_server_statistics {
  size_t struct_size;      /* sizeof(pint_server_statistics), set by caller    */
  uint64_t submitted, completed, failed, cancelled;
  int queued, active;
  size_t pool_bytes, pool_in_use, pool_peak;
  double p50_ms, p99_ms, mean_ms, max_ms;  /* submit-to-completion latency of
                                              completed requests             */
  double dof_completed;    /* sum of N_s * N_t over completed requests         */
  double busy_seconds;     /* first admission to last completion               */
  uint64_t graphs_captured, graph_updates, graph_launches;  /* graph_updates
                              stays 0: graphs are not re-targeted          */
  double worker_host_seconds;  /* worker thread time spent admitting requests and
                                  enqueueing their iterations                  */
  size_t host_pool_bytes, host_pool_in_use;  /* pinned result pool            */
} pint_server_statistics;

/* Start a server on the current device; *out receives it.  The pool stays
 * owned by the caller and must outlive the server.  A host-buffer request is
 * admitted only when its result also fits in the pinned host result pool;
 * its U is copied there when it finishes (freeing its device block) and stays
 * until pint_server_wait copies it out, so results that are never collected
 * hold pinned memory until the server is destroyed.  Every HIP call of the
 * server is made on its worker thread. */
int pint_server_create(const pint_server_config* cfg, pint_server** out);
/* Validate and enqueue one solve (u0 broadcast as the initial guess);
 * h_u0 ([N_y][N_x] FP64 host) is copied, so the caller may reuse it at once.
 * PINT_EINVAL for an invalid problem, PINT_ENOMEM if its footprint exceeds
 * the whole pool.  *ticket identifies the request. */
int pint_server_submit(pint_server* s, const pint_problem* p, const double* h_u0, uint64_t* ticket);
/* Device-resident variant: the solve reads d_u0 ([N_y][N_x] FP64) and
 * iterates in place on d_U ([N_t][N_y][N_x] FP64), both caller-owned device
 * memory on the server's device, 8-byte aligned and not overlapping.  No
 * host copy is made in either direction and only the plan tables and the
 * workspace come from the pool.  d_u0 must hold its final values when this is
 * called (synchronize the stream that wrote it first); both buffers must stay
 * allocated and untouched until pint_server_wait has returned for the ticket,
 * after which d_U holds the result, visible to work on any stream.
 * pint_server_wait ignores h_U for such requests.  Errors as for
 * pint_server_submit, and PINT_EINVAL for NULL or misaligned buffers. */
int pint_server_submit_device(pint_server* s, const pint_problem* p, const double* d_u0, double* d_U,
                              uint64_t* ticket);
/* Block until the request is done (timeout_ms < 0: no limit), copy U
 * ([N_t][N_y][N_x] FP64 host, caller-owned; may be NULL) and the report, and
 * release the ticket.  Returns the request's status (PINT_OK, PINT_ENOCONV, PINT_EDIVERGED,
 * PINT_ECANCELED, ...), PINT_ETIMEDOUT (ticket kept), PINT_ENOTFOUND, or
 * PINT_EINVAL if another thread is already waiting for the same ticket. */
int pint_server_wait(pint_server* s, uint64_t ticket, double* h_U, pint_report* rep, int timeout_ms);
/* Cancel a queued or running request (it completes with PINT_ECANCELED). */
int pint_server_cancel(pint_server* s, uint64_t ticket);
/* Snapshot of the counters and latency percentiles. */
int pint_server_stats(pint_server* s, pint_server_statistics* st);
/* Cancel queued requests, finish running ones, stop the worker, free the
 * server's streams and host buffers.  NULL is accepted.  Returns PINT_EHIP
 * (message in pint_server_last_error) if a HIP error stopped the server or if
 * a slot's stream reports one when it is synchronized here; the server is
 * freed either way. */
int pint_server_destroy(pint_server* s);
/* Message of the last failing server call made by the calling thread ("" if
 * none); for a request that failed on the device side, its message becomes the
 * error of the thread whose pint_server_wait returned that failure. */
const char* pint_server_last_error(const pint_server* s);

#ifdef __cplusplus
}
#endif
#endif /* PINT_H */
