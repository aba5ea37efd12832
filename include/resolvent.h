/*
 * resolvent.h -- C ABI of the MI355X time-stepping resolvent library.
 *
 * The library computes the action of the resolvent of a stable linear system du/dt = L u + f on forcings
 * at many frequencies at once by time marching (Martini, Rodriguez, Towne & Cavalieri, "Efficient
 * computation of global resolvent modes", Sec. 2), and the optimal and suboptimal gains and modes by a block
 * power iteration on R^H R (Appendix A).  Conventions:
 *
 *   - the paper's system du/dt + A u = B f, y = C u (Sec. 2.1, eq. system) with L = -A and B = C = I;
 *   - forcing f(t) = sum_j F_j exp(+i w_j t) on the uniform grid w_j = w0 + j dw, j = 0..n_w-1, with
 *     dw = 2 pi / (P h) for an integer P (Sec. 2.3: w_k = 2 pi k / T, T = P h);  the response amplitudes are
 *     U_j = R_d(w_j) F_j, where R_d is the resolvent (i w I - L)^{-1} of the RK4-discretised system
 *     (it converges to the continuous resolvent at fourth order in h);
 *   - the adjoint (Sec. 2.1, eqs. adsystem and adsystemFreqDomain) is taken in the Euclidean inner product:
 *     resolvent_adjoint_apply returns R_d(w_j)^H G_j;
 *   - complex arrays are interleaved (re, im), row-major, [n_w][k][N] with N the number of state unknowns
 *     (all instances of a batch back to back); complex128 for RES_FP64 operators and complex64 for
 *     RES_MIXED operators.  Gains are always double.
 *
 * All compute calls are asynchronous on the HIP stream passed in (NULL = the default stream); device
 * arrays are owned by the caller and must stay valid until the stream reaches the call.  Calls that return
 * host data (resolvent_modes, resolvent_op_create's decay probe, resolvent_op_check) synchronise the stream.
 * A handle must not be used from two host threads at once, and calls on one handle must not overlap on
 * different streams (they share the handle's device workspace).
 */
#ifndef RESOLVENT_H
#define RESOLVENT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------------------------------- */
enum {
  RES_OK = 0,
  RES_EINVAL = 1,      /* invalid argument (NULL pointer, bad size, unsupported combination)            */
  RES_EGRID = 2,       /* frequency grid not commensurate with the step: |dw| P h != 2 pi, or n_w > P,   */
                       /* or the periodic projection stride does not divide P / leaves fewer than n_w    */
                       /* samples per period                                                             */
  RES_ESTEP = 3,       /* the decay probe diverged at a rate only an unstable RK4 step explains           */
  RES_EUNSTABLE = 4,   /* the decay probe did not decay: the operator is not stable (Sec. 2.1 assumes it) */
  RES_ENONFINITE = 5,  /* a result contained NaN or Inf                                                   */
  RES_ENOMEM = 6,      /* device allocation failed                                                        */
  RES_EHIP = 7,        /* HIP runtime error (message in resolvent_last_error)                             */
  RES_ENOTSUP = 8      /* operation not supported for this operator kind                                  */
};

/* ---- operator kinds, precisions, methods ---------------------------------------------------------- */
enum {
  RES_OP_TRIDIAG = 1,  /* 1-D three-point operator, complex coefficients, instances back to back        */
  RES_OP_ADR2D = 2,    /* 2-D five-point operator, real coefficients, one complex unknown per node       */
  RES_OP_ADR3D3C = 3   /* 3-D seven-point operator, real coefficients, three coupled unknowns per node   */
};
enum { RES_FP64 = 0, RES_MIXED = 1 };
/* RES_TRANSIENT: transient-response method with a one-window forcing (Sec. 2.2): force for P steps, march a
 *   further `tail` steps while the response decays, project every step.
 * RES_PERIODIC: steady-state-response method (Sec. 2.3): force for `periods` periods, project the last
 *   period every `stride` steps. */
enum { RES_TRANSIENT = 0, RES_PERIODIC = 1 };

typedef struct resolvent_op resolvent_op;

/* Operator description.  All arrays are host arrays, read during resolvent_op_create only.
 *
 * RES_OP_TRIDIAG:  (L u)_i = lower_i u_{i-1} + diag_i u_i + upper_i u_{i+1}, complex (interleaved re,im),
 *   length n_total = inst_offsets[ninst].  Instances [inst_offsets[m], inst_offsets[m+1]) are independent:
 *   lower at an instance's first unknown and upper at its last are ignored (treated as 0: homogeneous
 *   Dirichlet values outside each instance).  ninst = 1 with inst_offsets = NULL means one instance of
 *   length nx.
 * RES_OP_ADR2D / RES_OP_ADR3D3C: grid nx * ny * nz nodes, x fastest (nz = 1 in 2-D), homogeneous Dirichlet
 *   values outside the grid.  For node (x, y, z) with line index l = z*ny + y and component c:
 *     (L q)_c = cxm[l] q_c(x-1) + cxp[l] q_c(x+1) + cym[l] q_c(y-1) + cyp[l] q_c(y+1)
 *             + czm[l] q_c(z-1) + czp[l] q_c(z+1) + dfield[node] q_c + sum_c' coupling[l][c][c'] q_c'
 *   (czm, czp and coupling are ignored in 2-D; coupling[l] is a row-major 3x3 real matrix whose diagonal
 *   adds to dfield).  Unknowns are component-major: [c][z][y][x].
 */
typedef struct {
  int32_t kind;              /* RES_OP_*                                                             */
  int32_t precision;         /* RES_FP64 or RES_MIXED (FP32 stepping and phase GEMMs, FP64 QR/gains)  */
  double h;                  /* RK4 step                                                              */
  int32_t ninst;             /* RES_OP_TRIDIAG: number of instances (>= 1)                             */
  const int64_t* inst_offsets; /* [ninst + 1] or NULL                                                 */
  const double* lower;       /* RES_OP_TRIDIAG: complex [n_total]                                     */
  const double* diag;        /* RES_OP_TRIDIAG: complex [n_total]                                     */
  const double* upper;       /* RES_OP_TRIDIAG: complex [n_total]                                     */
  int64_t nx, ny, nz;        /* grid sizes (RES_OP_TRIDIAG with inst_offsets == NULL: nx = n_total)    */
  const double* cxm; const double* cxp;  /* [ny * nz]                                                 */
  const double* cym; const double* cyp;  /* [ny * nz]                                                 */
  const double* czm; const double* czp;  /* [ny * nz] (3-D)                                          */
  const double* dfield;      /* [nz * ny * nx]                                                        */
  const double* coupling;    /* [ny * nz][3][3] (3-D)                                                 */
  /* Decay probe (Sec. 2.3: the transient time is estimated from a prior run in which the norm of a random
   * initial condition falls to a prescribed small value).  probe = 0 skips it. */
  int32_t probe;
  double probe_tol;          /* relative norm to reach (e.g. 1e-9)                                     */
  double probe_tmax;         /* give up (RES_EUNSTABLE) after this much time                           */
  uint64_t probe_seed;       /* seed of the SplitMix64 stream of the random initial condition          */
} resolvent_op_desc;

/* Frequency grid w_j = omega0 + j * domega, j = 0 .. n_omega-1; |domega| P h must equal 2 pi for an integer
 * P (relative tolerance 1e-9) and n_omega <= P, else RES_EGRID. */
typedef struct {
  double omega0;
  double domega;
  int32_t n_omega;
} resolvent_grid;

/* The grid of an array of n_omega >= 2 analysis frequencies (host, ascending or descending): the array must be
 * uniform (every entry within 1e-9 |domega| of omega[0] + j domega with domega = (omega[n-1] - omega[0]) / (n - 1)).
 * The spacing is snapped to 2 pi / (P h) with P the multiple of `stride` (>= 1, the projection stride of a
 * periodic run; 1 otherwise) nearest 2 pi / (|domega| h), as the time grid of Sec. 2.3 requires (eq. fourier's
 * frequencies are the harmonics of the period P h); omega0 = omega[0].  *out gets the snapped grid and *P_out
 * (may be NULL) the period in steps.  Host only, no device call.  RES_EINVAL for NULL arguments, h <= 0 or
 * stride < 1; RES_EGRID for n_omega < 2, a non-uniform or non-finite array, equal end points, or a snapped P
 * with fewer than n_omega steps. */
int resolvent_grid_from_omegas(const double* omega, int32_t n_omega, double h, int64_t stride,
                               resolvent_grid* out, int64_t* P_out);

/* Schedule of one run (one application of R_d or R_d^H). */
typedef struct {
  int32_t method;            /* RES_TRANSIENT or RES_PERIODIC                                          */
  int64_t tail;              /* RES_TRANSIENT: steps marched after the forcing window                  */
  int32_t periods;           /* RES_PERIODIC: periods marched (>= 1); the last one is projected        */
  int64_t stride;            /* RES_PERIODIC: projection stride (divides P, P/stride >= n_omega)       */
} resolvent_run;

/* Create / destroy.  Uploads the operator, builds the RK4 step stencils of L and L^H, and runs the decay
 * probe when asked (synchronising `stream`).  On failure *out is NULL. */
int resolvent_op_create(const resolvent_op_desc* desc, void* stream, resolvent_op** out);
void resolvent_op_destroy(resolvent_op* op);

/* Number of unknowns of one column (n_total of the description). */
int64_t resolvent_op_size(const resolvent_op* op);
/* Probe result: time (in time units) the random initial condition took to fall below probe_tol, or -1. */
double resolvent_op_decay_time(const resolvent_op* op);

/* Replace the diagonal (the reaction field): RES_OP_TRIDIAG takes complex [n_total] (the new diag),
 * ADR kinds take real [nz*ny*nx] (the new dfield).  `on_device` = 1 if the array is device memory.
 * Stream-ordered; the array must stay valid until the stream reaches the call. */
int resolvent_op_set_diagonal(resolvent_op* op, const double* values, int32_t on_device, void* stream);

/* u_hat[j] = R_d(w_j) f_hat[j]  for every frequency j and every one of the k columns, in ONE time-marched run
 * (Sec. 2.1: all frequencies from one direct run).  f_hat, u_hat: device [n_omega][k][N] complex (dtype per
 * precision, see above); they may not alias. */
int resolvent_apply(resolvent_op* op, const resolvent_grid* grid, const resolvent_run* run, int32_t k,
                    const void* f_hat, void* u_hat, void* stream);

/* resolvent_apply for callers that cannot allocate device memory: code under HIP graph capture (it may be
 * captured without a prior uncaptured call), tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, layout, ownership and results as resolvent_apply (up to rounding: the forcing may be synthesised
 * in tiles where resolvent_apply holds a whole period, and the stepper relaunches at every neighbour exchange
 * unless the handle already holds its exchange area).  Its workspace is one fixed device array of
 * RESOLVENT_NOALLOC_SCRATCH_BYTES that the library defines; each GPU the library runs on holds its own copy from
 * the first call on it until the process ends.  The call allocates and frees nothing, on the device or through
 * any allocating library routine.  Every call on a GPU uses that GPU's array, which keeps the last call's
 * contents: calls that overlap on one GPU (other streams, other handles, other host threads) race and give wrong
 * results; serialise them.  The workspace a run needs grows with n_omega * k * N (the pre-filtered forcing, and for
 * RES_MIXED handles the FP64 accumulator, are whole blocks of that size); a run that needs more than the array
 * holds returns RES_EINVAL with the byte counts in resolvent_last_error before any work is queued.  Also
 * RES_EINVAL when the current device is not the one the handle was created on.  Asynchronous on `stream`. */
#define RESOLVENT_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int resolvent_apply_noalloc(resolvent_op* op, const resolvent_grid* grid, const resolvent_run* run, int32_t k,
                            const void* f_hat, void* u_hat, void* stream);

/* Smallest device workspace, in bytes, that resolvent_apply_noalloc needs for this grid, run and k (the layout
 * with the shortest tiles and flushes; given more room, it takes longer ones), so that a caller can tell before
 * the call whether the run fits RESOLVENT_NOALLOC_SCRATCH_BYTES.  Host only: no device call, no allocation.
 * Errors as resolvent_apply's argument checks (RES_EINVAL, RES_EGRID). */
int resolvent_workspace_size(resolvent_op* op, const resolvent_grid* grid, const resolvent_run* run, int32_t k,
                             size_t* bytes);

/* z_hat[j] = R_d(w_j)^H g_hat[j]: the adjoint run (Sec. 2.1, eq. adsystemFreqDomain): L^H marched with the
 * frequencies negated (equivalent to the paper's backward integration in reversed time). */
int resolvent_adjoint_apply(resolvent_op* op, const resolvent_grid* grid, const resolvent_run* run, int32_t k,
                            const void* g_hat, void* z_hat, void* stream);

/* Block power iteration (Appendix A, eqs. iteration, powerMethod, arDec) with per-frequency normalisation and
 * orthogonalisation of the Fourier coefficients (Sec. 2.3), `iters` iterations of a direct and an adjoint run:
 *   F = Q(QR(F_hat));  Y = R_d F = Q_Y R_Y;  R_Y = Phi Sigma Psi^H;  gains = Sigma, V = F Psi, U = Q_Y Phi;
 *   F_hat <- R_d^H Q_Y R_Y Psi.
 * f0_hat: device [n_omega][k][N] initial forcings (caller-generated, e.g. random).
 * gains:  host double [ninst][n_omega][k], descending per frequency (the last iteration's estimates).
 * V, U:   device [n_omega][k][N] force and response modes (each up to a common unit-modulus factor), or NULL.
 * hist:   host double [iters][ninst][n_omega][k][2] or NULL: per iteration the Rayleigh-Ritz gains and the
 *         norm-ratio estimate sqrt(||F_hat_i||) of eq. tildeSig.
 * Synchronises `stream`.  k <= 8.  Returns what the device flagged during the call, as resolvent_op_check
 * does: RES_ENONFINITE for non-finite values or a rank-deficient QR block, RES_EHIP for an abandoned exchange. */
int resolvent_modes(resolvent_op* op, const resolvent_grid* grid, const resolvent_run* run, int32_t k,
                    int32_t iters, const void* f0_hat, double* gains, void* V, void* U, double* hist,
                    void* stream);

/* Block Arnoldi (Krylov-subspace) estimates (Appendix A, eqs. RRFi, arDec, freqOrt and the mode estimates that
 * follow them), `blocks` direct and `blocks` adjoint runs: the forcing blocks are B_0 = Q(QR(f0_hat)) and
 * B_{i+1} = Q(QR(part of R_d^H R_d B_i orthogonal to B_0 .. B_i)) (classical Gram-Schmidt, two passes, per
 * frequency and instance, FP64); H = B^H R_d^H R_d B (from the upper block triangle of the Gram-Schmidt
 * coefficients, mirrored) gives gains = sqrt(eigenvalues of H), V = B psi, U = R_d B psi / gain.  Converges to
 * suboptimal gains much faster than resolvent_modes when the gains are close (the paper's recommendation for
 * suboptimal modes with the periodic method).
 * f0_hat: device [n_omega][k][N] start block (working precision, as resolvent_modes).
 * gains:  host double [ninst][n_omega][k], the k largest estimates per frequency, descending.
 * V, U:   device [n_omega][k][N] force and response modes (each up to a unit-modulus factor), or NULL.
 * hist:   host double [blocks][ninst][n_omega][k] or NULL: the estimates after each block.
 * Synchronises `stream`.  k <= 8, blocks * k <= 40 and at most the unknowns of every instance; RES_EINVAL
 * otherwise.  Reports the device's flags as resolvent_modes does. */
int resolvent_krylov(resolvent_op* op, const resolvent_grid* grid, const resolvent_run* run, int32_t k,
                     int32_t blocks, const void* f0_hat, double* gains, void* V, void* U, double* hist,
                     void* stream);

/* Gradient of a real objective J(u_hat) of u_hat = resolvent_apply(f_hat) through the time-stepped run
 * (discrete adjoint of the RK4 march, recomputing the forward trajectory from checkpoints taken every
 * `checkpoint_every` steps).  g_hat = dJ/du_hat (device, same layout/dtype as u_hat, with the convention
 * dJ/dRe + i dJ/dIm).  Outputs: f_grad (device, same layout as f_hat, same convention) if not NULL, and
 * mu_grad (device double, RES_OP_TRIDIAG: [n_total], ADR kinds: [nz*ny*nx]) = dJ/d(real part of the diagonal)
 * if not NULL.  Supported for RES_TRANSIENT and RES_PERIODIC runs.  checkpoint_every <= 0 picks about
 * sqrt(steps).  Arithmetic is FP64 and both gradients accumulate in FP64; the rows the mode stores (states,
 * checkpoints, stage values, adjoint states, synthesised forcing and seed rows) are FP64 for RES_FP64 operators and
 * FP32 for RES_MIXED ones (FP64 with resolvent_op_set_backward_rows(op, 1)).  Memory (held by the handle): the
 * seed, pre-filtered forcing and (mixed operators, or chunked columns) forcing blocks [n_omega][kc][N] in the row
 * precision, the FP64 gradient accumulator [n_omega][kc][N], Horner work blocks within
 * RESOLVENT_HORNER_BUDGET_GB, ceil(steps / C) checkpoints and a few C-row segments of [kc][N] rows
 * (C = checkpoint_every).  The columns evolve independently, so when the rows of all k columns do not fit the
 * mode frees the handle's forward workspace and then runs the columns in chunks of kc < k (the mu gradient sums
 * over the chunks; RESOLVENT_BACKWARD_COLUMNS = kc forces a chunk size).  The three stage rows of every step of a
 * segment are kept when they fit in half of the free device memory, else recomputed.  With mu_grad NULL only the
 * adjoint recursion runs (the forcing gradient does not depend on the forward trajectory): no forward march,
 * checkpoints or recomputation.  An allocation that fails returns RES_ENOMEM. */
int resolvent_apply_backward(resolvent_op* op, const resolvent_grid* grid, const resolvent_run* run, int32_t k,
                             const void* f_hat, const void* g_hat, void* f_grad, double* mu_grad,
                             int32_t checkpoint_every, void* stream);

/* Row precision of resolvent_apply_backward for a RES_MIXED operator: fp64 != 0 keeps its rows in FP64 (twice the
 * memory and traffic; gradients then agree with the FP64 operator's to the rounding of the forward run's
 * coefficients), 0 (the default) in FP32.  No effect on RES_FP64 operators.  Reverse-mode differentiation is an
 * extension of the paper's method (it differentiates the time-stepped run of Sec. 2.3). */
int resolvent_op_set_backward_rows(resolvent_op* op, int32_t fp64);

/* HIP graphs.  resolvent_apply, resolvent_adjoint_apply and resolvent_apply_backward may be recorded into a
 * caller's graph (stream capture) once an uncaptured call with the same sizes has sized the handle's workspace:
 * nothing inside them then allocates, copies from the host or synchronises (fills are kernels, not memset
 * nodes); a call that would need to grow the workspace during capture fails with RES_EINVAL.  The graph reads
 * and writes the device buffers given at capture time.  resolvent_modes returns host data and cannot be
 * captured; with resolvent_op_set_graphs(op, 1) it instead records its second iteration once and replays it for
 * every iteration but the first and the last (results are identical to the eager form).  For callers that
 * replay launch sequences (batched serving loops, graph-based pipelines); not part of the paper's method. */
int resolvent_op_set_graphs(resolvent_op* op, int32_t enable);

/* Stepper plan of a RES_OP_TRIDIAG operator (how the time march is laid out on the device; results do not
 * depend on it, bit for bit): plan[0] = kernel configuration (0..15: threads per workgroup, unknowns per
 * thread and forcing prefetch depth), plan[1] = owned unknowns per workgroup (0: each column in one
 * workgroup), plan[2] = steps between neighbour exchanges (the halo is 4 * plan[2] unknowns per side),
 * plan[3] = 1 for one persistent launch per march with in-kernel exchange, 0 for a relaunch per exchange.
 * set_plan raises the configuration to the smallest that holds the longest region and drops persistence when
 * the plan cannot exchange in-kernel; get_plan returns what is in effect.  RES_ENOTSUP for grid operators,
 * RES_EINVAL for a malformed plan.  These are layout choices of this implementation, not of the paper. */
int resolvent_op_get_plan(const resolvent_op* op, int32_t plan[4]);
int resolvent_op_set_plan(resolvent_op* op, const int32_t plan[4]);

/* Input and output matrices and metrics of the resolvent problem (Sec. 2.1, eqs. systemFreqDomain, adsystem and
 * the discrete adjoints after them), diagonal: B = diag(b), C = diag(c) (force and observation masks or weights),
 * W_f = diag(wf), W_y = diag(wy) (force and observation metrics, e.g. non-uniform-grid quadrature).  Host arrays of
 * the operator's N unknowns (all instances, grid layout for grid operators), each NULL for the identity; all NULL
 * restores B = C = W = I.  Afterwards
 *   resolvent_apply returns y = C R_d B f, resolvent_adjoint_apply returns R_y^dagger y = W_f^{-1} B^H R_d^H C^H W_y y
 *   (the adjoint of R_y = C R_d B in these metrics; W_u of the state cancels),
 *   resolvent_modes and resolvent_krylov maximise ||C R_d B f||_{W_y} / ||f||_{W_f}: they iterate on the Euclidean
 *   R~ = W_y^{1/2} C R_d B W_f^{-1/2}, take f0_hat in the problem's coordinates and return W_f-orthonormal force
 *   modes V and response modes U = C R_d B V / sigma.
 * The reverse mode (resolvent_apply_backward) differentiates y = C R_d B f: the forcing gradient is
 * B R_d^H C g and the mu gradient that of R_d at the input B f with the cotangent C g.  RES_EINVAL for
 * non-finite b or c, wf or wy not finite and positive, or during graph capture. */
int resolvent_op_set_weights(resolvent_op* op, const double* b, const double* c, const double* wf,
                             const double* wy);

/* Multi-step march of a RES_OP_TRIDIAG operator (Sec. 2.1, the RK4 march written as one step): with m = 2 or 4
 * each kernel step advances m RK4 steps at once, u_{s+m} = P(Z)^m u_s + sum_j e^{i w_j t_s} G_j^(m) with
 * G_j^(m) = sum_{r<m} e^{i w_j r h} P(Z)^(m-1-r) h Q_j(Z) F_j.  P(Z)^m is formed once in FP64 on the host (a
 * band of radius 4m), so the march reaches the same discrete response as m = 1 up to rounding (not bit for bit).
 * A run uses m only when its period, projection start and stride, and the plan's exchange interval (plan[2])
 * are multiples of m and the forcing stays on for the whole run (the periodic method); otherwise, e.g. for the
 * transient method, it marches one step at a time.  Default 4.  A handle on its default stepper plan moves
 * to the default plan of the new power (set_plan and the autotuner fix the plan).  RES_EINVAL for m not in
 * {1, 2, 4} or during graph capture, RES_ENOTSUP for grid operators.  The autotuner times plans in the current
 * form. */
int resolvent_op_set_step_power(resolvent_op* op, int32_t m);
int resolvent_op_get_step_power(const resolvent_op* op, int32_t* m);

/* Stepper autotuner for RES_OP_TRIDIAG operators: times every candidate plan on `steps` forced steps of k
 * columns on `stream` (the handle's state buffers are overwritten; run results are unaffected), keeps the
 * fastest, and writes it to plan_out and its time per step in microseconds to us_per_step (each may be NULL).
 * Synchronises the stream.  steps >= 16.  RES_ENOTSUP for grid operators. */
int resolvent_op_tune(resolvent_op* op, int32_t k, int32_t steps, int32_t plan_out[4], double* us_per_step,
                      void* stream);

/* Opt-in kernel timing: while enabled, the library records HIP events on the caller's stream around each of its
 * kernel launches.  resolvent_op_get_timing synchronises the stream, returns the summed device time (ms) and
 * the number of launches of one kernel class since the last query, and resets that class.  Classes:
 * 0 = time stepper, 1 = forcing synthesis GEMM, 2 = Fourier projection GEMM, 3 = per-frequency QR/SVD. */
enum { RES_TIMING_STEPPER = 0, RES_TIMING_SYNTHESIS = 1, RES_TIMING_PROJECTION = 2, RES_TIMING_QR = 3 };
int resolvent_op_set_timing(resolvent_op* op, int32_t enable);
int resolvent_op_get_timing(resolvent_op* op, int32_t kind, double* total_ms, int64_t* launches);

/* ---- Transient-response method with time-domain hand-off (Sec. 2.2, App. B, App. C) ----------------------------
 * A signal is a series of samples [n_samples][k][N] (caller-owned device memory, complex128 for RES_FP64 handles,
 * complex64 for RES_MIXED ones, interleaved): sample i is the signal at t_i = i * every * h.
 *
 * resolvent_signal_run: the run of an operator (three-point or grid) forced by a sampled signal, from rest (Sec. 2.2,
 * eqs. system and adsystem with B = C = I).  adjoint = 0: du/dt = L u + f(t), u(0) = 0; y receives u(t_i).
 * adjoint = 1: -dz/dt = L^H z + f(t) backward in time from z(T) = 0, T = (n_samples - 1) every h; y receives
 * z(t_i).  Classical RK4 with step h; each stage is forced by the signal at its own time, interpolated between
 * samples (App. C) by scheme 0 (C0, linear), 1 (C1, cubic Hermite on second-order central derivatives, first-order
 * one-sided at the end samples) or 2 (C2, quintic Hermite on five-point first and second derivatives;
 * second-order at the samples next to the ends, first-order first derivative and zero second derivative at the end
 * samples).  Three-point operators take m RK4 steps per kernel step (resolvent_op_set_step_power) when every is a
 * multiple of m; grid operators one.  With B, C and metrics set (resolvent_op_set_weights) the run returns C u for
 * the forcing B f, and the adjoint run W_f^{-1} B^H z for the forcing C^H W_y f, as resolvent_apply and
 * resolvent_adjoint_apply do.  f and y must not alias.  RES_EINVAL for k < 1, n_samples < 2, every < 1 or an
 * unknown scheme.  Asynchronous on `stream`.
 *
 * resolvent_fir_design: a linear-phase FIR filter of even order n (n + 1 taps, App. B) approximating a desired
 * amplitude response given at npts breakpoints nu (non-decreasing in [-1, 1]: frequency over the Nyquist
 * frequency pi / dt, negative frequencies included; linear between breakpoints, the end values beyond them) with
 * gains >= 0: the response sampled on M = 2 max(512, 2^ceil(log2 n)) uniform frequencies nu_q = -1 + 2q/M,
 * transformed back with an n/2-sample delay and multiplied by a Hamming window,
 *     b_m = (0.54 - 0.46 cos(2 pi m / n)) (1/M) sum_q D(nu_q) e^{i pi nu_q (m - n/2)}.
 * A response symmetric in nu gives real taps.  Host only: taps receives n + 1 complex128 (2 (n + 1) doubles,
 * caller-owned host memory).  RES_EINVAL for an odd order, order < 2 or beyond the limit of resolvent_fir_apply,
 * or malformed breakpoints.
 *
 * resolvent_fir_apply: y[t][c] = sum_{m=0}^{n} b[m] x[t + n/2 - m][c] for t < n_t, c < ncols (x = 0 outside
 * [0, n_t)): the filter with its delay removed, so a complex exponential of frequency nu leaves multiplied by
 * H(nu) = sum_m b_m e^{-i pi nu (m - n/2)}.  taps: device complex128 [order + 1]; x, y: device [n_t][ncols],
 * complex128 if fp64 else complex64, not aliased.  Order even, 0 <= order <= 4080.  Asynchronous on `stream`.
 *
 * resolvent_trm_modes: the power iteration with time-domain hand-off (Sec. 2.2 and App. A).  Starting from the
 * sampled forcing f0 (tapered: zero on the first and last `pad` samples, raised-cosine ramps of `ramp` samples,
 * one between; then normalised), each of `iters` iterations
 *   1. runs the direct signal run of the forcing F and the adjoint signal run forced by its response Y, giving W;
 *   2. transforms F, Y and W at the n_omega analysis frequencies omegas (host array, any values with
 *      |w| every h <= pi): X(w) = dt sum_i x_i e^{-i w t_i}, dt = every h, and writes
 *      gains[it][j] = ||Y(w_j)|| / ||F(w_j)|| and (if amps is not NULL) amps[it][j] = ||F(w_j)||, norms over all
 *      k N values of the frequency;
 *   3. flattens W (App. B): `passes` passes of the FIR filter of order `order` designed for
 *      (1/||W(w_j)||)^(1/passes) at the analysis frequencies (largest 1), falling linearly to zero `margin`
 *      rad per time unit outside them and zero beyond (passes = 0: no filter);
 *   4. hands the result back, tapered and normalised, as the next F.
 * With B, C and metrics set the iteration runs on the Euclidean R~ = W_y^{1/2} C R B W_f^{-1/2} as resolvent_modes
 * does: f0 is taken in the problem's coordinates (times W_f^{1/2} before the taper), F, Y, W and the gains are those
 * of R~, and the modes come back as W_f^{-1/2} V~ and W_y^{-1/2} U~.
 * f_out (device, may be NULL) receives the last F; V and U (device [n_omega][k][N] in the handle's I/O type, each
 * may be NULL) receive the force and response modes of the last iteration, F(w_j) / ||F(w_j)|| and
 * Y(w_j) / ||Y(w_j)|| (for k = 1 the leading modes at any analysis frequency).  The flattening response spans the square of the gain range,
 * more than one windowed filter realises when gains differ by 1e3 (passes = 2 realises 1e6).  Synchronises
 * `stream` every iteration and cannot be captured; reports the device's flags as resolvent_modes does.  Errors as resolvent_signal_run, and RES_EINVAL for
 * n_omega < 1, iters < 1, a bad order, a taper that leaves no sample at one or frequencies beyond Nyquist. */
int resolvent_signal_run(resolvent_op* op, int32_t k, int64_t n_samples, int32_t every, int32_t scheme,
                         int32_t adjoint, const void* f, void* y, void* stream);
int resolvent_fir_design(int32_t order, int32_t npts, const double* nu, const double* gain, double* taps);
int resolvent_fir_apply(int32_t fp64, int64_t n_t, int64_t ncols, int32_t order, const double* taps, const void* x,
                        void* y, void* stream);
int resolvent_trm_modes(resolvent_op* op, int32_t k, int64_t n_samples, int32_t every, int32_t scheme,
                        const void* f0, int32_t n_omega, const double* omegas, int32_t iters, int32_t order,
                        int32_t passes, int64_t pad, int64_t ramp, double margin, double* gains, double* amps,
                        void* f_out, void* V, void* U, void* stream);

/* Synchronise `stream` and report RES_ENONFINITE if any result produced since the last check held NaN/Inf. */
int resolvent_op_check(resolvent_op* op, void* stream);

/* Static message for a status code. */
const char* resolvent_strerror(int status);
/* Detail of the last error on this host thread (empty if none). */
const char* resolvent_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RESOLVENT_H */
