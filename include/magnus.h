/*
 * magnus.h - C ABI of the MI355X (gfx950) iterated stochastic Magnus library.
 *
 * Method: Kamm, Pagliarani, Pascucci, "Numerical solution of kinetic SPDEs
 * via stochastic Magnus expansion" (arXiv 2207.09776).  The library computes,
 * for many Brownian paths at once, the iterated Magnus scheme of Section 2
 * ("Iterated Magnus expansion") for the space-discretised SPDE
 * eq. (generalSPDE) -> eq. (SPDEvec):
 *
 *     u_{k+1} = exp(Y_{p,k}) u_k,   Y_{p,k} = sum_l c_{p,k,l} M_l,
 *     M = (B, A, A^2, [B,A], [[B,A],A], [[B,A],B])      (eq. (MagnusFormulas))
 *
 * plus the Euler-Maruyama baseline (eq. (EulerMaruyama)) and the error norm
 * of eq. (meanErr) against the closed-form Langevin solution (Section 3.1).
 *
 * Conventions shared by every entry point
 *   - A grid function has N = nx*nv entries stored [nv][nx], x fastest: the
 *     column stacking vec of Section 2.  Batches are [P][nv][nx].
 *   - "device" pointers are HIP device memory owned by the caller; "host"
 *     pointers are ordinary host memory owned by the caller.  The library
 *     never frees or keeps caller memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Compute calls are asynchronous on that stream: they enqueue kernels and
 *     return; results (including per-path flags) are valid after the stream
 *     is synchronised.  They do not allocate device memory or synchronise.
 *   - Return value: MG_OK or a negative mg_status for argument, shape, support
 *     or launch errors, detected on the host before anything is enqueued (a
 *     launch error after enqueueing returns MG_EHIP).  mg_last_error() gives a
 *     message for the calling thread.  Numerical trouble inside a path (a
 *     non-finite value, or a step beyond the convergence radius of the Magnus
 *     expansion, Theorem 'convergence') does not abort the batch: it is
 *     reported per path in the `flags` array.
 */
#ifndef MAGNUS_H
#define MAGNUS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mg_status;
#define MG_OK            0
#define MG_EINVAL       (-1)   /* bad argument value or NULL pointer         */
#define MG_ESHAPE       (-2)   /* inconsistent sizes                         */
#define MG_EUNSUPPORTED (-3)   /* valid input this library does not implement */
#define MG_EHIP         (-4)   /* HIP runtime error                          */
#define MG_ENOMEM       (-5)   /* host allocation failed / workspace too small */
#define MG_ENONFINITE   (-6)   /* mg_check_flags: at least one path is flagged  */

/* Per-path flag bits written to `flags[p]` (0 = path finished normally). */
#define MG_FLAG_NONFINITE 1    /* a NaN or Inf appeared in the path's state   */
#define MG_FLAG_NORM      2    /* ||Y_{p,k} - mu I||_1 exceeded the supported range */
#define MG_FLAG_ABORT     4    /* a multi-workgroup launch gave up waiting for a
                                  workgroup of its group (result not valid)    */
#define MG_FLAG_NEGATIVE  8    /* mg_magnus_expmv: the initial state was non-negative
                                  and the final one has a negative part beyond 0.1
                                  of its maximum.  The exact solution of the forward
                                  equation stays a density, so this marks a Magnus
                                  step beyond the convergence region of the
                                  expansion (Theorem 'convergence'): rerun the path
                                  with more steps (the result is still written).
                                  A gross-failure check: the central differences
                                  leave small negative values on coarse grids
                                  (a few 1e-2 of the maximum), which stay unflagged. */

/* Precision forms of the Taylor chain (the state u is FP64 in both). */
#define MG_FP64  0             /* every operation in FP64                     */
#define MG_FP32C 1             /* FP32 stencil products with a compensated FP32
                                  Taylor sum; FP64 norm, (m,s) choice, e^{mu/s}
                                  scaling and state between Magnus steps       */

/* Homogeneous grids of eq. (xGrid)/(vGrid): interior nodes
 * x_i = ax + i*(bx-ax)/(nx+1), i = 1..nx (same for v); u = 0 on the boundary. */
typedef struct {
    int32_t nx, nv;
    double ax, bx, av, bv;
} mg_grid;

/* Coefficient grids of eq. (generalSPDE), host arrays of nx*nv doubles in
 * [nv][nx] order; NULL means identically zero.  Every coefficient may depend
 * on v, or on x and v when its grid is a sum of at most 4 products b(v) a(x)
 * (to rounding).  The build supports what the Magnus basis of the requested
 * order then holds in its factored form: x words diag(x_0) L diag(x_1)
 * [L diag(x_2)] of at most two letters L (D^x or D^xx) per term, at most 32
 * such x-terms over 16 distinct x vectors, v bands of radius at most 2 beside
 * x-dependent factors.  That covers the Langevin SPDE with constant
 * (eq. (coeffsLangevinConst)) and the paper's variable coefficients
 * (eq. (coeffsLangevinVar)) at every order, gxx, x-dependent fx and gxv at
 * every order, sx at orders 1 and 2, and an x,v-dependent diffusion gvv at
 * orders 1 and 2.  Anything else returns MG_EUNSUPPORTED. */
typedef struct {
    const double *h, *fx, *fv, *gxx, *gxv, *gvv, *sig, *sx, *sv;
} mg_coeffs;

/* Parameters of the closed-form constant-coefficient solution (Section 3.1):
 * g^vv = a, sigma^v = sigma (0 < sigma^2 < a), Gaussian initial density
 * N(0, s0sq I), time T. */
typedef struct {
    double a, sigma, s0sq, T;
} mg_exact;

/* Opaque operator set built once per (grid, coefficients, order). */
typedef struct mg_ops mg_ops;

/* --------------------------------------------------------------------------
 * mg_build_operators  (Section 2, "Computation of A and B"; eq. (MagnusFormulas))
 *
 * Builds on the host, in FP64, the drift B and noise A of eq. (SPDEvec) and
 * the commutators needed by Magnus order `order` (1..3) as exact products of
 * the truncated matrices, in the factored form
 *     M_l = sum_{q=0..2} V_{l,q} (x) (D^x)^q + sum_t W_{l,t} (x) diag(a_t)
 *           + sum_k C_{l,k} (x) X_k,
 * V_{l,q}, W_{l,t}, C_{l,k} banded nv x nv, a_t the x profiles of the
 * x-dependent coefficients, X_k the x words that D^x, D^xx and the x profiles
 * form in the products (see mg_coeffs), and uploads the tables to the current
 * HIP device.  Operators with x-dependent factors run on grids up to
 * 512 x 512 (FP64; the FP32C form takes no x-terms).
 *   grid, coeffs : host, read during the call only.
 *   out          : receives a library-owned handle; free with
 *                  mg_free_operators.  The handle is immutable after build and
 *                  may be used from several streams at once.
 * Errors: MG_EINVAL (NULL, order outside 1..3, nx or nv < 1, empty domain),
 *         MG_EUNSUPPORTED (coefficients outside the supported set),
 *         MG_EHIP, MG_ENOMEM.  Grid sizes without a kernel are reported by
 *         the compute calls.
 * ------------------------------------------------------------------------ */
mg_status mg_build_operators(const mg_grid* grid, const mg_coeffs* coeffs, int32_t order,
                             mg_ops** out);

/* Frees a handle from mg_build_operators (NULL is accepted).  The caller must
 * make sure no enqueued work still uses it. */
mg_status mg_free_operators(mg_ops* ops);

/* --------------------------------------------------------------------------
 * mg_iterated_integrals  (eq. (MagnusFormulas); Section 3 "Implementation")
 *
 * For each path p and Magnus step k (sub-interval of length h = T/K, path
 * restarted at its left end) computes from the fine increments the weights
 *   c0 = h, c1 = dW, c2 = -h/2, c3 = I1 - h dW/2,
 *   c4 = I2/2 - dW I1/2 + h dW^2/12, c5 = J - h I1/2 - h^2 dW/12
 * with I1 = int W, I2 = int W^2, J = int r W dr over the sub-interval, taken
 * exactly for the piecewise-linear path through the fine nodes.  Weights
 * beyond `order` are written as 0.  Also writes per path (W_T, int_0^T W).
 *   dW       : device, [P][Nf] fine increments (delta = T/Nf).
 *   coef     : device, [P][K][6] output.
 *   pathstat : device, [P][2] output (may be NULL).
 * Errors: MG_EINVAL (NULL, T <= 0, order outside 1..3), MG_ESHAPE (P < 0,
 *         K < 1, Nf < 1, Nf % K != 0).  P = 0 is a no-op.
 * ------------------------------------------------------------------------ */
mg_status mg_iterated_integrals(const double* dW, int64_t P, int64_t Nf, double T, int32_t K,
                                int32_t order, double* coef, double* pathstat, void* stream);

/* --------------------------------------------------------------------------
 * mg_iterated_integrals_steps  (eq. (MagnusFormulas) with a step size per
 *                               path; Remark "stepSizeControl")
 *
 * As mg_iterated_integrals, with path p split into K[p] sub-intervals of
 * length T/K[p]: coef[p][k] for k < K[p] are that path's weights and
 * coef[p][k] for K[p] <= k < Kmax are zero (a zero step is the identity in
 * mg_magnus_expmv, which then takes K = Kmax for the whole batch).
 *   K       : device int32 [P], each a divisor of Nf in 1 .. Kmax; a path
 *             whose count is not gets NaN weights (and NaN pathstat), which
 *             mg_magnus_expmv flags as non-finite.
 *   coef    : device FP64 [P][Kmax][6] output;  pathstat as in
 *             mg_iterated_integrals (may be NULL).
 * Errors: MG_EINVAL (NULL, T <= 0, order outside 1..3), MG_ESHAPE (P < 0,
 * Kmax < 1, Nf < 1).  P = 0 is a no-op.
 * ------------------------------------------------------------------------ */
mg_status mg_iterated_integrals_steps(const double* dW, int64_t P, int64_t Nf, double T,
                                      const int32_t* K, int32_t Kmax, int32_t order, double* coef,
                                      double* pathstat, void* stream);

/* Bytes of device workspace mg_magnus_expmv needs for P paths and K steps. */
size_t mg_workspace_bytes(const mg_ops* ops, int64_t P, int32_t K, int32_t precision);

/* --------------------------------------------------------------------------
 * mg_magnus_expmv  (Section 2, "Iterated Magnus expansion"; the action of the
 *                   matrix exponential, Section 3 "Implementation")
 *
 * uT[p] = exp(Y_{p,K-1}) ... exp(Y_{p,0}) u0[p], Y_{p,k} = sum_l coef[p][k][l] M_l.
 * Each factor is applied matrix-free by the truncated Taylor series with
 * trace shift mu = tr(Y)/N and s scaling steps chosen from ||Y - mu I||_1
 * (Al-Mohy-Higham thresholds for `tol`), stopping a Taylor sum early once two
 * consecutive terms are below tol * ||partial sum||_inf.
 *   coef      : device, [P][K][6] weights (mg_iterated_integrals layout).
 *   u0        : device FP64, [N] if u0_broadcast != 0 else [P][N].
 *   uT        : device FP64, [P][N] output (may not alias coef or ws).
 *   precision : MG_FP64 or MG_FP32C.
 *   tol       : Taylor tolerance; <= 0 selects 2^-53 (FP64) / 2^-24 (FP32C).
 *   ws        : device workspace of ws_bytes >= mg_workspace_bytes(...),
 *               16-byte aligned (MG_EINVAL otherwise).
 *   stats     : device int32 [P][K][2] = (Taylor terms applied, s), or NULL.
 *   flags     : device int32 [P] (MG_FLAG_* bits), or NULL.
 * Errors: MG_EINVAL, MG_ESHAPE (P < 0, K < 1), MG_EUNSUPPORTED (precision or
 *         size without a kernel), MG_ENOMEM (ws too small), MG_EHIP.
 * P = 0 is a no-op.
 * Coefficients piecewise constant in time (Remark piecewise) take one call
 * per piece: the operators built from that piece's coefficients, the weights
 * of that piece's fine increments (mg_iterated_integrals on a [P][Nf_piece]
 * array with T = the piece's length) and the previous piece's uT as u0.
 * ------------------------------------------------------------------------ */
mg_status mg_magnus_expmv(const mg_ops* ops, const double* coef, int64_t P, int32_t K,
                          const double* u0, int32_t u0_broadcast, double* uT, int32_t precision,
                          double tol, void* ws, size_t ws_bytes, int32_t* stats, int32_t* flags,
                          void* stream);

/* --------------------------------------------------------------------------
 * mg_magnus_expmv_noalloc  (for callers that cannot allocate device memory:
 *                           code under HIP graph capture, tight serving
 *                           loops, harnesses that forbid hipMalloc)
 *
 * mg_magnus_expmv without a workspace argument: the same kernels, with the
 * workspace (per-(path, step) tables and the cooperative exchange area) in a
 * fixed device array of MG_NOALLOC_SCRATCH_BYTES that the library holds on
 * every device it runs on until the process ends.  The call allocates no
 * device or host memory and creates no events (the timing instrumentation
 * does not see it).  Arguments, results and errors as for mg_magnus_expmv;
 * the caller still provides u0, uT, stats and flags.
 *   A call whose mg_workspace_bytes(ops, P, K, precision) exceeds
 *   MG_NOALLOC_SCRATCH_BYTES returns MG_ENOMEM before anything is enqueued.
 *   Every call on one device shares that device's array, and each call
 *   writes all of the array it reads: calls that may overlap on one device
 *   (different streams without ordering between them) race and must not be
 *   issued; calls on one stream are ordered and safe.
 * ------------------------------------------------------------------------ */
#define MG_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
mg_status mg_magnus_expmv_noalloc(const mg_ops* ops, const double* coef, int64_t P, int32_t K,
                                  const double* u0, int32_t u0_broadcast, double* uT,
                                  int32_t precision, double tol, int32_t* stats, int32_t* flags,
                                  void* stream);

/* --------------------------------------------------------------------------
 * mg_autotune_expmv  (kernel shape of the Taylor chain of mg_magnus_expmv)
 *
 * Times the workgroup shapes the library holds for this grid (x points per
 * lane, rows per wave, waves per workgroup; the same rows per workgroup) on
 * the given batch, `reps` launches each, checks that every shape reproduces
 * the default shape's uT bit for bit (they apply the same operations in the
 * same order), and records the fastest in `ops` for `precision`; later
 * mg_magnus_expmv calls with this ops and precision use it.  Arguments as
 * for mg_magnus_expmv (stats and flags are not written); uT is overwritten.
 * Register-resident grids: points per lane, rows per wave and waves per
 * workgroup.  Cooperative grids: the workgroup shapes with the same rows per
 * workgroup (FP64 at nx <= 256 without x-dependent factors, FP32C at
 * 256 < nx <= 512); mg_workspace_bytes covers all of them.  Every candidate
 * must reproduce the default shape's uT bit for bit; one that does not is
 * excluded (reported).  Other operators
 * have one shape: the call records nothing.  The choice also enters the
 * library's autotune cache (mg_autotune_cache_save/load).
 * Unlike the other calls it allocates device memory (a copy of uT) and waits
 * for the stream; do not run it concurrently with other calls that use ops.
 *   reps   : 1..100.
 *   report : host buffer for a one-line summary (may be NULL).
 * Errors: those of mg_magnus_expmv; MG_ESHAPE (P < 1).
 * ------------------------------------------------------------------------ */
mg_status mg_autotune_expmv(mg_ops* ops, const double* coef, int64_t P, int32_t K,
                            const double* u0, int32_t u0_broadcast, double* uT, int32_t precision,
                            double tol, void* ws, size_t ws_bytes, int32_t reps, char* report,
                            size_t report_bytes, void* stream);

/* --------------------------------------------------------------------------
 * mg_autotune_cache_save / mg_autotune_cache_load  (persisted kernel shapes)
 *
 * The library keeps the shapes mg_autotune_expmv picks in a process-wide
 * cache keyed by the device architecture, the grid, the precision, the order
 * and the form of the factored operator (band radii, x-factors, x-terms).
 * mg_build_operators starts every new operator with the cached shapes of its
 * key.  save writes the whole cache to a text file (first line
 * "mg-autotune-cache 1", one entry per line); load merges a file written by
 * save into the cache (operators built earlier are not changed).
 *   path    : host string, the file.
 *   entries : nullable; receives the entries written / read.
 * Errors: MG_EINVAL (NULL path, a file that cannot be opened, a malformed
 *         line: nothing of that file is merged).  Host-only; thread-safe.
 * ------------------------------------------------------------------------ */
mg_status mg_autotune_cache_save(const char* path, int32_t* entries);
mg_status mg_autotune_cache_load(const char* path, int32_t* entries);

/* --------------------------------------------------------------------------
 * mg_magnus_expmv_multi  (the operation of mg_magnus_expmv for several
 *                         independent batches in one call, e.g. groups of
 *                         paths on grids of different sizes)
 *
 * Job i is the mg_magnus_expmv call with the fields of jobs[i] (same meaning,
 * layouts and device pointers) and its own slice of one workspace: the
 * slices follow each other in job order, each rounded up to 256 bytes.
 * Every job is checked before anything is launched: an invalid job fails the
 * whole call (mg_last_error names the job) and no kernel runs.  The jobs then
 * run in order on `stream`.
 *   jobs : host array of njobs descriptors;  ws : device workspace of
 *          ws_bytes >= mg_workspace_bytes_multi(jobs, njobs), 16-byte aligned.
 * Errors: those of mg_magnus_expmv; MG_EINVAL (njobs < 0, NULL jobs).
 * njobs = 0 is a no-op.
 * ------------------------------------------------------------------------ */
typedef struct {
    const mg_ops* ops;
    const double* coef;       /* device [P][K][6] */
    int64_t P;
    int32_t K;
    const double* u0;         /* device FP64 [N] or [P][N] */
    int32_t u0_broadcast;
    double* uT;               /* device FP64 [P][N] */
    int32_t precision;        /* MG_FP64 or MG_FP32C */
    double tol;               /* <= 0: default of the precision */
    int32_t* stats;           /* device [P][K][2] or NULL */
    int32_t* flags;           /* device [P] or NULL */
} mg_job;

/* Total workspace of mg_magnus_expmv_multi (0 for an invalid job list). */
size_t mg_workspace_bytes_multi(const mg_job* jobs, int32_t njobs);

mg_status mg_magnus_expmv_multi(const mg_job* jobs, int32_t njobs, void* ws, size_t ws_bytes,
                                void* stream);

/* --------------------------------------------------------------------------
 * mg_euler_increments  (eq. (EulerMaruyama): Delta W_{t_k} = W_{t_{k+1}} - W_{t_k})
 *
 * dWE[p][n] = sum of the Nf/NE fine increments dW[p][n*Nf/NE .. (n+1)*Nf/NE - 1],
 * the Brownian increment of Euler step n on the same path.
 *   dW  : device FP64 [P][Nf];  dWE : device FP64 [P][NE] output.
 * Errors: MG_EINVAL (NULL), MG_ESHAPE (P < 0, NE < 1, Nf % NE != 0).
 * ------------------------------------------------------------------------ */
mg_status mg_euler_increments(const double* dW, int64_t P, int64_t Nf, int32_t NE, double* dWE,
                              void* stream);

/* --------------------------------------------------------------------------
 * mg_select_magnus_steps  (Remark "stepSizeControl")
 *
 * Chooses a uniform number of Magnus steps for a batch by comparing orders 2
 * and 3 on a sample of paths: for K = K0, K0*factor, K0*factor^2, ... (each
 * dividing Nf and <= Kmax) it runs both orders over the sample with K steps
 * and forms gap(K) = max_p ||u3_p - u2_p||_F / ||u3_p||_F; the first K with
 * gap(K) <= tol is returned with *accepted = 1, else the last K tried with
 * *accepted = 0.  A flagged or non-finite sample path counts as an infinite
 * gap.
 *   ops2, ops3 : operators of orders 2 and 3 on the same grid and
 *                coefficients.
 *   dW         : device FP64 [Ps][Nf], the sample paths' fine increments.
 *   u0         : device FP64 [N], the initial value of every path.
 *   precision  : MG_FP64 or MG_FP32C (both orders run in it).
 *   K_out, gap_out, accepted : host outputs.
 * A set-up call: it allocates its own device buffers and waits for the
 * stream.
 * Errors: MG_EINVAL (NULL, orders not 2 and 3, different grids, K0 not
 * dividing Nf, factor < 2, Kmax < K0, tol <= 0, T <= 0), MG_ESHAPE,
 * MG_EUNSUPPORTED, MG_EHIP.
 * ------------------------------------------------------------------------ */
mg_status mg_select_magnus_steps(const mg_ops* ops2, const mg_ops* ops3, const double* dW,
                                 int64_t Ps, int64_t Nf, double T, const double* u0, int32_t K0,
                                 int32_t factor, int32_t Kmax, double tol, int32_t precision,
                                 int32_t* K_out, double* gap_out, int32_t* accepted,
                                 void* stream);

/* --------------------------------------------------------------------------
 * mg_select_magnus_steps_per_path  (Remark "stepSizeControl", per trajectory)
 *
 * The same ladder as mg_select_magnus_steps, decided per path: every path
 * runs rung K = K0, K0*factor, ... (each dividing Nf and <= Kmax) until its
 * own distance ||u3_p - u2_p||_F / ||u3_p||_F is <= tol; K_out[p] is that K
 * (or the last K tried), gap_out[p] its distance (+inf for a flagged or
 * non-finite path).  The ladder stops once every path is accepted.  The
 * counts feed mg_iterated_integrals_steps, so that one batch runs each path
 * with its own step size.
 *   ops2, ops3 : operators of orders 2 and 3 on the same grid and
 *                coefficients.
 *   dW         : device FP64 [P][Nf];  u0 : device FP64 [N].
 *   K_out      : host int32 [P];  gap_out : host FP64 [P];
 *   n_accepted : host, the number of paths within tol.
 * A set-up call: it allocates its own device buffers and waits for the
 * stream.
 * Errors: as mg_select_magnus_steps.
 * ------------------------------------------------------------------------ */
mg_status mg_select_magnus_steps_per_path(const mg_ops* ops2, const mg_ops* ops3,
                                          const double* dW, int64_t P, int64_t Nf, double T,
                                          const double* u0, int32_t K0, int32_t factor,
                                          int32_t Kmax, double tol, int32_t precision,
                                          int32_t* K_out, double* gap_out, int64_t* n_accepted,
                                          void* stream);

/* --------------------------------------------------------------------------
 * mg_magnus_adaptive  (Remark "stepSizeControl", step by step along each path)
 *
 * Integrates every path with the step size controlled step by step: the
 * horizon is cut into K0 coarse steps of h = T/K0; from the path's state at
 * the start of coarse step k the step is taken as factor^l uniform
 * sub-steps, l = 0, 1, ..., max_level, of orders 2 and 3 with the same
 * (order-3) weights, and the first l whose distance
 * ||u3 - u2||_F / ||u3||_F is <= tol is accepted (at l = max_level the step
 * is accepted whatever its distance); the path continues from u3, and a
 * rejected level is redone from the same state with the step shortened by
 * the factor.  A flagged or non-finite step counts as an infinite distance.
 * Every level runs as one batch over the paths still undecided.
 *   ops2, ops3 : operators of orders 2 and 3 on the same grid and
 *                coefficients.
 *   dW         : device FP64 [P][Nf] fine increments over [0, T].
 *   u0         : device FP64 [N] (u0_broadcast = 1) or [P][N].
 *   uT         : device FP64 [P][N] output.
 *   K0         : coarse steps, dividing Nf; factor >= 2; max_level in 0..20
 *                with factor^max_level dividing Nf/K0.
 *   levels     : host int32 [P][K0] output, the accepted level of each step.
 *   gaps       : host FP64 [P][K0] output, its distance.
 *   precision  : MG_FP64 or MG_FP32C (both orders run in it).
 * A set-up call: it allocates its own device buffers and waits for the
 * stream after every level.
 * Errors: MG_EINVAL (NULL, orders not 2 and 3, different grids, K0 not
 * dividing Nf, factor < 2, max_level out of range or factor^max_level not
 * dividing Nf/K0, tol <= 0, T <= 0), MG_ESHAPE, MG_EUNSUPPORTED, MG_EHIP.
 * ------------------------------------------------------------------------ */
mg_status mg_magnus_adaptive(const mg_ops* ops2, const mg_ops* ops3, const double* dW, int64_t P,
                             int64_t Nf, double T, const double* u0, int32_t u0_broadcast,
                             double* uT, int32_t K0, int32_t factor, int32_t max_level,
                             double tol, int32_t precision, int32_t* levels, double* gaps,
                             void* stream);

/* --------------------------------------------------------------------------
 * mg_euler_step  (eq. (EulerMaruyama))
 *
 * Runs NE Euler-Maruyama steps in place on every path:
 *     u <- u + dt * B u + dWE[p][n] * A u,   n = 0..NE-1,
 * with the B and A of `ops` (built at any order).
 *   u     : device FP64 [P][N], updated in place.
 *   dWE   : device FP64 [P][NE], the Brownian increment of each Euler step.
 *   flags : device int32 [P] or NULL (MG_FLAG_NONFINITE; MG_FLAG_ABORT if
 *           the workgroups sharing a path stopped waiting for each other).
 *   precision must be MG_FP64.
 *   ws    : device workspace of ws_bytes >= mg_euler_workspace_bytes(ops, P)
 *           (the exchange area of grids with nx > 128, where several
 *           workgroups share a path), 16-byte aligned; may be NULL when that
 *           size is 0.
 * Errors: MG_EINVAL, MG_ESHAPE, MG_EUNSUPPORTED (nx > 512), MG_ENOMEM (ws
 * too small), MG_EHIP.  P = 0 or NE = 0 is a no-op.
 * ------------------------------------------------------------------------ */
/* Bytes of device workspace mg_euler_step needs for P paths (0 for grids
 * with nx, nv <= 128; (size_t)-1 if no Euler kernel fits the grid). */
size_t mg_euler_workspace_bytes(const mg_ops* ops, int64_t P);

mg_status mg_euler_step(const mg_ops* ops, double* u, int64_t P, const double* dWE, int32_t NE,
                        double dt, int32_t precision, void* ws, size_t ws_bytes, int32_t* flags,
                        void* stream);

/* --------------------------------------------------------------------------
 * mg_error_vs_exact  (eq. (meanErr); closed form of Section 3.1)
 *
 * err[p] = ||U_ref - U_p||_F / ||U_ref||_F over the central window I^kappa x
 * I^kappa (0-based indices i0 .. i0 + floor(n/2^kappa) - 1 with
 * i0 = floor(n/2 - n/2^(kappa+1)), per axis).  U_ref is uref[p] when uref is
 * not NULL, else the closed-form solution at time ex->T of the SPDE with
 * f^x = -v, g^vv = a, sigma^v = sigma and initial density N(0, s0sq I),
 * evaluated from pathstat[p] = (W_T, int_0^T W).
 *   grid     : host.  ex : host (unused when uref != NULL).
 *   pathstat : device [P][2] (unused when uref != NULL).
 *   u, uref  : device FP64 [P][N].   err : device FP64 [P] output.
 * Errors: MG_EINVAL (NULL, kappa < 0, window empty, sigma^2 >= a),
 *         MG_ESHAPE, MG_EHIP.  The mean over paths (Err) is left to the caller.
 * ------------------------------------------------------------------------ */
mg_status mg_error_vs_exact(const mg_grid* grid, const mg_exact* ex, const double* pathstat,
                            const double* u, const double* uref, int64_t P, int32_t kappa,
                            double* err, void* stream);

/* --------------------------------------------------------------------------
 * mg_check_flags  (per-path failure report of the asynchronous calls)
 *
 * The compute calls are asynchronous, so a non-finite or out-of-range path
 * cannot change their return value; it sets bits in their `flags` array.
 * This call waits for `stream`, reads the P flags and returns MG_ENONFINITE
 * when any path has a bit set (mg_last_error gives the number of flagged
 * paths and the first one), MG_OK otherwise.
 *   flags    : device int32 [P], as written by mg_magnus_expmv,
 *              mg_magnus_expmv_multi or mg_euler_step.
 *   bits_out : host, the OR of all flags (may be NULL).
 *   first_out: host, the first flagged path or -1 (may be NULL).
 * A synchronous check (it waits for the stream); it allocates host memory
 * only.  Errors: MG_EINVAL (NULL flags with P > 0), MG_ESHAPE (P < 0),
 * MG_EHIP, MG_ENOMEM.
 * ------------------------------------------------------------------------ */
mg_status mg_check_flags(const int32_t* flags, int64_t P, int32_t* bits_out, int64_t* first_out,
                         void* stream);

/* Message describing the last failing call on this thread ("" if none). */
const char* mg_last_error(void);

/* --------------------------------------------------------------------------
 * Kernel timing (instrumentation, not part of the method).  While enabled,
 * every launch of the Taylor-chain kernel inside mg_magnus_expmv and of the
 * Euler kernel is bracketed by HIP events recorded on the caller's stream.
 * mg_timing_read synchronises those events and returns the summed kernel
 * time in milliseconds and the number of launches for "expmv" or "euler".
 * Enabling allocates host-side event objects; do not enable under graph
 * capture.
 * ------------------------------------------------------------------------ */
mg_status mg_timing_enable(int32_t on);
mg_status mg_timing_read(const char* kernel, double* total_ms, int64_t* launches);
mg_status mg_timing_reset(void);

/* Library version string. */
const char* mg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MAGNUS_H */
