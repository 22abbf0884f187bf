/*
 * oqp.h -- C-ABI of the batched OCP-QP interior-point solver for MI355X.
 *
 * Problem (paper "HPIPM: a high-performance quadratic programming framework
 * for model predictive control", Section 2.2, the OCP QP without slacks):
 *
 *   min  sum_{n=0}^{N} 1/2 [u_n; x_n]' [[R_n, S_n], [S_n', Q_n]] [u_n; x_n] + r_n'u_n + q_n'x_n
 *   s.t. x_{n+1} = A_n x_n + B_n u_n + b_n,                        n = 0..N-1
 *        lbu_n <= u_n[idxbu_n] <= ubu_n,  lbx_n <= x_n[idxbx_n] <= ubx_n,
 *        lg_n <= D_n u_n + C_n x_n <= ug_n,                        n = 0..N
 *
 * S_n is nu_n x nx_n.  All sizes may vary per stage.  An initial-state
 * constraint x_0 = x0 is written as a box with equal limits (Section 2.2).
 *
 * Solver (Section 3 and Section 4.2): primal-dual interior-point method in the
 * delta formulation of eq:alg:pdipm:delta, Newton systems reduced to
 * eq:alg:kkt and factorized by the square-root Riccati recursion, Mehrotra
 * predictor-corrector with the conditional corrector, primal regularization
 * and lower clamps on multipliers and slacks; optional FP32 factorization
 * corrected by FP64 iterative refinement on the full Newton system
 * (Section 3.4).
 *
 * Memory (Section 1, memory management): the library never allocates.  Every
 * object lives in memory the caller provides, sized by the matching *_bytes
 * call.  Device memory is a caller-owned buffer (for example a byte tensor)
 * and all device work is enqueued on a caller-owned HIP stream.
 *
 * Conventions: matrices are column-major FP64 with an explicit leading
 * dimension; index lists are int32 and 0-based.  Return values: 0 on success,
 * a negative OQP_E* code on a usage or device error (nothing is printed and
 * the process is never aborted; oqp_last_error() describes the failure),
 * OQP_PENDING (1) where documented.
 */
#ifndef OQP_H
#define OQP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define OQP_OK 0
#define OQP_PENDING 1
#define OQP_EINVAL (-1)  /* bad argument: sizes, indices, lo > hi, NULL */
#define OQP_ENOMEM (-2)  /* caller-provided buffer smaller than required */
#define OQP_EDEVICE (-3) /* a HIP call failed */
#define OQP_EBUSY (-4)   /* no capacity to admit a request (serving) */
#define OQP_ESTATE (-5)  /* call out of order (e.g. solve before load) */

/* ---- per-instance solver outcome (oqp_stat.status) --------------------- */
#define OQP_SUCCESS 0  /* all four residual norms within tolerance */
#define OQP_MAX_ITER 1 /* iteration limit reached */
#define OQP_MIN_STEP 2 /* step length fell below alpha_min */
#define OQP_NAN 3      /* a residual norm or the duality measure is NaN */

/* ---- modes ------------------------------------------------------------- */
#define OQP_MODE_F64 0   /* FP64 factorization ("speed" mode, delta formulation); with ir_max > 0 the
                            prediction-centering-correction direction is refined in FP64 (Section
                            3.4: late iterations of ill-conditioned systems) by up to ir_max
                            corrections with the same factors (not with slacks) */
#define OQP_MODE_MIXED 1 /* FP32 factorization + FP64 iterative refinement */
#define OQP_MODE_ABS 2   /* FP64, absolute formulation (eq:alg:pdipm:abs; mode "speed_abs" of Section 4.2):
                            right-hand sides from the data, no residuals in the loop, exit when the
                            duality measure mu <= tol_comp (or on the iteration limit or a too-short
                            step); stat.res holds the residual norms of the returned point */
#define OQP_MODE_ROBUST 3 /* FP64, delta formulation, Riccati factors from an array algorithm (QR of
                             [chol(Phi)'; U]) instead of the Cholesky factor of the normal matrix
                             Phi + U'U (mode "robust" of Section 4.2), and up to ir_max (default 4)
                             refinement steps on the prediction-centering-correction direction;
                             batch only (one-wave variants and block kernel) */
#define OQP_MODE_BALANCE 4 /* FP64, delta formulation (mode "balance" of Section 4.2): Cholesky
                              factors whose accuracy is checked each iteration by the refinement
                              residual of the predictor step; when it exceeds
                              ir_tol * max(1, ||r||_inf) the iteration is factored again with the
                              array algorithm of OQP_MODE_ROBUST (oqp_stat.qr_refactors counts
                              them), and up to ir_max (default 2) refinement steps run on the
                              prediction-centering-correction direction; batch only (one-wave
                              variants and block kernel) */

typedef struct oqp_dims oqp_dims;
typedef struct oqp_qp oqp_qp;
typedef struct oqp_batch oqp_batch;
typedef struct oqp_server oqp_server;
typedef struct oqp_sol oqp_sol;

/* Solver arguments (Section 4.2).  Fill with oqp_arg_default. */
typedef struct {
    int mode;          /* OQP_MODE_* */
    double tol_stat;   /* exit: ||r_g||_inf <= tol_stat */
    double tol_eq;     /* exit: ||r_b||_inf <= tol_eq */
    double tol_ineq;   /* exit: ||r_d||_inf <= tol_ineq */
    double tol_comp;   /* exit: ||lam .* t||_inf <= tol_comp */
    int iter_max;      /* iteration limit */
    double alpha_min;  /* minimum step length */
    double gamma;      /* fraction to the boundary */
    double lam_min;    /* lower clamp on multipliers */
    double t_min;      /* lower clamp on slacks */
    double reg_prim;   /* primal regularization added during factorization */
    double corr_ratio; /* corrector rejected if mu after it > corr_ratio * mu_aff */
    int ir_max;        /* max iterative-refinement corrections per refined direction (Section 3.4);
                          a correction that does not lower ||r_ir||_inf is taken back.  Defaults:
                          4 (mixed, robust), 2 (balance), 0 (F64: no refinement) */
    double ir_tol;     /* refinement stops at ||r_ir||_inf <= ir_tol * max(1, ||r||_inf) */
    int warm_start;    /* batch only (Section 4.2): 0 cold start; 1 primal guess, 2 primal and dual
                          guess, read from the batch's iterate records (see oqp_batch_solve) */
    int cond_N;        /* batch only: solve after partial condensing to this horizon
                          (Section 3.5; min(cond_N, N) stages per instance; 1 = full
                          condensing into one stage of every input); 0 = off */
} oqp_arg;

/* Per-instance result. */
typedef struct {
    int status;        /* OQP_SUCCESS / OQP_MAX_ITER / OQP_MIN_STEP / OQP_NAN */
    int iters;         /* IPM iterations taken */
    int ir_steps;      /* refinement corrections kept in total */
    int fell_back_f64; /* mixed path only: 1 if the FP32 factorization broke down (or the mixed
                          IPM stopped on NaN / a too-short step) and the FP64 kernel finished the
                          instance: from the mixed iterate when that is finite (iters and
                          ir_steps then count both kernels, at most iter_max iterations in all),
                          else from a cold start */
    double mu;         /* duality measure lam't / n_c at the returned iterate */
    double res[4];     /* inf-norms of r_g, r_b, r_d and lam .* t (eq:alg:pdipm:delta) */
    int qr_refactors;  /* balance mode: iterations factored again with the array algorithm */
} oqp_stat;

/* ---- dims (Section 2.2: per-stage nx, nu, nbu, nbx, ng) ---------------- */
/* Bytes for a dims object with horizon N (N >= 1). */
size_t oqp_dims_bytes(int N);
/* Create a dims object in mem (at least oqp_dims_bytes(N) bytes, 8-byte
 * aligned).  All stage sizes start at 0.  OQP_EINVAL for N < 1 or NULL mem,
 * OQP_ENOMEM if bytes is too small. */
int oqp_dims_init(void* mem, size_t bytes, int N, oqp_dims** out);
/* Sizes of stage n (0 <= n <= N): states nx, inputs nu, boxed inputs nbu,
 * boxed states nbx, general rows ng.  Requires nbu <= nu, nbx <= nx. */
int oqp_dims_set_stage(oqp_dims* dims, int n, int nx, int nu, int nbu, int nbx, int ng);
/* Soft constraints of stage n (Section 2.2, the slack variables): ns slack
 * pairs, 0 <= ns <= nbu + nbx + ng (checked again when a QP or a batch is
 * created, in case the stage sizes change afterwards).  Default 0. */
int oqp_dims_set_soft(oqp_dims* dims, int n, int ns);

/* ---- qp data (Section 2.2), copied at set time -------------------------- */
size_t oqp_qp_bytes(const oqp_dims* dims);
/* Create a QP with all data zero.  The dims object must outlive the QP and
 * must not change afterwards. */
int oqp_qp_init(const oqp_dims* dims, void* mem, size_t bytes, oqp_qp** out);
/* A_n (nx_{n+1} x nx_n, lda), B_n (nx_{n+1} x nu_n, ldb), b_n; 0 <= n < N. */
int oqp_qp_set_dyn(oqp_qp* qp, int n, const double* A, int lda, const double* B, int ldb, const double* b);
/* Q_n (nx_n x nx_n, lower triangle read), S_n (nu_n x nx_n), R_n (nu_n x nu_n,
 * lower triangle read), q_n, r_n.  NULL pointers leave the field zero. */
int oqp_qp_set_cost(oqp_qp* qp, int n, const double* Q, int ldq, const double* S, int lds, const double* R, int ldr,
                    const double* q, const double* r);
/* Box on inputs: nbu_n distinct indices into u_n with bounds lo <= hi. */
int oqp_qp_set_box_u(oqp_qp* qp, int n, const int* idx, const double* lo, const double* hi);
/* Box on states: nbx_n distinct indices into x_n with bounds lo <= hi. */
int oqp_qp_set_box_x(oqp_qp* qp, int n, const int* idx, const double* lo, const double* hi);
/* General rows lo <= D_n u_n + C_n x_n <= hi: D (ng_n x nu_n), C (ng_n x nx_n). */
int oqp_qp_set_general(oqp_qp* qp, int n, const double* D, int ldd, const double* C, int ldc, const double* lo,
                       const double* hi);

/* Soft constraints of stage n (Section 2.2): slack j relaxes row idxs[j] of
 * the stage's rows [box u (idxbu order), box x (idxbx order), general] on
 * both sides, the lower row reading G z + s^l_j >= lo and the upper row
 * G z - s^u_j <= hi, with s^l_j >= lls[j], s^u_j >= lus[j] and the cost
 * 1/2 Zl[j] (s^l_j)^2 + zl[j] s^l_j + 1/2 Zu[j] (s^u_j)^2 + zu[j] s^u_j
 * (diagonal Hessians: L2 penalties; linear terms: L1 penalties).  ns_n
 * entries each; rows distinct and in range, Zl, Zu >= 0, all finite, else
 * OQP_EINVAL.  A stage with ns_n = 0 ignores the call. */
int oqp_qp_set_soft(oqp_qp* qp, int n, const int* idxs, const double* Zl, const double* Zu, const double* zl,
                    const double* zu, const double* lls, const double* lus);

/* Getters, the mirror of the setters (Section 1): copies into caller arrays
 * with the given leading dimensions; Q and R are returned in full, box index
 * lists in their stored order.  NULL pointers skip a field. */
int oqp_qp_get_dyn(const oqp_qp* qp, int n, double* A, int lda, double* B, int ldb, double* b);
int oqp_qp_get_cost(const oqp_qp* qp, int n, double* Q, int ldq, double* S, int lds, double* R, int ldr, double* q,
                    double* r);
int oqp_qp_get_box_u(const oqp_qp* qp, int n, int* idx, double* lo, double* hi);
int oqp_qp_get_box_x(const oqp_qp* qp, int n, int* idx, double* lo, double* hi);
int oqp_qp_get_general(const oqp_qp* qp, int n, double* D, int ldd, double* C, int ldc, double* lo, double* hi);
int oqp_qp_get_soft(const oqp_qp* qp, int n, int* idxs, double* Zl, double* Zu, double* zl, double* zu, double* lls,
                    double* lus);

/* ---- arguments ----------------------------------------------------------- */
void oqp_arg_default(oqp_arg* arg, int mode);

/* ---- batch solve on the GPU ---------------------------------------------- */
/* Sizes of the host and device buffers for a batch of `count` instances with
 * the given dims.  Each instance is assigned a kernel (see oqp_set_wave_max);
 * OQP_EINVAL if none covers it. */
int oqp_batch_bytes(const oqp_dims* const* dims, int count, const oqp_arg* arg, size_t* host_bytes,
                    size_t* dev_bytes);
/* Create a batch in caller memory: host_mem (host_bytes, 16-byte aligned),
 * dev_mem (dev_bytes of device memory, 256-byte aligned), stream (a
 * hipStream_t, or NULL for the default stream).  OQP_ENOMEM when a buffer is
 * smaller than oqp_batch_bytes reports.  The dims objects are copied. */
int oqp_batch_init(const oqp_dims* const* dims, int count, const oqp_arg* arg, void* host_mem, size_t host_bytes,
                   void* dev_mem, size_t dev_bytes, void* stream, oqp_batch** out);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): oqp_batch_init
 * without the caller's device buffer.  The batch's device records
 * (descriptors, problem data, iterates, workspace, statuses) go to a static
 * region of OQP_STATIC_DEV_BYTES bytes inside the library's code object, one
 * per GPU, held until the process ends; the caller still passes the host
 * buffer (host_bytes from oqp_batch_bytes) and the stream, and the rest of the
 * batch calls are unchanged.  Nothing is allocated: no hipMalloc or hipFree,
 * here or in the later calls (oqp_batch_set_streams, which creates events, is
 * the one call to leave out).  OQP_ENOMEM, with a message naming both sizes,
 * when the batch needs more device bytes than the region holds.  Every batch
 * created this way on a GPU shares that GPU's region: a new one overwrites the
 * previous one's device records, so use one at a time per GPU; calls whose
 * work overlaps on one GPU race.  The region keeps what the last batch left;
 * the batch writes every record it reads before reading it, as with a caller
 * buffer. */
#define OQP_STATIC_DEV_BYTES (128u << 20)
int oqp_batch_init_static(const oqp_dims* const* dims, int count, const oqp_arg* arg, void* host_mem,
                          size_t host_bytes, void* stream, oqp_batch** out);
/* Pack the QPs (one per instance, dims matching) into the device layout and
 * enqueue the host-to-device copy.  Asynchronous on the batch stream; the host
 * buffer must stay untouched until oqp_batch_sync. */
int oqp_batch_load(oqp_batch* batch, const oqp_qp* const* qps);
/* Enqueue the IPM for every instance (one launch per kernel group present;
 * the block kernel solves its instances of all sizes in one launch, largest
 * first).  Initial point: cold start (y = 0, pi = 0, t = max(C y - d, 1),
 * lam = 1), or with arg.warm_start the iterate records: the last solve's
 * solution, or, if oqp_batch_set_iterate was called since, the host copy of
 * every instance's iterate (uploaded first; instances not set start from what
 * that copy holds, the last fetched solution).  warm_start = 1 keeps u, x and
 * sets the rest as in the cold start at that point; 2 keeps all blocks,
 * clamping multipliers and slacks below at lam_min and t_min.  The mixed
 * path's FP64 fallback continues from the mixed iterate when it is finite.
 * Not combinable with cond_N. */
int oqp_batch_solve(oqp_batch* batch);
/* Extra streams (default priority, caller-owned, at most OQP_BATCH_MAX_AUX)
 * for running kernel groups concurrently: a solve then forks from the batch
 * stream to them and joins back, so its completion is still ordered on the
 * batch stream.  The first group launched stays on the batch stream.  Creates
 * one HIP event per stream plus one; n = 0 returns to a single stream.
 * oqp_batch_release waits for the batch stream and destroys those events (call
 * it before freeing the batch memory when streams were set). */
#define OQP_BATCH_MAX_AUX 8
int oqp_batch_set_streams(oqp_batch* batch, void* const* streams, int n);
int oqp_batch_release(oqp_batch* batch);
/* Replace the arguments used by later solves (mode must not change). */
int oqp_batch_set_arg(oqp_batch* batch, const oqp_arg* arg);
/* Enqueue the device-to-host copy of solutions and statistics. */
int oqp_batch_fetch(oqp_batch* batch);
/* Wait for all work enqueued on the batch stream. */
int oqp_batch_sync(oqp_batch* batch);
/* Results of instance i after fetch + sync.  Solution arrays in the user
 * layout: u (sum nu_n), x (sum nx_n), pi (sum_{n<N} nx_{n+1}; pi_{n+1}
 * multiplies the dynamics n -> n+1), and per-stage constraint vectors
 * lam_l, lam_u, t_l, t_u of length sum(nbu_n + nbx_n + ng_n), ordered per
 * stage [box u (idxbu order), box x (idxbx order), general].  Any pointer may
 * be NULL. */
int oqp_batch_get_stat(const oqp_batch* batch, int i, oqp_stat* stat);
int oqp_batch_get_sol(const oqp_batch* batch, int i, double* u, double* x, double* pi, double* lam_l, double* lam_u,
                      double* t_l, double* t_u);

/* ---- soft constraints (Section 2.2) --------------------------------------- */
/* A batch in which some instance has slacks solves every instance with the
 * soft builds of the kernels (the one-wave variants and the block kernel,
 * chosen by stage size as usual): the FP64 delta formulation, each slack pair
 * eliminated with its bounds row by row (the Riccati recursion sees the row
 * weight w (Z + w_s) / (Z + w + w_s), the slack step follows from the state
 * and input step), cost linear in the number of slacks.  Such a batch needs
 * arg.mode OQP_MODE_F64 and cond_N 0 (OQP_EINVAL otherwise); a warm start's
 * guess includes the slack blocks (oqp_batch_set_soft_iterate, or the last
 * solution): warm_start = 1 keeps u, x, s^l, s^u and sets the rest by the
 * cold-start rule at that point, 2 keeps every block, clamped below;
 * packed requests with slacks take the soft builds too (a kernel group of
 * their own in the server, which must run in the FP64 mode).  The duality
 * measure and
 * oqp_stat.res count the slack rows: r_g includes the slack stationarity
 * rows, r_d the slack bounds, lam .* t their complementarity.
 *
 * Slack blocks of instance i after fetch + sync, each of length sum ns_n,
 * stage by stage in idxs order: s^l, s^u, the multipliers and slacks of
 * s^l >= lls and s^u >= lus.  Any pointer may be NULL; a batch without slacks
 * writes nothing. */
int oqp_batch_get_soft_sol(const oqp_batch* batch, int i, double* s_l, double* s_u, double* lam_sl, double* lam_su,
                           double* t_sl, double* t_su);
/* Slack blocks of the iterate of instance i on the host (after
 * oqp_batch_set_iterate, which clears them): the point of oqp_batch_newton.
 * OQP_ESTATE on a batch without slacks. */
int oqp_batch_set_soft_iterate(oqp_batch* batch, int i, const double* s_l, const double* s_u, const double* lam_sl,
                               const double* lam_su, const double* t_sl, const double* t_su);
/* Slack blocks of the Newton step of instance i (after oqp_batch_newton,
 * fetch + sync). */
int oqp_batch_get_soft_step(const oqp_batch* batch, int i, double* ds_l, double* ds_u, double* dlam_sl,
                            double* dlam_su, double* dt_sl, double* dt_su);
/* Number of slack pairs of instance i (>= 0), or OQP_EINVAL. */
int oqp_batch_nsoft(const oqp_batch* batch, int i);

/* ---- partial condensing (Section 3.5) ------------------------------------ */
/* A batch whose arg has cond_N > 0 solves each instance through partial
 * condensing: oqp_batch_solve first condenses it on the GPU into an OCP QP
 * with N2 = min(cond_N, N) stages, solves that and ends with the expansion,
 * so oqp_batch_get_sol and oqp_batch_fill_sol return the solution of the
 * original QP.  Blocks: the
 * stages [s_b, s_{b+1}) with N = q N2 + r, the first r blocks one stage
 * longer; stage N is the condensed terminal stage.  Condensed stage b has
 * u = [u_{s_b}; ...; u_{s_{b+1}-1}] and x = x_{s_b}; its box list holds the
 * input boxes at their offsets and the box of x_{s_b}, in increasing
 * component order; its general rows are, stage by stage, the state boxes of
 * the later stages of the block (increasing component) and the stage's own
 * general rows.  oqp_batch_get_stat reports the solve of the condensed QP
 * (its residual norms).  The single-Newton-step entries are not available on
 * such a batch (OQP_ESTATE), nor is condensing in the server.
 *
 * Dims of the condensed QP of an instance (caller memory of
 * oqp_pcond_dims_bytes, 8-byte aligned). */
size_t oqp_pcond_dims_bytes(const oqp_dims* dims, int cond_N);
int oqp_pcond_dims(const oqp_dims* dims, int cond_N, void* mem, size_t bytes, oqp_dims** out);
/* Enqueue the device-to-host copy of the condensed QPs (after a solve);
 * after oqp_batch_sync, oqp_batch_get_cond_qp fills a QP created on the dims
 * oqp_pcond_dims reports (OQP_EINVAL if they differ, OQP_ESTATE on a batch
 * without condensing or before the copy). */
int oqp_batch_fetch_cond(oqp_batch* batch);
int oqp_batch_get_cond_qp(const oqp_batch* batch, int i, oqp_qp* out);

/* ---- solution object with per-stage getters (Section 1) ------------------ */
/* Caller memory (16-byte aligned, oqp_sol_bytes) for the solution of a QP with
 * the given dims; the dims object must outlive it. */
size_t oqp_sol_bytes(const oqp_dims* dims);
int oqp_sol_init(const oqp_dims* dims, void* mem, size_t bytes, oqp_sol** out);
/* Copy the result of batch instance i (after fetch + sync) or of a finished
 * server request into sol.  OQP_EINVAL if the stage sizes differ. */
int oqp_batch_fill_sol(const oqp_batch* batch, int i, oqp_sol* sol);
int oqp_server_fill_sol(oqp_server* server, uint64_t ticket, oqp_sol* sol);
/* Stage-n blocks (OQP_ESTATE before a fill): u_n (nu_n), x_n (nx_n), pi (n < N:
 * nx_{n+1} entries, the multiplier of the dynamics n -> n+1); multipliers and
 * slacks of the lower/upper input boxes (nbu_n, idxbu order), state boxes
 * (nbx_n, idxbx order) and general rows (ng_n). */
int oqp_sol_get_u(const oqp_sol* sol, int n, double* out);
int oqp_sol_get_x(const oqp_sol* sol, int n, double* out);
int oqp_sol_get_pi(const oqp_sol* sol, int n, double* out);
int oqp_sol_get_lam_lb_u(const oqp_sol* sol, int n, double* out);
int oqp_sol_get_lam_ub_u(const oqp_sol* sol, int n, double* out);
int oqp_sol_get_lam_lb_x(const oqp_sol* sol, int n, double* out);
int oqp_sol_get_lam_ub_x(const oqp_sol* sol, int n, double* out);
int oqp_sol_get_lam_lg(const oqp_sol* sol, int n, double* out);
int oqp_sol_get_lam_ug(const oqp_sol* sol, int n, double* out);
int oqp_sol_get_t_lb_u(const oqp_sol* sol, int n, double* out);
int oqp_sol_get_t_ub_u(const oqp_sol* sol, int n, double* out);
int oqp_sol_get_t_lb_x(const oqp_sol* sol, int n, double* out);
int oqp_sol_get_t_ub_x(const oqp_sol* sol, int n, double* out);
int oqp_sol_get_t_lg(const oqp_sol* sol, int n, double* out);
int oqp_sol_get_t_ug(const oqp_sol* sol, int n, double* out);
/* Outcome of the filled solve, and its residual norms (stat.res: inf-norms of
 * r_g, r_b, r_d and lam .* t, eq:alg:pdipm:delta). */
int oqp_sol_get_stat(const oqp_sol* sol, oqp_stat* stat);
int oqp_res_get_norms(const oqp_sol* sol, double out[4]);

/* ---- single Newton step (eq:alg:pdipm:delta) ------------------------------ */
/* Set the iterate of instance i on the host (user layout as above; lam and
 * t > 0): the point of oqp_batch_newton, or the guess of a warm-started
 * oqp_batch_solve. */
int oqp_batch_set_iterate(oqp_batch* batch, int i, const double* u, const double* x, const double* pi,
                          const double* lam_l, const double* lam_u, const double* t_l, const double* t_u);
/* Upload the iterates set so far and enqueue one Newton step per instance with
 * r_m = lam .* t - tau (no line search, no update).  After fetch + sync the
 * step is read with oqp_batch_get_step (same layout as the solution). */
int oqp_batch_newton(oqp_batch* batch, double tau);
int oqp_batch_get_step(const oqp_batch* batch, int i, double* du, double* dx, double* dpi, double* dlam_l,
                       double* dlam_u, double* dt_l, double* dt_u);

/* ---- packed requests ------------------------------------------------------ */
/* A QP packed once into a relocatable blob in the device record layout of the
 * kernel variant that covers its stage sizes (header, per-stage sizes,
 * constraint slot map, slack slot map, stage records; the soft layout when
 * the QP has slacks).  The blob is what a serving client hands to
 * oqp_server_submit.  OQP_EINVAL if no variant covers the QP. */
int oqp_pack_bytes(const oqp_qp* qp, size_t* bytes);
/* Pack into mem (64-byte aligned, at least oqp_pack_bytes).  Keep the blob in
 * page-locked memory for asynchronous uploads. */
int oqp_pack(const oqp_qp* qp, void* mem, size_t bytes);
/* Device bytes a packed request occupies while admitted (data, iterate and
 * workspace records: its HBM footprint) and its kernel group (plus the
 * number of kernel groups when the request has slacks). */
int oqp_pack_footprint(const void* packed, size_t* dev_bytes, int* variant);

/* ---- continuous-batching server (device-resident IPM state) --------------- */
/* Requests (packed QPs of any covered size) are admitted when a block of the
 * device arena large enough for their footprint is free (first-fit; freed on
 * release), otherwise submit returns OQP_EBUSY and the caller retries later.
 * oqp_server_progress retires finished launches and, on each idle stream of
 * streams[1..nstreams-1] (one with no launch in flight), launches the queued
 * requests of one kernel group (the oldest request's, at most max_launch per
 * launch): requests that arrive while the device is busy join the next
 * launch, so launches grow with the load and several run at once.
 * streams[0] serves oqp_server_get_sol.
 * The solver arguments (mode included) are fixed at init.  A server is used
 * from one host thread at a time. */
#define OQP_SERVER_MAX_STREAMS 32
typedef struct {
    int max_requests;     /* requests admitted at once (queued, running or finished, not released) */
    int max_launch;       /* requests per kernel launch (1 = one launch per request) */
    int max_groups;       /* launches in flight at once */
    size_t staging_bytes; /* host staging for oqp_server_get_sol: the largest padded iterate */
    int iter_block;       /* 0: each launch solves its requests to the end; K > 0 (FP64 mode): each
                             launch runs at most K IPM iterations, and a request that needs more
                             is queued again (ahead of new arrivals) and continues from its
                             device-resident iterate in a later launch, so arrivals join at
                             iteration-block boundaries; results are bitwise the same */
} oqp_server_cfg;

typedef struct {
    uint64_t submitted;   /* requests admitted */
    uint64_t rejected;    /* submit calls refused with OQP_EBUSY */
    uint64_t completed;   /* requests finished */
    uint64_t launches;    /* kernel launch groups */
    int queued, running, done; /* requests in each state now */
    size_t dev_arena;     /* device bytes available to requests */
    size_t dev_used;      /* device bytes held by admitted requests now */
    size_t dev_peak;      /* high-water mark of dev_used */
} oqp_server_counters;

void oqp_server_cfg_default(oqp_server_cfg* cfg);
/* Host bytes for the server and the fixed device part (launch descriptors and
 * status blocks); the rest of the device buffer given to init is the arena. */
int oqp_server_bytes(const oqp_server_cfg* cfg, size_t* host_bytes, size_t* dev_fixed_bytes);
/* host_mem: page-locked (hipHostMalloc), 64-byte aligned, >= host_bytes
 * (OQP_EINVAL if it is pageable).  dev_mem: 256-byte aligned device buffer.
 * streams: 2..OQP_SERVER_MAX_STREAMS hipStream_t handles owned by the caller.
 * Creates one HIP event per launch slot (released by oqp_server_destroy). */
int oqp_server_init(const oqp_server_cfg* cfg, const oqp_arg* arg, void* host_mem, size_t host_bytes, void* dev_mem,
                    size_t dev_bytes, void* const* streams, int nstreams, oqp_server** out);
/* Wait for all work on the server's streams and destroy its events. */
int oqp_server_destroy(oqp_server* server);
/* Admit a packed request (the blob must stay unchanged until release).
 * OQP_EBUSY when no request slot or device block is free now; OQP_ENOMEM if
 * the request can never fit the arena. */
int oqp_server_submit(oqp_server* server, const void* packed, uint64_t* ticket);
/* Retire finished launches and launch admitted requests; *completed (may be
 * NULL) receives the number of requests finished by this call. */
int oqp_server_progress(oqp_server* server, int* completed);
/* OQP_PENDING until the request has finished, then OQP_OK and its stat. */
int oqp_server_poll(const oqp_server* server, uint64_t ticket, oqp_stat* stat);
/* Seconds from submit to the progress call that saw the request finish. */
int oqp_server_latency(const oqp_server* server, uint64_t ticket, double* seconds);
/* Solution of a finished request (layout as oqp_batch_get_sol); copies the
 * padded iterate from the device on streams[0] and waits for that copy. */
/* Slack blocks of a finished request with slacks (user layout as for
 * oqp_batch_get_soft_sol); a request without slacks writes nothing. */
int oqp_server_get_soft_sol(oqp_server* server, uint64_t ticket, double* s_l, double* s_u, double* lam_sl,
                            double* lam_su, double* t_sl, double* t_su);
int oqp_server_get_sol(oqp_server* server, uint64_t ticket, double* u, double* x, double* pi, double* lam_l,
                       double* lam_u, double* t_l, double* t_u);
/* Free a finished request's device block and slot; the ticket becomes invalid. */
int oqp_server_release(oqp_server* server, uint64_t ticket);
int oqp_server_stats(const oqp_server* server, oqp_server_counters* stats);
/* Replay an arrival schedule in real time on an idle server: request i is
 * submitted once arrival[i] seconds (non-decreasing) have passed since the
 * call began (later while admission is refused), progress is driven in a busy
 * loop, and each finished request is released.  latency[i] = finish time -
 * scheduled arrival.  stat (may be NULL) receives each outcome, wall_s (may be
 * NULL) the elapsed time.  OQP_EDEVICE if no request finishes for timeout_s
 * seconds while some are in flight. */
int oqp_server_replay(oqp_server* server, const void* const* packed, const double* arrival, int count,
                      double timeout_s, double* latency, oqp_stat* stat, double* wall_s);

/* ---- kernels and introspection ---------------------------------------------- */
/* Kernel families: one-wave kernels compiled for fixed padded stage sizes
 * (the "variants"); a 256-thread block kernel with runtime stage sizes (stage
 * blocks nu + nx up to 256, at most 64 inputs and 64 general rows per stage);
 * and, for batches, a wide-stage kernel for stages beyond those limits (any
 * sizes whose LDS vectors fit a CU; FP64 delta formulation only, ir_max 0, no
 * slacks: other modes refuse such instances with OQP_EINVAL), which is what
 * full condensing (cond_N = 1, Section 3.5) produces: its stage-0
 * factorization is the dense Cholesky factorization of the condensed Hessian
 * (Section 3.3).  An instance goes to the cheapest covering variant when that
 * variant's stage block nx_pad + nu_pad is at most the wave bound, else to the
 * block kernel, padded only to its own largest stage, else to the wide-stage
 * kernel.  The bound is process wide and applies to batches and packed
 * requests created after the call. */
int oqp_set_wave_max(int nz); /* 0..64; 0 sends every instance to the block kernel */
int oqp_get_wave_max(void);
/* Variants allowed (bit v for variant v, all by default): an instance whose
 * cheapest covering variant is masked out goes to the block kernel.  Process
 * wide, like the wave bound (the schedule autotuner sets it per kernel
 * group). */
int oqp_set_variant_mask(unsigned mask);
unsigned oqp_get_variant_mask(void);
/* Batches launch a block-kernel group's instances that need more than half a
 * CU's LDS apart from the rest, so the rest can share CUs two by two (1, the
 * default), or every group in one launch (0).  OQP_EINVAL for other values. */
int oqp_set_lds_split(int on);
int oqp_get_lds_split(void);
/* Kernel group of instance i (a variant index < oqp_variant_count(); the six
 * block-kernel builds follow; oqp_variant_count() + 6 is the wide-stage
 * kernel) and its padded stage sizes. */
int oqp_batch_variant(const oqp_batch* batch, int i, int* nx_pad, int* nu_pad, int* ng_pad);
/* Number of compiled one-wave variants and the stage sizes of variant v. */
int oqp_variant_count(void);
int oqp_variant_dims(int v, int* nx_pad, int* nu_pad, int* ng_pad);
/* Message for the last failing call on this thread. */
const char* oqp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* OQP_H */
