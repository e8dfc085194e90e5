/*
 * fids.h -- C ABI of the MI355X (gfx950) library for the fast implicit
 * difference scheme (FIDS) of the 1-D time-space fractional diffusion
 * equation with the integral fractional Laplacian:
 *
 *     D_t^gamma u = -kappa(x,t) (-Delta)^{alpha/2} u + f   on (-l, l) x (0, T],
 *     u = 0 outside (-l, l),   u(x, 0) = phi(x)                        (eq. 1.1)
 *
 * Discretisation (Sec. 2.1): N_p = n + 1 spatial intervals, h = 2l/N_p,
 * interior nodes x_i = -l + i h (i = 1..n, array index i-1); graded time
 * levels t_m = T (m/M)^r; graded L1 formula with the sum-of-exponentials
 * (SOE) history of Lemma 2.2 / eq. (2.9); IFL matrix A of eq. (3.16x).
 * Each time level solves the matrix form (3.16gu)
 *
 *     (g b_m I + K_m A) u^m = g [b_m u^{m-1} - sum_j w_j F_j^{(m)}] + f^m,
 *
 * g = 1/Gamma(1-gamma), K_m = diag(kappa(x_i, t_m)), with a Krylov method
 * preconditioned by Strang's circulant (eq. 4.3).
 *
 * Conventions for every entry point:
 *   - Array arguments whose names end in _d are DEVICE pointers (HIP global
 *     memory on the device that is current when the handle is created), owned
 *     by the caller.  kappa_d / f_d / phi_d are BORROWED: the library keeps the
 *     pointers and reads them during fids_step / fids_solve_all /
 *     fids_adjoint, so they must stay alive and unchanged until fids_destroy.
 *   - All device work is enqueued on the hip_stream given at creation (NULL =
 *     the default stream).  Calls that return device results (u_out_d, uT_d,
 *     gradients) enqueue the writes and synchronise the stream before they
 *     return, because they also report a status computed on the device.
 *     A problem (not a batch) whose level launch leaves at least half of the
 *     CUs free also creates one stream of its own (default priority) at
 *     fids_init_problem: fids_step / fids_solve_levels / fids_solve_all build
 *     the per-level symbols of the levels they run there, after the work
 *     already on hip_stream, while the levels run; hip_stream waits for it
 *     before the call returns.  The symbol stream therefore needs free CUs:
 *     other work that fills the device while the levels wait for a symbol
 *     makes the level kernel give up after 4 s (FIDS_EDEVICE).  Such a
 *     caller builds the symbols first with fids_prepare.
 *   - The library never calls hipMalloc: all device memory it uses lives in
 *     the caller's workspace ws_d of at least fids_workspace_size() bytes
 *     (256-byte aligned).  Host memory for the handle and the set-up tables is
 *     allocated with malloc/new and released by fids_destroy.
 *   - Status codes: FIDS_OK = 0 or one of the negative FIDS_E* values below;
 *     no C++ exception crosses the ABI.  A handle is not thread safe; use one
 *     handle per host thread / stream.
 *   - Layouts: kappa_d is [M][n] with row m-1 = kappa(x_i, t_m) when
 *     kappa_time_dependent != 0, else [n]; f_d is [M][n] with row m-1 =
 *     f(x_i, t_m); phi_d and every u vector are [n]; u_all_d is [M+1][n]
 *     with row m = u^m.  All are dense row-major FP64.
 *
 * Tuning overrides read from the environment when a problem or batch is
 * created (for measurement; results do not depend on them beyond rounding
 * order, except where noted):
 *   FIDS_WG          workgroups of a problem when wg_count = 0 (default about
 *                    N_c / 1024, at most 64)
 *   FIDS_TILES       column tiles of the level plan (default: the group size)
 *   FIDS_SKEW        moves factors of two from the column FFT length to the row
 *                    FFT length (default 0)
 *   FIDS_HELPERS     SOE helper workgroups when soe_helpers = -1 (default: as
 *                    many as the solver group has workgroups)
 *   FIDS_BATCH_MODE  "graph": a batch places every member on one workgroup
 *                    and advances by one captured HIP-graph launch per level
 *                    (fids_batch_solve_all from level 0; the graph is captured
 *                    once and replayed) instead of one persistent launch for
 *                    all levels
 *   FIDS_FLOOR_SCALE factor (default 1) on the rounding level up to which a
 *                    stalled true residual is accepted (FIDS_LEVEL_ABOVE_TOL);
 *                    0 accepts only residuals within 4 krylov_tol (changes
 *                    which levels report FIDS_ENOCONV)
 */
#ifndef FIDS_H
#define FIDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define FIDS_OK        0
#define FIDS_EINVAL   -1  /* bad parameter, null pointer, workspace too small     */
#define FIDS_EDEVICE  -2  /* a HIP runtime call failed                             */
#define FIDS_ENOCONV  -3  /* Krylov maxit reached or breakdown; the step is not    */
                          /* advanced and the step info holds iters and relres.    */
                          /* After any failed level, stepping again needs          */
                          /* fids_reset (FIDS_ESTATE until then).                  */
#define FIDS_ENUMERIC -4  /* NaN/Inf met on the device                             */
#define FIDS_ESTATE   -5  /* step after M, adjoint without stored forward states  */

/* ------------------------------------------------------------ knobs */
#define FIDS_BICGSTAB 0   /* right-preconditioned BiCGSTAB (the paper's solver, Sec. 5) */
#define FIDS_FGMRES   1   /* flexible GMRES(restart), right preconditioning          */
#define FIDS_PCG      2   /* conjugate gradients on the symmetrised system           */
                          /* K_m^{-1} M^{(m)} = b_m' K_m^{-1} + A (SPD: K_m diagonal */
                          /* positive, A SPD by Prop. 3.1) with the SPD            */
                          /* preconditioner P^{(m)} / kbar_m (Sec. 4.2 names PCG   */
                          /* for these systems); FIDS_STRANG and FIDS_STRANG_K     */
                          /* are then the same operator, FIDS_NONE is plain CG on  */
                          /* the symmetrised system; stops on the residual of the  */
                          /* original system like the others, then verifies it by  */
                          /* an explicit matvec (a true residual above 4 x tol     */
                          /* restarts CG, at most 3 checks; a level whose true     */
                          /* residual stalls is accepted at its FP64 rounding      */
                          /* floor as described at FIDS_LEVEL_ABOVE_TOL); FP64     */
                          /* only                                                  */
#define FIDS_FP64     0   /* every FFT, vector and reduction in FP64                 */
#define FIDS_MIXED    1   /* preconditioner FFTs in FP32, everything else FP64; a    */
                          /* level unconverged after one restart cycle continues   */
                          /* with the FP64 preconditioner                          */
#define FIDS_STRANG   0   /* Strang circulant preconditioner, eq. (4.3)              */
#define FIDS_NONE     1   /* no preconditioner (identity)                            */
#define FIDS_HISTORY_SOE    0  /* fast history: SOE recurrence (FIDS)              */
#define FIDS_HISTORY_DIRECT 1  /* direct history: full L1 sum (DIDS, eq. 4.1)      */
#define FIDS_STRANG_K 2   /* kappa-scaled Strang: P = K_m C_m, C_m the Strang        */
                          /* circulant of b_m'/kbar_m I + A (same symbols as       */
                          /* FIDS_STRANG, input scaled by kbar_m / kappa_i^m)      */

/* Problem statement (1.1) plus discretisation and solver knobs.
 * Fill with fids_params_default() first, then set what differs. */
typedef struct fids_params {
    double  alpha;        /* IFL order, (0, 2)                                     */
    double  gamma;        /* Caputo order, (0, 1)                                  */
    double  l;            /* half-width of the domain (-l, l), > 0                 */
    double  T;            /* final time, > 0                                       */
    int64_t n;            /* interior unknowns per level (paper: N - 1), >= 1      */
    int64_t M;            /* number of graded time levels, >= 1                    */
    double  r;            /* grading exponent t_m = T (m/M)^r, >= 1                */
    double  mu;           /* splitting parameter of (2.11), (alpha, 2]; 0 selects  */
                          /* 1 + alpha/2; kappa_mu = 2 when mu == 2 else 1         */
    double  soe_tol;      /* relative SOE tolerance on [tau_1, T] (Lemma 2.2)      */
    double  krylov_tol;   /* stop when ||b - M x||_2 <= tol ||b||_2 (BiCGSTAB: its  */
                          /* updated residual; FGMRES, PCG: the true FP64          */
                          /* residual, or that residual's rounding floor with      */
                          /* FIDS_LEVEL_ABOVE_TOL set -- see fids_step_info --     */
                          /* and the true value in fids_step_info.relres)          */
    int32_t krylov_maxit; /* max BiCGSTAB iterations / max FGMRES inner iterations */
                          /* summed over restarts, per time level                  */
    int32_t restart;      /* FGMRES Krylov dimension J (<= 32)                     */
    int32_t solver;       /* FIDS_BICGSTAB | FIDS_FGMRES | FIDS_PCG                */
    int32_t precision;    /* FIDS_FP64 | FIDS_MIXED (MIXED needs FIDS_FGMRES)      */
    int32_t precond;      /* FIDS_STRANG | FIDS_NONE | FIDS_STRANG_K               */
    int32_t kappa_time_dependent; /* 1: kappa_d is [M][n]; 0: kappa_d is [n]      */
    int32_t x0_mode;      /* 0: zero initial guess (Sec. 5); k = 1, 2, 3:          */
                          /* polynomial extrapolation of degree k in t^gamma       */
                          /* through u^{m-1}, ..., u^{m-1-k} (lower degree where   */
                          /* fewer levels exist; the solution's leading term near  */
                          /* t = 0, u^0 + c t^gamma, is linear in t^gamma); the    */
                          /* adjoint extrapolates its solutions backward the same  */
                          /* way                                                   */
    int32_t store_states; /* 1: keep every u^m in the workspace (fids_adjoint     */
                          /* then needs no recomputation); 0: keep only what       */
                          /* stepping needs                                        */
    int32_t wg_count;     /* workgroups that cooperate on one problem; 0 = auto    */
    int32_t soe_helpers;  /* workgroups that stream the history one level ahead   */
                          /* of the solve (the SOE recurrence, or the direct sum   */
                          /* over the stored states): -1 auto (SOE: one per        */
                          /* solver workgroup; direct: every workgroup the solver  */
                          /* group leaves free), 0                                 */
                          /* none, k > 0 at most k (as many as can be resident     */
                          /* beside the group, at most 1024); 0 when               */
                          /* checkpoint_every > 0                                  */
    int32_t history;      /* FIDS_HISTORY_SOE: the fast scheme (sum-of-exponentials */
                          /* history recurrence, Lemma 2.2); FIDS_HISTORY_DIRECT: */
                          /* the direct scheme (4.1), the full graded-L1 sum over */
                          /* every earlier state (keeps all states; O(m n) per    */
                          /* level; no adjoint, no batch)                         */
    int32_t checkpoint_every; /* C > 0: the forward run snapshots its state         */
                          /* (u^{m-1..m-4}, A u^{m-1..m-4}, the SOE history        */
                          /* F^{(m-1)}) at levels m = kC + 1 and fids_adjoint      */
                          /* recomputes each segment of C levels from its          */
                          /* snapshot, bit for bit; 0: no snapshots                */
    int32_t dims;         /* spatial dimensions: 1 (the paper's problem) or 2, the */
                          /* multi-dimensional case its Sec. 6 names: the square   */
                          /* (-l, l)^2 with n interior nodes per axis, so that      */
                          /* kappa_d is [M][n*n] (or [n*n]), f_d [M][n*n], phi_d    */
                          /* and every state [n*n], node (i, j) (x index i) at     */
                          /* i + n j; the IFL matrix is the 2-D form of eq.        */
                          /* (3.16x) (block Toeplitz with Toeplitz blocks; see     */
                          /* fids_ifl2d_coefficients), applied through a padded    */
                          /* 1-D layout of rows of stride S = the smallest power   */
                          /* of two >= 2n - 1, so that S (n - 1) + n <= 2^21;      */
                          /* mu 0 selects the 2-D splitting exponent mu*(alpha)    */
                          /* (fids_ifl2d_mu), an explicit mu must lie in           */
                          /* (alpha, 2)                                            */
} fids_params;

/* Per-level report. */
typedef struct fids_step_info {
    int64_t m;            /* time level 1..M                                       */
    int32_t iters;        /* Krylov iterations (BiCGSTAB: full iterations, a       */
                          /* converged half iteration counts as one)               */
    int32_t matvecs;      /* applications of M^{(m)} (the paper's Its is           */
                          /* matvecs/2 for BiCGSTAB)                               */
    double  relres;       /* final ||b - M x|| / ||b|| as computed by the solver   */
    int32_t pc_fp64_iters;/* FIDS_MIXED: iterations run with the FP64              */
                          /* preconditioner after the first restart cycle missed   */
                          /* the tolerance (0: the level finished in FP32)         */
    int32_t flags;        /* FIDS_LEVEL_* bits                                     */
} fids_step_info;

/* fids_step_info.flags: the level was accepted with relres above krylov_tol.
 * FGMRES and PCG check the true FP64 residual b - M x, which stagnates at a
 * rounding level of about u log2(L) kmax_m ||A||_inf ||x|| / ||b|| (u = 2^-53,
 * L the embedding length, kmax_m = max_i kappa(x_i, t_m)): a level whose true
 * residual stops improving above the tolerance is accepted (FIDS_OK, this
 * flag set) if it is within max(4 krylov_tol, that rounding level), and
 * reported as FIDS_ENOCONV otherwise.  PCG also accepts a true residual within
 * 4 krylov_tol without a stall.  Theorem 3.4 bounds the scheme's error by the
 * SOE and solver tolerances, so flagged levels carry the larger residual. */
#define FIDS_LEVEL_ABOVE_TOL 1

typedef struct fids_problem fids_problem;

/* Fills *p with: alpha 1.5, gamma 0.5, l 1, T 1, n 255, M 64, r 3, mu 0,
 * soe_tol 1e-10, krylov_tol 1e-12, krylov_maxit 200, restart 20, BiCGSTAB,
 * FP64, Strang, kappa_time_dependent 1, x0_mode 0, store_states 0, wg_count 0,
 * soe_helpers -1, history FIDS_HISTORY_SOE, checkpoint_every 0. */
int fids_params_default(fids_params* p);

/* Bytes of device workspace the problem needs (256-byte multiple).
 * FIDS_EINVAL for an invalid parameter set (see fids_init_problem). */
int fids_workspace_size(const fids_params* p, size_t* bytes);

/* Host set-up (Sec. 2.1, 3.1, 4.1) and upload: graded mesh, b_m, SOE nodes
 * and their per-level recurrence factors, the first column of A (3.16x) and
 * its circulant-embedding symbol, the eigenvalues of Strang's s(A), FFT
 * twiddles.  FIDS_EINVAL if alpha not in (0,2), gamma not in (0,1), mu not in
 * (alpha, 2], r < 1, n < 1, M < 1, l <= 0, T <= 0, soe_tol or krylov_tol not
 * in (0, 1), restart not in [1, 32], MIXED without FGMRES, a NULL pointer, or
 * ws_bytes below fids_workspace_size.  On success *out owns host memory
 * released by fids_destroy; the state is at level m = 0 with u^0 = phi. */
int fids_init_problem(const fids_params* p, const double* kappa_d, const double* f_d,
                      const double* phi_d, void* ws_d, size_t ws_bytes, void* hip_stream,
                      fids_problem** out);

/* Advance one level m -> m+1 (eq. 3.15): SOE history update and right-hand
 * side, preconditioned Krylov solve.  u_out_d (may be NULL) receives u^{m+1};
 * info (may be NULL) the level report.  FIDS_ESTATE after level M. */
int fids_step(fids_problem* h, double* u_out_d, fids_step_info* info);

/* Advance `count` levels from the current level m (m -> m + count, each level
 * as in fids_step) in one device launch, 1 <= count <= M - m; the per-level
 * Strang symbols of exactly these levels are built first if they are not
 * built yet (fids_prepare builds all of them).  u_out_d (may be NULL)
 * receives u^{m+count}; per_step (may be NULL) is a host array of `count`
 * entries, entry k for level m + 1 + k.  On a failed level the state stops at
 * the last completed level, per_step holds the reports up to the failed one,
 * and stepping again needs fids_reset.  FIDS_EINVAL for count outside that
 * range, FIDS_ESTATE after level M. */
int fids_solve_levels(fids_problem* h, int64_t count, double* u_out_d, fids_step_info* per_step);

/* Advance from the current level to M in one device launch.  uT_d (may be
 * NULL) receives u^M; u_all_d (may be NULL; needs store_states = 1) receives
 * u^0..u^M; per_step (may be NULL) is a host array of M entries filled for
 * the levels advanced by this call (index m-1). */
int fids_solve_all(fids_problem* h, double* uT_d, double* u_all_d, fids_step_info* per_step);

/* Allocation-free solve, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): fids_init_problem + fids_solve_all + fids_destroy in one call,
 * with the workspace taken from a fixed 64 MiB device array inside the
 * library (each device holds its own copy until the process ends) instead of
 * a caller's buffer.  The call makes no hipMalloc / hipFree; host memory for
 * the set-up tables is allocated and released as in fids_init_problem.
 * Arguments as in fids_init_problem and fids_solve_all: uT_d (may be NULL)
 * receives u^M, per_step (may be NULL) is a host array of M reports.  The
 * problem's workspace (with a 4 MiB batch for the per-level symbols) must fit
 * the array: problems up to about n = 4095 with M = 512 do; larger ones get
 * FIDS_EINVAL with the sizes in fids_last_error().  Calls on one device share
 * the array: this library serialises them within a process (each call clears
 * what it uses and synchronises hip_stream before returning), and calls that
 * overlap on one device from separate processes are not possible because
 * each process has its own array. */
int fids_solve_static(const fids_params* p, const double* kappa_d, const double* f_d, const double* phi_d,
                      double* uT_d, fids_step_info* per_step, void* hip_stream);

/* Exact discrete adjoint of the FIDS steps (eq. 3.16gu with the SOE history
 * recurrence of Lemma 2.2 / eq. 2.9), for a loss J(u^M): given dJ/du^M
 * (dJ_duT_d, [n]) it returns dJ/dkappa (shape of kappa_d: [M][n] or [n]),
 * dJ/df ([M][n], row m-1 for f^m) and dJ/dphi ([n]); any output may be NULL.
 * Backward over m = M..1 it solves the transposed systems
 *     (b_m' I + A K_m) lambda^m = ubar^m,   computed as   lambda^m = K_m^{-1} y,
 *     (b_m' I + K_m A) y = K_m ubar^m       (the same preconditioned solver),
 * runs the history recurrence in reverse (one adjoint history array of the
 * forward's size) and accumulates dJ/dkappa^m_i = -lambda^m_i (A u^m)_i,
 * dJ/df^m = lambda^m, dJ/dphi = ubar^0.  Needs a completed forward run to
 * level M and either store_states = 1 (forward states read back, the forward
 * state stays at level M) or checkpoint_every > 0 (each segment is recomputed
 * from its snapshot; afterwards the forward state is at level
 * min(checkpoint_every, M), and fids_solve_all advances it to M again), else
 * FIDS_ESTATE.  FIDS_ENOCONV / FIDS_ENUMERIC if a transposed solve fails
 * (the outputs are then incomplete).  Synchronous. */
int fids_adjoint(fids_problem* h, const double* dJ_duT_d, double* g_kappa_d,
                 double* g_f_d, double* g_phi_d);

/* The level-m Strang preconditioner as the device builds it (eq. 4.3):
 * P_m = b_m' I + kbar_m s(A), kbar_m the mean of kappa^m and s(A) Strang's
 * circulant of A.  q (host, [n], may be NULL) receives the first column of
 * the n x n circulant P_m^{-1} (a length-n DFT of 1 / (b_m' + kbar_m lam_k)
 * by Bluestein's method; e_0 for FIDS_NONE), which is symmetric, so P_m^{-1}
 * is also the symmetric Toeplitz matrix with first column q; qhat (host,
 * [L/2 + 1], may be NULL) receives the real spectrum of its length-L
 * circulant embedding [q_0, ..., q_{n-1}, 0, ..., 0, q_{n-1}, ..., q_1]
 * through which the solver applies P_m^{-1} (qhat[k] = sum_i e_i
 * cos(2 pi i k / L)).  Rebuilds level m's symbol in place (same values);
 * synchronous; FIDS_EINVAL for m outside 1..M.  For checking. */
int fids_precond_symbol(fids_problem* h, int64_t m, double* q, double* qhat);

/* Host copy of the per-level reports of the last fids_adjoint's transposed
 * solves (M entries, index m-1; relres relative to ||K_m ubar^m||). */
int fids_adjoint_report(const fids_problem* h, fids_step_info* per_step);

/* Back to level 0 (u^0 = phi, empty history).  Set-up tables are kept; the
 * per-level preconditioner symbols are marked stale, so each level's symbol
 * is rebuilt by the call that next advances through it (every solve from
 * level 0 includes that work). */
int fids_reset(fids_problem* h);

/* Builds the per-level Strang preconditioner symbols now (eq. 4.3 for every
 * level: b_m' + kbar_m Lambda inverted through a length-n DFT and re-embedded
 * in the length-L circulant) instead of inside the next step/solve. */
int fids_prepare(fids_problem* h);

/* Release the handle (not the caller's workspace or arrays).  NULL is a no-op. */
int fids_destroy(fids_problem* h);

/* Static message for a status code. */
const char* fids_strerror(int status);

/* The call site and HIP message of the last failed HIP call made by the
 * library in the calling thread ("" if none).  Valid until the next call. */
const char* fids_last_error(void);

/* ---------------- batched problems: independent instances of (1.1) -------- */
typedef struct fids_batch fids_batch;

/* Workspace for `count` problems p[0..count-1] advanced together. */
int fids_batch_workspace_size(const fids_params* p, int32_t count, size_t* bytes);

/* Like fids_init_problem for each problem i with its own parameters p[i] and
 * borrowed arrays kappa_d[i], f_d[i], phi_d[i] (host arrays of device
 * pointers).  All problems must share M, solver and precision (FIDS_EINVAL
 * otherwise); n, alpha, gamma, r, the tolerances, x0_mode, the
 * preconditioner and the fields may differ.  The batch chooses each
 * member's workgroups (fids_batch_groups); store_states, checkpoint_every,
 * soe_helpers and wg_count are ignored. */
int fids_batch_init(const fids_params* p, int32_t count, const double* const* kappa_d,
                    const double* const* f_d, const double* const* phi_d, void* ws_d,
                    size_t ws_bytes, void* hip_stream, fids_batch** out);

/* Advance every problem by one level; info (may be NULL) is [count]. */
int fids_batch_step(fids_batch* b, fids_step_info* info);

/* Advance every problem to level M in one launch; uT_d (may be NULL) is a host
 * array of `count` device pointers receiving u^M; info (may be NULL) is a host
 * array [count][M]. */
int fids_batch_solve_all(fids_batch* b, double* const* uT_d, fids_step_info* info);

/* Advance every problem by `count` levels (1 <= count <= M - level) in one
 * launch (the batch's per-level graph is not used); u_d (may be NULL) is a
 * host array with one device pointer per member (NULL entries skipped) that
 * receive each member's state at the new level; info (may be NULL) is a host
 * array [members][M] of the reports of every level run so far. */
int fids_batch_solve_levels(fids_batch* b, int64_t count, double* const* u_d, fids_step_info* info);

/* Builds every member's per-level Strang preconditioner symbols now (as
 * fids_prepare) instead of inside the next batch step or solve. */
int fids_batch_prepare(fids_batch* b);

/* Per-member status after the last batch call: status[i] (FIDS_OK or the
 * member's failure; a failed member stops while the others go on) and, if
 * last_level is not NULL, the last level member i completed.  Host arrays of
 * `count` entries. */
int fids_batch_status(const fids_batch* b, int32_t* status, int64_t* last_level);

/* Workgroups each member runs on (host array of `count`).  The batch places
 * its members on the co-resident workgroups so that the slowest slot is as
 * short as possible: members whose level costs more than that target get a
 * group of several workgroups, the others are packed into one-workgroup
 * slots that run their members one after another. */
int fids_batch_groups(const fids_batch* b, int32_t* ng);

/* Host-only: the placement fids_batch_init would choose on `resident`
 * co-resident workgroups.  ng[i] is member i's group size and slot[i] its
 * slot (members of a one-workgroup slot run in turn); *makespan (may be NULL)
 * is the modelled cost of the slowest slot, in units of one level of a
 * length-1 embedding on one workgroup. */
int fids_batch_plan(const fids_params* p, int32_t count, int32_t resident, int32_t* ng, int32_t* slot,
                    double* makespan);

/* Autotuner: for every class of members with the same embedding length and
 * group size, times `levels` levels of one member with each candidate
 * column/row tiling (tile counts 1x, 2x, 4x the group, 2048- or 4096-point
 * LDS tiles, within the device's LDS) and gives the whole class the fastest.
 * Needs the batch at level 0; leaves it reset to level 0.  tile_ct (may be
 * NULL) receives each member's chosen columns per tile. */
int fids_batch_tune(fids_batch* b, int32_t levels, int32_t* tile_ct);

/* Back to level 0 for every member (per-level symbols rebuilt on the next call). */
int fids_batch_reset(fids_batch* b);
int fids_batch_destroy(fids_batch* b);

/* ---------------- host-only introspection (no device work) ---------------- */
/* SOE of Lemma 2.2: nodes s[j] and weights w[j] with
 * |t^gamma sum_j w_j e^{-s_j t} - 1| <= tol for t in [delta, T].
 * *count receives the node number; FIDS_EINVAL if it exceeds cap. */
int fids_soe_nodes(double gamma, double delta, double T, double tol, int32_t cap,
                   double* s, double* w, int32_t* count);

/* First column of A, eq. (3.16x), into col[0..n-1]; mu = 0 selects 1+alpha/2. */
int fids_ifl_column(int64_t n, double alpha, double l, double mu, double* col);

/* 2-D operator (dims = 2), for inspection and tests.
 *
 * fids_ifl2d_mu: the splitting exponent mu*(alpha) in (alpha, 2) that the
 *   2-D operator uses when mu = 0: the root of the summed error, over all
 *   unit lattice cells, of the weighted trapezoidal rule applied to the
 *   leading term |eta|^{2-mu} of psi (the requirement that, in 1-D, the
 *   paper's mu = 1 + alpha/2 meets on every interval; Sec. 2.2).  Computed by
 *   the library once per alpha (partial sums over [-K, K]^2, K = 32, 64, 128,
 *   extrapolated in K).  EINVAL unless 0 < alpha < 2.
 * fids_ifl2d_coefficients: a[p + n q], 0 <= p, q < n, the entry of the 2-D
 *   matrix coupling nodes whose indices differ by (+-p, +-q) (a[0] is the
 *   diagonal) on (-l, l)^2 with n interior nodes per axis, h = 2l/(n+1):
 *     A = (c_{2,alpha}/h^alpha) [ D I - sum_{0<|m|_inf<=n-1} W_m |m|^{-mu} S_m ],
 *     W_m = 1/4 sum of int_C |eta|^{mu-2-alpha} over the unit cells C of
 *           [-(n+1), n+1]^2 with corner m,
 *     D   = sum_{0<|m|_inf<=n+1} W_m |m|^{-mu}
 *           + (8/alpha) (n+1)^{-alpha} int_0^{pi/4} cos^alpha t dt
 *   (the splitting of (2.11) with psi averaged over each cell's corners and
 *   omega integrated exactly, and the exact integral beyond the square where
 *   both neighbours lie outside the domain).  mu = 0 selects mu*(alpha).
 *   a holds n*n doubles (host).  EINVAL for n < 1, alpha outside (0, 2),
 *   mu outside (alpha, 2), l <= 0. */
int fids_ifl2d_mu(double alpha, double* mu);
int fids_ifl2d_coefficients(int64_t n, double alpha, double l, double mu, double* a);

/* Eigenvalues of Strang's circulant s(A), lam[k] = sum_j c_S[j] cos(2 pi jk/n). */
int fids_strang_eigs(int64_t n, double alpha, double l, double mu, double* lam);

/* Row m of the direct scheme's history weights (eq. 4.1, 1 <= m <= M <= 65536):
 * w[k], k = 0..m-1, such that b^m = sum_k w[k] u^k + f^m, i.e. w[0] = g a_1^{(m)},
 * w[k] = g (a_{k+1}^{(m)} - a_k^{(m)}) with g = 1 / Gamma(1 - gamma). */
int fids_direct_weights(double gamma, double T, int64_t M, double r, int64_t m, double* w);

/* b_m = tau_m^{-gamma} / Gamma(2-gamma) for m = 1..M into beta[m-1]. */
int fids_level_coefficients(double gamma, double T, int64_t M, double r, double* beta);

#ifdef __cplusplus
}
#endif
#endif /* FIDS_H */
