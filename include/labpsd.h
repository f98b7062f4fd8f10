/*
 * labpsd.h -- C ABI of the MI355X (gfx950) LABPSD eigensolver library, liblabpsd.so.
 *
 * LABPSD is the locally accelerated block preconditioned steepest descent method
 * with hybrid (global + locally accelerated) preconditioning of Cai, Bai, Pask and
 * Sukumar, arXiv:1308.2445.  It computes the lowest eigenpairs of a sparse
 * symmetric-definite pencil H x = lambda S x (Section 2, eq. (ghep)) in which H
 * and S share one sparsity pattern (Section 4, footnote to eq. (k1)).
 *
 * Conventions shared by every call
 *   - Status: 0 OK; > 0 warning with valid outputs; < 0 error.  On error the
 *     message is available from labpsd_last_error() (thread-local) and no
 *     output buffer has been written unless the call says otherwise.
 *   - Block vectors are column-major FP64 with an explicit leading dimension
 *     (ld >= number of rows).  "device" pointers are HIP device memory on the
 *     context's device; "host" pointers are ordinary host memory.
 *   - Every call that takes device pointers enqueues its work on the context's
 *     stream and returns without waiting, unless it returns host data (it then
 *     synchronises that stream).  The caller keeps ownership of all buffers it
 *     passes; the library owns the device copies it makes (matrix, factor,
 *     workspaces) and frees them in the matching destroy call.
 *   - A context is used by one host thread at a time.
 *   - No C++ exception crosses this interface.
 */
#ifndef LABPSD_H
#define LABPSD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LABPSD_OK = 0,
    LABPSD_NOT_CONVERGED = 1, /* iteration cap reached; outputs hold the last iterate   */
    LABPSD_EINVAL = -1,       /* invalid argument or input (message says which)         */
    LABPSD_ENOMEM = -2,       /* device or host allocation failed                       */
    LABPSD_EHIP = -3,         /* a HIP runtime call failed                              */
    LABPSD_ENOTSPD = -4,      /* H - eps_bar S is not positive definite                 */
    LABPSD_ERANK = -5,        /* search space [Psi P] lost rank below the block width   */
    LABPSD_PENDING = 2,       /* serving: the request has not finished yet              */
    LABPSD_ESTATE = -6        /* call out of order (e.g. solve before set_global_precond)*/
} labpsd_status;

/* Precision of the preconditioner step (global apply and MINRES refinement).
 * Residuals, products of the search directions, Gram matrices, the
 * S-orthonormalisation and Rayleigh-Ritz are FP64 in both modes.           */
typedef enum { LABPSD_FP64 = 0, LABPSD_MIXED = 1 } labpsd_precision;

/* Which preconditioner acts on the residuals (Section 3 hybrid scheme;
 * Section 5.4 compares the three).                                         */
typedef enum {
    LABPSD_HYBRID = 0,      /* global everywhere, MINRES refinement of localised pairs */
    LABPSD_GLOBAL_ONLY = 1, /* step 6(a) only                                          */
    LABPSD_LOCAL_ONLY = 2   /* localised pairs: MINRES from zero; others global        */
} labpsd_precond_mode;

typedef enum { LABPSD_MEM_HOST = 0, LABPSD_MEM_DEVICE = 1 } labpsd_mem;

typedef struct labpsd_ctx labpsd_ctx;
typedef struct labpsd_problem labpsd_problem;

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device` that enqueues all work on `stream`
 * (a hipStream_t; NULL means the null stream).  The stream is borrowed.     */
labpsd_status labpsd_ctx_create(int device, void* stream, labpsd_ctx** out);
void labpsd_ctx_destroy(labpsd_ctx* ctx);
/* Rebind the context to another stream of the same device. */
labpsd_status labpsd_ctx_set_stream(labpsd_ctx* ctx, void* stream);
/* Message of the last error on this thread ("" if none). */
const char* labpsd_last_error(void);
/* Library version string. */
const char* labpsd_version(void);

/* ------------------------------------------------------------------ problem */

/* Upload the pencil (H, S) (Section 2, eq. (ghep)).  rowptr int64[n+1],
 * col int32[nnz] (per row strictly increasing; the pattern must be structurally
 * symmetric), h_val and s_val float64[nnz] on that one pattern.  `where` says
 * whether the four arrays are host memory or device memory of the context's
 * device (device arrays are read with a synchronous copy on the context's stream:
 * the pattern is validated, the sliced-ELL layout built and, later, the global
 * factorisation computed on the host).  The library copies everything (a
 * sliced-ELL device layout plus FP32 value copies for the mixed-precision
 * preconditioner); the caller may free on return.  EINVAL on n < 1, nnz < n,
 * unsorted/duplicate/out-of-range columns, an empty row or a pattern that is not
 * structurally symmetric.                                                     */
labpsd_status labpsd_problem_create(labpsd_ctx* ctx, int64_t n, int64_t nnz,
                                    const int64_t* rowptr, const int32_t* col,
                                    const double* h_val, const double* s_val, labpsd_mem where,
                                    labpsd_problem** out);
/* Replace the values of H (float64[nnz] on the same pattern, host or device per
 * `where`) for the next GHEP of an SCF-like sequence (Section 2).  S and the
 * global factorisation are kept: the paper builds the global preconditioner once,
 * from the first H (Section 4).                                               */
labpsd_status labpsd_problem_update_h(labpsd_problem* p, const double* h_val, labpsd_mem where);
void labpsd_problem_destroy(labpsd_problem* p);
int64_t labpsd_problem_n(const labpsd_problem* p);

/* The nonlocal part of H (Section 2, eq. (ghep); Section 4, eqs. (k1), (fgf)):
 * H = H_loc + F G F^T with F n x k and G k x k symmetric (k projectors).  F is given by
 * columns: colptr int64[k+1] (colptr[0] = 0), rowidx int32[nnz] (strictly increasing
 * within a column, < n), fval float64[nnz]; G float64[k*k] column-major.  Host arrays,
 * copied.  Every product with H (the solve's H Psi and H P, labpsd_spmm, the shifted
 * products of the refinement) then includes F (G (F^T x)), and the global apply becomes
 * (H_loc + F G F^T - eps_bar S)^{-1} by the Sherman-Morrison-Woodbury steps of Section 4
 * (Fh = (H_loc - eps_bar S)^{-1} F, T = I + G F^T Fh, then P -= Fh T^{-1} G F^T P after
 * every plain apply); the factorisation itself stays that of H_loc - eps_bar S.  The
 * SMW factor is built here if a global preconditioner exists, else by
 * labpsd_set_global_precond (with the FP64 panels when uploaded, else the FP32 ones).
 * k = 0 removes the term.  labpsd_problem_update_h replaces H_loc only.  EINVAL on
 * malformed F, an empty F, k > n, a G that is not symmetric or a singular T.       */
labpsd_status labpsd_problem_set_nonlocal(labpsd_problem* p, int k, const int64_t* colptr,
                                          const int32_t* rowidx, const double* fval,
                                          const double* G);

/* Global preconditioner K = (H - eps_bar S)^{-1} (eq. (globalprecond), eq. (k1p)).
 * Factorises H - eps_bar S once on the host (FP64 supernodal Cholesky after a
 * nested-dissection ordering; eq. (ldl) with 1x1 pivots only, since eps_bar
 * below lambda_1 makes the matrix positive definite) and uploads the factor
 * panels in the precisions that `precisions` selects: LABPSD_PANELS_FP64 (the
 * apply of LABPSD_FP64 solves), LABPSD_PANELS_FP32 (the apply of LABPSD_MIXED
 * solves), or their OR; neither means both.  A solve or apply in a precision whose
 * panels were not uploaded returns ESTATE.  LABPSD_FACTOR_FP32 (ORed in) runs the
 * numeric factorisation itself in single precision (the conclusions' suggestion):
 * fronts, pivots and inverses in FP32; FP64 panels, if uploaded, hold those values.  `coords` (host float64[n*3],
 * row-major x,y,z per dof, or NULL) guides the ordering by coordinate
 * bisection; with NULL a breadth-first level-structure bisection of the graph
 * is used.  LABPSD_APPLY_LEVELS (ORed in) applies the factor with one launch per
 * elimination-tree level and phase instead of the single dependency-ordered
 * launch: the same products, each level's time separately measurable.  ENOTSPD if
 * a pivot is not positive (eps_bar too high); EINVAL for a mask with other bits
 * set.                                                                       */
enum { LABPSD_PANELS_FP64 = 1, LABPSD_PANELS_FP32 = 2, LABPSD_FACTOR_FP32 = 4, LABPSD_APPLY_LEVELS = 8 };
labpsd_status labpsd_set_global_precond(labpsd_problem* p, double eps_bar, const double* coords,
                                        unsigned precisions);

/* Locally accelerated preconditioner parameters (Section 3 remark 4, Section 5):
 * a pair is localised when Res_i <= tau1 and |eps_i - eps_i^prev| <= tau2
 * |eps_i^prev|; its direction is refined by MINRES on (H - eps_i S) p = -r_i
 * (eq. (indls)) until ||(H - eps_i S) p + r_i|| <= eta ||r_i|| (eq. (approxp))
 * or max_inner iterations.  Defaults: 0.1, 0.1, 0.25, 20, HYBRID.           */
labpsd_status labpsd_set_local_precond(labpsd_problem* p, double tau1, double tau2, double eta,
                                       int max_inner, labpsd_precond_mode mode);

/* How localised directions are refined (step 6(b)).  LABPSD_REFINE_MINRES: MINRES on
 * eq. (indls) (Section 4; the default).  LABPSD_REFINE_ONESTEP: the first-order one-step
 * method the conclusions propose instead, p <- p - alpha [(H - eps_i S) p + r_i] with
 * alpha minimising ||(H - eps_i S) p + r_i|| at every step (the bracket read as eq.
 * (idealp)'s residual, + r_i), under the same stopping test (eq. (approxp)) and cap.
 * Applies to labpsd_solve and labpsd_local_refine of this problem.                  */
typedef enum { LABPSD_REFINE_MINRES = 0, LABPSD_REFINE_ONESTEP = 1 } labpsd_refine_method;
labpsd_status labpsd_set_refine_method(labpsd_problem* p, int method);

/* Factor statistics: supernodes, levels, nnz(L), host factorisation seconds. */
typedef struct {
    int64_t n_supernodes;
    int32_t n_levels;
    int64_t nnz_factor;      /* stored entries of L (lower triangles of diagonal blocks + off-diagonal) */
    double flops_factor;     /* host factorisation flops                                                */
    double t_order_s, t_factor_s, t_upload_s;
} labpsd_factor_info;
labpsd_status labpsd_get_factor_info(const labpsd_problem* p, labpsd_factor_info* info);

/* ------------------------------------------------------------------ solve */

typedef struct {
    int nev;              /* m: wanted eigenpairs                                         */
    int m0;               /* guard vectors; block width b = nev + m0 (Section 3 remark 1)  */
    double tol;           /* converged when max_i Res_i <= tol over the first nev (eq. (resL)) */
    int max_outer;        /* outer iteration cap                                          */
    double sigma0;        /* shift in the Res denominator ||(H - sigma0 S) psi|| (Section 5) */
    int precision;        /* labpsd_precision                                             */
    int refresh_every;    /* recompute H Psi, S Psi from H and S every this many iterations */
    int timing;           /* nonzero: time every step with HIP events (stats.t_step_s)      */
    double reorth_tol;    /* at every refresh, Psi^T S Psi is formed from the fresh products;
                           * if max |Psi^T S Psi - I| exceeds this (0: the default 1e-10;
                           * negative: always), Psi is S-orthonormalised again by a
                           * Rayleigh-Ritz step on span(Psi) (Cholesky of Psi^T S Psi) */
    uint64_t seed;        /* start block when X0 is NULL: entry (i, j) is a standard normal
                           * drawn from counter i + n j of this seed (splitmix64 hash,
                           * Box-Muller); the same seed gives the same block           */
} labpsd_solve_params;

typedef struct {
    int outer_iters;          /* outer LABPSD iterations performed                         */
    int64_t minres_iters;     /* total MINRES iterations (M_s of Section 5.2)               */
    int64_t localized_cols;   /* total localised columns refined                           */
    int rank_dropped;         /* search directions dropped by the rank-revealing RR         */
    int refreshes;            /* explicit recomputations of H Psi, S Psi                    */
    double hp;                /* outer iterations per solve (Hp for one GHEP)               */
    double la;                /* M_s / (outer_iters * nev) (La, Section 5.2)                */
    double t_solve_s;         /* wall time inside labpsd_solve                              */
    /* per-step device time (timing != 0), seconds, and kernel launches:
     * 0 products of Psi, 1 residual+Res, 2 global apply, 3 local refinement,
     * 4 products of P, 5 Gram, 6 Rayleigh-Ritz, 7 block update, 8 gather/cast  */
    double t_step_s[12];
    int64_t n_launch[12];
    int64_t n_cols[12];       /* columns processed by each step, summed over its launches */
    int reorths;              /* S-orthonormality restorations (see reorth_tol)            */
} labpsd_stats;

/* Run LABPSD (Section 3 outline) from the start block X0 (n x (nev+m0),
 * column-major, ld n; host or device per in_where), or, with X0 NULL, from the
 * seeded random block that params->seed selects (a cold start: step 1 of the
 * outline with no previous SCF iteration).  E0 (nev+m0 values or
 * NULL) are the previous Ritz values of a warm start; they serve as the
 * previous-iteration values of the first localisation test.
 * Outputs (host or device per out_where, caller-allocated):
 *   lambda[nev] ascending; X n x nev (ld n), S-orthonormal;
 *   res_hist[max_outer * nev] (may be NULL): Res_i at the start of every
 *   iteration, iteration-major; ritz_hist[max_outer * (nev+m0)] (may be NULL):
 *   the Ritz values those Res_i belong to, iteration-major;
 *   *n_hist = iterations recorded (may be NULL).  stats may be NULL.
 * Returns OK, NOT_CONVERGED (outputs hold the last iterate) or an error.
 * Requires labpsd_set_global_precond first (ESTATE otherwise).              */
labpsd_status labpsd_solve(labpsd_problem* p, const labpsd_solve_params* params, const double* X0,
                           const double* E0, labpsd_mem in_where, double* lambda, double* X,
                           double* res_hist, double* ritz_hist, int* n_hist, labpsd_mem out_where,
                           labpsd_stats* stats);

/* ------------------------------------------------------------------ k-points
 * Away from the Gamma point (Section 2's k-point sampling) H and S are complex Hermitian
 * (the paper solves the reduced problem with ZHEGVX).  The library stores such a pencil
 * as its real symmetric embedding: a complex vector x = a + i b is the interleaved real
 * vector (a_0, b_0, a_1, b_1, ...) (the same memory as a column-major complex128 array),
 * entry h of H becomes the 2 x 2 block [Re h, -Im h; Im h, Re h], and every eigenvalue of
 * (H, S) is an eigenvalue of the embedded pencil twice.  Every step of the solve is the
 * real one on the embedded pencil (2n dofs, 2 nev pairs, 2 m0 guards).                */

/* Upload a complex Hermitian pencil: host rowptr int64[n+1], col int32[nnz] as for
 * labpsd_problem_create, and the real and imaginary parts of H and S on that pattern
 * (float64[nnz] each).  EINVAL as labpsd_problem_create, or if H or S is not Hermitian
 * to rounding.  labpsd_set_global_precond then takes coordinates of the n complex dofs
 * and factorises the embedding of H - eps_bar S (Hermitian positive definite below
 * lambda_1).  labpsd_solve refuses such a problem; the nonlocal term is not supported. */
labpsd_status labpsd_problem_create_hermitian(labpsd_ctx* ctx, int64_t n, int64_t nnz, const int64_t* rowptr,
                                              const int32_t* col, const double* h_re, const double* h_im,
                                              const double* s_re, const double* s_im, labpsd_problem** out);
/* New H values (real and imaginary parts, host float64[nnz]) on the same pattern.    */
labpsd_status labpsd_problem_update_h_hermitian(labpsd_problem* p, const double* h_re, const double* h_im);
/* LABPSD for the nev lowest pairs of a Hermitian problem.  X0: complex n x (nev+m0)
 * (interleaved, as a column-major complex128 array; host or device per in_where) or
 * NULL (seeded real start block of the embedding); E0 as labpsd_solve.  Outputs:
 * lambda[nev] ascending; X complex n x nev (interleaved), S-orthonormal (X^H S X = I);
 * res_hist, ritz_hist, n_hist and stats are those of the embedded real solve (2 nev
 * residuals and 2 (nev+m0) Ritz values per iteration).  After the solve, the 2 nev real
 * eigenvectors read as complex vectors span the wanted complex subspace twice over; a
 * Rayleigh-Ritz step on their span (rank-revealing: the nev dominant directions of
 * Z^H S Z) returns it once, its small Hermitian eigenproblems on the host.  ERANK if the
 * span has fewer than nev complex directions.                                         */
labpsd_status labpsd_solve_hermitian(labpsd_problem* p, const labpsd_solve_params* params, const double* X0,
                                     const double* E0, labpsd_mem in_where, double* lambda, double* X,
                                     double* res_hist, double* ritz_hist, int* n_hist, labpsd_mem out_where,
                                     labpsd_stats* stats);

/* ------------------------------------------------------------------ hot-path steps
 * The steps of one LABPSD iteration, each callable on its own for testing and
 * measurement.  All pointers are device pointers; work is enqueued on the
 * context's stream.                                                          */

/* Steps 3 and 7: YH = H X and YS = S X in one pass over the shared pattern.
 * X is n x w (ld ldx), YH and YS n x w (ld ldy).                             */
labpsd_status labpsd_spmm(labpsd_problem* p, const double* X, int64_t ldx, int w, double* YH,
                          double* YS, int64_t ldy);

/* Per-column shifted product Y[:, j] = (H - shift[j] S) X[:, j] (Section 5 shifted
 * matvec, used by the refinement).  precision LABPSD_FP64: X, Y float64 and
 * FP64 values; LABPSD_MIXED: X, Y float32 with FP32 values and accumulation.
 * shift: device float64[w].                                                   */
labpsd_status labpsd_spmm_shifted(labpsd_problem* p, int precision, const void* X, int64_t ldx,
                                  int w, const double* shift, void* Y, int64_t ldy);

/* Step 4 and eq. (res1): R = PsiH[:, :m] - PsiS[:, :m] diag(E[:m]) (n x m, ld ldr),
 * res[i] = ||r_i|| / ||PsiH[:, i] - sigma0 PsiS[:, i]||, rnorm[i] = ||r_i||.
 * E, res, rnorm: device float64[m].                                           */
labpsd_status labpsd_residual(labpsd_ctx* ctx, int64_t n, int m, const double* PsiH,
                              const double* PsiS, int64_t ld, const double* E, double sigma0,
                              double* R, int64_t ldr, double* res, double* rnorm);

/* As labpsd_residual, but allocates nothing: for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid hipMalloc).
 * Its partial sums go to a static device array of 2^17 doubles (1 MiB) that each GPU
 * holds for the life of the process; sizes with 2 * ceil(n / 4096) * m above that
 * return EINVAL.  Every call on one GPU shares the array: calls that overlap on one GPU
 * race.  Pointers and layouts as labpsd_residual; nothing needs clearing first.       */
labpsd_status labpsd_residual_noalloc(labpsd_ctx* ctx, int64_t n, int m, const double* PsiH,
                                      const double* PsiS, int64_t ld, const double* E,
                                      double sigma0, double* R, int64_t ldr, double* res,
                                      double* rnorm);

/* Step 6(a), eq. (k1p): P = -(H - eps_bar S)^{-1} R for p columns (R, P n x p).
 * precision LABPSD_MIXED runs the substitutions in FP32 on FP32 factor panels. */
labpsd_status labpsd_precond_apply(labpsd_problem* p, int precision, const double* R, int64_t ldr,
                                   int ncols, double* P, int64_t ldp);

/* Step 6(b): refine the columns cols[0..q) of P (n x *, ld ldp) in place so that
 * ||(H - shift_j S) p + r|| <= eta ||r||, r the matching column of R (ld ldr),
 * by MINRES on (H - shift_j S) dp = -((H - shift_j S) p + r) (eq. (indls)), or by
 * the one-step method (labpsd_set_refine_method), at most max_inner iterations.  cols: device int32[q] column indices into
 * both P and R; shift: device float64[q]; its: device int32[q] iterations used.
 * precision LABPSD_MIXED runs MINRES in FP32.                                 */
labpsd_status labpsd_local_refine(labpsd_problem* p, int precision, const double* R, int64_t ldr,
                                  double* P, int64_t ldp, int q, const int32_t* cols,
                                  const double* shift, double eta, int max_inner, int32_t* its);

/* Step 8: HR = Z^T ZH and SR = Z^T ZS for k columns (n rows), symmetric parts.
 * Z, ZH, ZS share ld ldz; HR, SR are k x k with ld ldr.                        */
labpsd_status labpsd_gram(labpsd_ctx* ctx, int64_t n, int k, const double* Z, const double* ZH,
                          const double* ZS, int64_t ldz, double* HR, double* SR, int64_t ldr);

/* Step 9 with S-orthonormalisation: lowest nwant eigenpairs of (HR, SR) (k x k):
 * gamma ascending, W (k x nwant, ld ldw) with W^T SR W = I.  SR is scaled to
 * unit diagonal and Cholesky-factorised; if that fails the scaled SR is
 * eigen-decomposed and directions below 1e-14 of its largest eigenvalue are
 * dropped (the rank-revealing step the conclusions call for).  info: device
 * int32[2] = {directions dropped, status (0 ok, -5 rank below nwant)}.
 * k <= 4096.  Orders above 128 run on many work-groups, one of the kernels a
 * cooperative launch (all its work-groups resident at once); if the runtime
 * refuses that launch, or one of its bounded waits runs out, the same result
 * comes from a one-work-group kernel instead.                                  */
labpsd_status labpsd_rayleigh_ritz(labpsd_ctx* ctx, int k, int nwant, const double* HR,
                                   const double* SR, int64_t ldr, double* gamma, double* W,
                                   int64_t ldw, int32_t* info);

/* Steps 10-11: Psi = Z W, PsiH = ZH W, PsiS = ZS W (Z* n x k, W k x b).
 * Outputs must not alias the inputs.                                           */
labpsd_status labpsd_block_update(labpsd_ctx* ctx, int64_t n, int k, int b, const double* Z,
                                  const double* ZH, const double* ZS, int64_t ldz, const double* W,
                                  int64_t ldw, double* Psi, double* PsiH, double* PsiS, int64_t ldo);

/* ------------------------------------------------------------------ serving
 * A request loop for SCF-like streams of GHEPs (Section 2: one GHEP per SCF step,
 * each warm-started from the previous step's Psi, Section 3 remark 1).  Systems
 * (labpsd_problem handles with their global preconditioner set) stay resident: H, S,
 * the factor and the last block Psi.  Requests are admitted as slots and device
 * memory free up (continuous batching: a request that arrives while others run
 * starts as soon as a slot and its footprint fit); every slot runs on its own HIP
 * stream, so the kernels of concurrent requests overlap on the device.  Requests of
 * one system run in submission order, one at a time.  All server calls are
 * thread-safe.                                                                     */
typedef struct labpsd_server labpsd_server;

/* hbm_budget_bytes bounds the device memory the server holds beyond the systems'
 * own storage (H, S, their sliced-ELL layout and factor): every slot keeps its solve
 * workspace between requests, grown to the largest request it ran, and every system
 * it served keeps its last block for the next warm start (charged from its first
 * request on).  A request starts when a slot is free, its system idle and the held
 * bytes plus its growth stay within the budget; idle slots give their workspace back
 * when a request would not fit otherwise.  A request that cannot fit even then, with
 * every slot idle, finishes with ENOMEM.  max_slots (1..64) bounds how many requests
 * run at once.                                                                      */
labpsd_status labpsd_server_create(labpsd_ctx* ctx, size_t hbm_budget_bytes, int max_slots,
                                   labpsd_server** out);
/* Queue one GHEP.  system: a problem with its global preconditioner set (it must
 * outlive the request).  h_val: host float64[nnz] new H values on the system's
 * pattern (NULL keeps the current H).  X0: host n x (nev+m0) start block, or NULL to
 * warm-start from the system's last result (EINVAL if it has none).  Returns at
 * once with *req_id.  ENOMEM if the request's footprint alone exceeds the budget.  */
labpsd_status labpsd_server_submit(labpsd_server* s, labpsd_problem* system, const double* h_val,
                                   const labpsd_solve_params* params, const double* X0,
                                   uint64_t* req_id);
/* Collect a finished request: lambda[nev], X (n x nev, host) and stats may be NULL;
 * times (may be NULL) receives {submitted, started, finished} in seconds since the
 * server was created.  Returns PENDING while it runs (outputs untouched), else the
 * request's solve status; a collected request is forgotten.                        */
labpsd_status labpsd_server_poll(labpsd_server* s, uint64_t req_id, double* lambda, double* X,
                                 labpsd_stats* stats, double* times);
/* As labpsd_server_poll, but blocks until the request has finished.               */
labpsd_status labpsd_server_wait(labpsd_server* s, uint64_t req_id, double* lambda, double* X,
                                 labpsd_stats* stats, double* times);
/* Device bytes one request of this shape needs: its solve workspace plus the
 * resident block it leaves (n x (nev+m0) doubles).                                 */
size_t labpsd_solve_footprint(int64_t n, int nev, int m0, int precision);
/* The device bytes the server holds now (slot workspaces and resident blocks, as
 * charged against the budget) and the most it has held; either may be NULL.         */
labpsd_status labpsd_server_memory(labpsd_server* s, size_t* held, size_t* peak);
/* Stops admitting, waits for running requests, frees the slots.                   */
void labpsd_server_destroy(labpsd_server* s);

#ifdef __cplusplus
}
#endif
#endif /* LABPSD_H */
