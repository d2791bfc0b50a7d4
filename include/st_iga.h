/*
 * st_iga.h -- C ABI of the MI355X space-time isogeometric solver for the
 * monodomain equation with the Rogers-McCulloch ionic model, stabilized by
 * Spline Upwind (Antonietti, Dede, Loli, Montardini, Sangalli, Tesini,
 * "Space-time Isogeometric Analysis of cardiac electrophysiology").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Errors:   every call returns st_iga_status; nothing throws across the ABI.
 *           A per-context message is available from st_iga_last_error.
 * Memory:   the caller owns every device buffer (vectors and the workspace);
 *           the library never allocates device memory.  The opaque context is
 *           host memory owned by the library (freed by st_iga_destroy); on the
 *           first Krylov solve it also takes a 4 KB pinned host buffer, two
 *           HIP events, a capture stream and the Arnoldi step graphs, all
 *           released by st_iga_destroy.
 * Streams:  `stream` is a hipStream_t passed as void*; NULL means the null
 *           stream.  apply/precond only enqueue work; calls that return
 *           scalars (residuals, reports) synchronize that stream.
 * Layout:   a space-time vector of unknowns has N_t * N_s FP64 entries laid
 *           out [N_t][n_d]...[n_1] (x_1 fastest, time slowest: the
 *           colexicographic order of Section 2), N_s = prod n_l, N_t = n_t - 1
 *           (the time functions b_2..b_{n_t} of X_t, Section 2).  "Full"
 *           vectors (u, w) have n_t * N_s entries; time layer 0 holds the
 *           coefficients of b_1, the only time function non-zero at t = 0.
 * Threads:  a context must not be used by two threads at once; different
 *           contexts are independent.
 */
#ifndef ST_IGA_H
#define ST_IGA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct st_iga_ctx st_iga_ctx;

typedef enum {
  ST_IGA_OK = 0,
  ST_IGA_EINVAL = -1,   /* invalid argument (knots, degrees, parameters, sizes, NULL) */
  ST_IGA_ENOMEM = -2,   /* caller workspace smaller than st_iga_workspace_bytes */
  ST_IGA_ENOCONV = -3,  /* iteration limit reached; best iterate written, report filled */
  ST_IGA_EDEVICE = -4,  /* a HIP runtime call failed */
  ST_IGA_ESTATE = -5    /* call out of order (e.g. apply before a linearization) */
} st_iga_status;

typedef enum {
  ST_IGA_FP64 = 0,        /* every kernel in FP64 */
  ST_IGA_MIXED_FP32 = 1,  /* apply/precond in FP32 inside FP64 FGMRES + iterative refinement */
  ST_IGA_MIXED_BF16 = 2   /* FP32 apply, preconditioner with BF16 storage and FP32 arithmetic, same FP64 loop */
} st_iga_precision;

/* Problem statement, paper Section 3, eq. (3.1), and Section 2 (knots, map).
 * Parametric domain (0,1)^d x (0,T) with a separable geometry map (identity
 * by default); homogeneous Neumann boundary conditions; D = diag(sigma). */
typedef struct {
  int32_t d;                 /* spatial dimension, 1..3 */
  int32_t p_s, p_t;          /* spline degrees in space / time, >= 1 */
  int32_t nknots[4];         /* knot-vector lengths: [0..d-1] space, [d] time */
  const double* knots[4];    /* HOST pointers: open knot vectors on [0,1] (Section 2) */
  double T;                  /* final time > 0 (time knots are scaled by T) */
  double Cm;                 /* membrane capacitance > 0 */
  double sigma[3];           /* diffusivities > 0 */
  double a, b, c1, c2, de;   /* Rogers-McCulloch parameters of eq. (3.1), > 0 (c1, c2 >= 0) */
  /* Separable geometry map x_l = F_l(eta_l) of each spatial direction (the
   * spatial part of G = (F, T tau), Section 2, with a diagonal Jacobian):
   * 0 identity (domain (0,1)); 1 affine F = a + (b - a) eta; 2 exponential
   * grading F = a + (b - a) (exp(k eta) - 1) / (exp(k) - 1), with
   * (a, b, k) = map_param[l], a < b, 1e-8 < |k| < 50.  Integrals carry
   * |det DF| = prod_l F_l', gradients 1/F_l', theta's residual the physical
   * Laplacian, and the initial datum, theta's interpolation and the source
   * use physical coordinates (mapped Greville and Gauss points).  The
   * fast-diagonalization preconditioner uses the mapped 1D pencils, which
   * keeps it exact for the constant-coefficient part on such geometries. */
  int32_t map_kind[3];
  double map_param[3][3];
} st_iga_problem;

/* Stimulus: an initial datum u0 (lifted into time layer 0 by sampling at the
 * spatial Greville abscissae) and/or a source f of eq. (3.1), which enters the
 * residual as -int f v and the residual inside theta (eq. (3.6)) as -f, both
 * evaluated at the space-time Gauss points.  The two source kinds are the
 * stimuli of the paper's experiments (Section 4): a characteristic function
 * of a ball times a time window (the 3D test), and a moving Gaussian times a
 * time window (the 2D test).  Times are absolute (0 <= t <= T). */
typedef struct {
  int32_t u0_kind;           /* 0 none, 1 half-space x_1 < u0_center[0], 2 closed ball |x - c| <= r */
  double u0_center[3];
  double u0_radius;
  double u0_value;
  int32_t f_kind;            /* 0 none; 1 f = f_amp on the closed ball |x - f_center| <= f_radius
                                for t in [f_t0, f_t1]; 2 f = f_amp exp(-f_kappa |x - f_center -
                                f_velocity t|^2) for t in [f_t0, f_t1]; 0 elsewhere */
  double f_center[3];
  double f_radius;           /* kind 1: > 0 */
  double f_t0, f_t1;         /* time window, f_t0 <= f_t1 */
  double f_amp;              /* finite */
  double f_kappa;            /* kind 2: > 0 */
  double f_velocity[3];      /* kind 2 */
} st_iga_stimulus;

typedef struct {
  int32_t su;                /* stabilization: 1 the Spline Upwind term of eq. (3.4), 0 none (plain
                                Galerkin), 2 SUPG + shock capturing of Section 4.2.2 (the comparison
                                method for splines of any regularity in time, C^0 included; needs
                                outer = 2): the test function v + tau v_t on the residual
                                C_m u_t - sum_l sigma_l u_ll + C_r u - f (strong form), tau = h/(2p_t+1),
                                plus int sc_c h^2/4 |R(u^k, w^k)| / (C_m (||u^k||_inf/T +
                                ||u^k_t||_inf)) u_t v_t (zero when that denominator is 0), h the
                                length of the time element; C_r and |R| are exact at every Gauss point
                                (the paper low-ranks both) */
  double eps_theta;          /* relative Frobenius tolerance of the theta low rank, eq. (3.9) (paper: 0.1) */
  double eps_react;          /* same tolerance for the reaction coefficient of the Jacobian */
  int32_t max_rank;          /* cap on each low rank (sizes the workspace); a capped rank misses eps
                                and is counted in st_iga_report.rank_capped */
  int32_t outer;             /* 0: Newton (dI_ion/du, low rank), w lagged (w = w(u^k));
                                1: defect-correction Picard with a low-rank C_r of eq. (3.8), w lagged;
                                2: the fixed-point scheme of Section 3.1 as stated: M_R with the exact
                                   C_r(u^k, w^k) at every space-time Gauss point (no low rank; the
                                   coefficient is stored, Q_t x Q_s values), u and w both relaxed with
                                   alpha from w^0 = 0 (solves are written in defect form, equivalent
                                   because C_r(u, w) u = I_ion(u, w)) */
  double alpha;              /* relaxation of the update, in (0, 1] (paper: 0.5 for Picard) */
  double theta_freeze;       /* theta is recomputed while ||delta||_inf > theta_freeze */
  double tol_nonlin;         /* stop when ||delta||_inf <= tol_nonlin */
  double tol_lin;            /* relative true residual of each linear solve */
  double inner_tol;          /* mixed precision: relative residual of each inner FGMRES */
  int32_t restart;           /* FGMRES restart length m (<= 64) */
  int32_t max_outer;         /* nonlinear iteration cap */
  int32_t max_krylov;        /* Krylov iteration cap per linear solve */
  st_iga_precision prec;
  double lin_forcing;        /* > 0: outer iteration k solves to max(tol_lin, min(1e-2, lin_forcing*||delta_{k-1}||_inf)) */
  int32_t coef_slab;         /* time rows per slab of the low-rank operator terms (0: automatic) */
  int32_t reorth;            /* Arnoldi classical Gram-Schmidt (CGS): 2 two passes with the second pass
                                of each basis vector merged into the next step (one multi-dot of V
                                against the new and the previous vector, one fused update: V read
                                twice per step; the last column of a restart cycle keeps one pass),
                                1 two passes in the same step (V read four times), 0 second pass
                                only when the first removes more than 1 - 1/sqrt(2) of the norm.
                                Other values: ST_IGA_EINVAL */
  int32_t graphs;            /* 1: with reorth = 1 or 2, replay each Arnoldi step (preconditioner,
                                operator, Gram-Schmidt) from a HIP graph captured on first use,
                                queueing the next step before the host reads the current one while
                                the residual estimate is far from the tolerance;
                                2: as 1, but with reorth = 2 the next step is always queued ahead
                                (extra work at the end of each cycle; for tests of that path);
                                0: eager launches; EINVAL otherwise */
  int32_t stall_cycles;      /* ENOCONV after this many consecutive FGMRES restart cycles (or
                                refinement steps) that reduce the true residual by less than
                                stall_reduction (relative); 0: never */
  double stall_reduction;    /* in [0, 1) */
  int32_t picard_switch;     /* > 0: a Newton solve (outer = 0) whose ||delta||_inf grows in this many
                                consecutive iterations continues as the outer = 1 Picard iteration
                                (alpha = 0.5); reported in st_iga_report.switched_at; 0: never */
  double sc_c;               /* shock-capturing constant c >= 0 of the su = 2 stabilization (the paper
                                leaves it as a tuning parameter; h is in the time units of T, so the
                                term scales with the square of the element length); 0 turns it off */
  int32_t precond;           /* 0: the fast-diagonalization preconditioner of Section 3.2, eqs.
                                (3.15)-(3.16) (arrowhead time core); 1: the same spatial fast
                                diagonalization with an exact banded LU per spatial mode in time, whose
                                time matrices also carry the time profiles (spatial means at each time
                                Gauss point) of theta's SU term and of the reaction coefficient (floored
                                at a*c1; needs a*c1 > 0 unless su = 2: the per-mode factorization has no
                                pivoting) of the current linearization (refactorized at each
                                linearization); it pays
                                when the front fills a large part of the domain and not when it is
                                localized (the spatial mean of theta is then near zero).  su = 2
                                always uses 1. */
} st_iga_options;

#define ST_IGA_MAX_OUTER_LOG 64
typedef struct {
  int32_t outer_iters;
  int32_t krylov_total;                        /* Krylov iterations summed over linear solves */
  int32_t refinements;                         /* iterative-refinement steps of the last solve */
  int32_t krylov[ST_IGA_MAX_OUTER_LOG];        /* per outer iteration */
  int32_t rank_theta[ST_IGA_MAX_OUTER_LOG];
  int32_t rank_react[ST_IGA_MAX_OUTER_LOG];
  double delta_inf[ST_IGA_MAX_OUTER_LOG];
  double lin_relres[ST_IGA_MAX_OUTER_LOG];     /* FP64 true relative residual of each linear solve */
  double final_delta_inf;
  double seconds_linearize, seconds_krylov;
  int32_t rank_capped;                         /* low ranks cut to max_rank (each misses its tolerance) */
  double lr_relerr_theta[ST_IGA_MAX_OUTER_LOG]; /* achieved ||Theta - U S V^T||_F / ||Theta||_F */
  double lr_relerr_react[ST_IGA_MAX_OUTER_LOG]; /* same for the reaction coefficient */
  int32_t switched_at;                         /* iterations done before a Newton -> Picard switch; -1: none */
} st_iga_report;

/* Defaults: su=1, eps_theta=0.1, eps_react=1e-2, max_rank=48, outer=0,
 * alpha=1 (Newton), theta_freeze=1e-4, tol_nonlin=1e-10, tol_lin=1e-10,
 * inner_tol=1e-4, restart=30, max_outer=60, max_krylov=3000, prec=FP64, lin_forcing=0,
 * coef_slab=0, reorth=2, graphs=1, stall_cycles=10, stall_reduction=1e-3, picard_switch=0, sc_c=0.1, precond=0. */
void st_iga_default_options(st_iga_options* opt);

/* Bytes of device workspace st_iga_setup needs for this problem/options
 * (256-byte aligned sub-buffers included).  Returns 0 on invalid input. */
size_t st_iga_workspace_bytes(const st_iga_problem* prob, const st_iga_options* opt);

/* Build the 1D operators (Section 3.1.1), tau_k (eq. (3.5)) and the
 * fast-diagonalization factors (Section 3.2) on the host in FP64 and upload
 * them into `workspace` (device, >= st_iga_workspace_bytes, 256-byte aligned).
 * Errors: EINVAL for invalid problems (knots not open/non-decreasing on
 * [0,1], interior multiplicity > degree, interior time multiplicity > 1 when
 * su = 1, d not in 1..3, non-positive T/Cm/sigma, NULL pointers);
 * ENOMEM if workspace_bytes is too small; EDEVICE on HIP failures. */
st_iga_status st_iga_setup(const st_iga_problem* prob, const st_iga_options* opt, void* workspace,
                           size_t workspace_bytes, void* stream, st_iga_ctx** out);

/* Linearize at (u, w) (full device vectors): theta of eq. (3.6) on the
 * Greville grid (when su = 1 and refresh_theta != 0), its low rank (eq. (3.9)),
 * the reaction coefficient (Newton: dI_ion/du; Picard: C_r) on the Greville
 * grid and its low rank; the result defines J_k for apply/krylov.  Synchronizes. */
st_iga_status st_iga_linearize(st_iga_ctx* ctx, const double* u, const double* w, int32_t refresh_theta,
                               void* stream);

/* Set J_k directly from low-rank factors given on the Greville grid (HOST
 * pointers): theta ~ sum_r s_r U[:,r] V[:,r]^T with U (N_t x R) and V (N_s x R)
 * row-major, same for the reaction coefficient.  R may be 0.  EINVAL if a
 * rank exceeds max_rank. */
st_iga_status st_iga_set_factors(st_iga_ctx* ctx, int32_t r_theta, const double* U_theta,
                                 const double* s_theta, const double* V_theta, int32_t r_react,
                                 const double* U_react, const double* s_react, const double* V_react);

/* Copy the current low-rank factors to HOST buffers (capacities in entries:
 * U needs N_t*max_rank, V N_s*max_rank, s max_rank).  Ranks are returned. */
st_iga_status st_iga_get_factors(st_iga_ctx* ctx, int32_t* r_theta, double* U_theta, double* s_theta,
                                 double* V_theta, int32_t* r_react, double* U_react, double* s_react,
                                 double* V_react);

/* Take the source of `stim` (its f_* fields; the initial datum is ignored)
 * for every later residual, theta and linearization of this context;
 * st_iga_solve sets it from its own stimulus.  EINVAL for an unknown kind,
 * a non-positive radius or kappa, f_t0 > f_t1 or a non-finite amplitude. */
st_iga_status st_iga_set_stimulus(st_iga_ctx* ctx, const st_iga_stimulus* stim);

/* Theta grid of eq. (3.6) before the low rank (N_t x N_s, device) at (u, w). */
st_iga_status st_iga_theta_grid(st_iga_ctx* ctx, const double* u, const double* w, double* theta,
                                void* stream);

/* y = J_k x on unknown vectors (device).  Section 3.1.1: C_m W_t (x) M_s +
 * M_t (x) K_s + the low-rank SU and reaction terms.  ESTATE before a
 * linearization.  Asynchronous. */
st_iga_status st_iga_apply(st_iga_ctx* ctx, const double* x, double* y, void* stream);

/* z = A-hat^{-1} r (device): the fast-diagonalization preconditioner of
 * eq. (3.15)-(3.16) with sigma-scaled stiffness.  Asynchronous. */
st_iga_status st_iga_precond(st_iga_ctx* ctx, const double* r, double* z, void* stream);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): z = A-hat^{-1} r,
 * the same kernels and result as st_iga_precond, with the preconditioner's
 * three intermediate vectors in a static device array that each GPU the
 * library runs on holds from the library's first use until the process ends
 * (3 x 2^21 FP64 entries, 48 MiB) instead of the context's workspace.  The
 * array's address is resolved per device by st_iga_setup; no device or host
 * memory is allocated and no profiler events are recorded by this call.
 * Every call on one GPU uses that GPU's one array: calls that overlap in time
 * on one GPU (any contexts, any streams) race and give wrong results.  The
 * array needs no clearing (every intermediate is written before it is read).
 * Errors: EINVAL if the problem has more than 2^21 = 2,097,152 unknowns or
 * the context's device is not the current device; EDEVICE if the array's
 * address could not be resolved.  Asynchronous. */
st_iga_status st_iga_precond_noalloc(st_iga_ctx* ctx, const double* r, double* z, void* stream);

/* The same two operators in the context's low precision (FP32; in BF16 mode
 * the preconditioner uses BF16 storage with FP32 arithmetic and the operator
 * stays FP32): FP64 in and out, converted at the boundary.
 * These are the operators of the inner FGMRES of a mixed-precision solve.
 * EINVAL for an FP64 context.  Asynchronous. */
st_iga_status st_iga_apply_lowp(st_iga_ctx* ctx, const double* x, double* y, void* stream);
st_iga_status st_iga_precond_lowp(st_iga_ctx* ctx, const double* r, double* z, void* stream);

/* Residual N(u) (unknown-sized output) of eq. (3.4) at full vectors (u, w) with
 * the current low-rank theta and the exact ionic current at the Gauss points. */
st_iga_status st_iga_residual(st_iga_ctx* ctx, const double* u, const double* w, double* r,
                              void* stream);

/* w-update of Section 3.2: solves L w = g(u) (full vectors; w layer 0 = 0;
 * u and w must not overlap). */
st_iga_status st_iga_w_update(st_iga_ctx* ctx, const double* u, double* w, void* stream);

/* Solve J_k x = b (device, unknown-sized) with right-preconditioned FGMRES
 * (FP64 Arnoldi with re-orthogonalization; the Givens rotations and the
 * least-squares solve run on the device in FP64); in mixed
 * precision, inner FGMRES solves with low-precision apply/precond inside an
 * FP64 iterative refinement on the true residual.  x is overwritten (zero
 * initial guess).  Stops at ||b - J x|| <= tol ||b|| (FP64 true residual).
 * iters/relres may be NULL.  ENOCONV after max_krylov iterations. */
st_iga_status st_iga_krylov(st_iga_ctx* ctx, const double* b, double* x, double tol, int32_t* iters,
                            double* relres, void* stream);

/* Full nonlinear solve (Section 3.1 outer loop): lifts the initial datum,
 * starts from u^0 = datum in every time layer and w^0 = 0, and iterates
 * w-update, linearize, krylov, update until ||delta||_inf <= tol_nonlin.
 * u, w: full device vectors (outputs). */
st_iga_status st_iga_solve(st_iga_ctx* ctx, const st_iga_stimulus* stim, double* u, double* w,
                           st_iga_report* rep, void* stream);

/* One outer iteration from the state u_in (full, device; unchanged unless
 * u_out == u_in): w = w(u) (Section 3.2), linearize (theta refreshed when
 * refresh_theta != 0), r = N(u), solve J delta = -r to relative residual tol,
 * u_out = u_in + alpha delta.  Reports Krylov iterations, the FP64 true
 * relative residual and ||alpha delta||_inf.  Synchronizes. */
st_iga_status st_iga_newton_step(st_iga_ctx* ctx, const double* u_in, double* u_out, double* w,
                                 int32_t refresh_theta, double tol, int32_t* iters, double* relres,
                                 double* delta_inf, void* stream);

/* Kernel-class timing with HIP events recorded around each launch on its
 * stream (process-wide switch).  Classes: 0 other gathers, 1 time mixing of
 * the low-rank terms, 2 arrowhead core, 3 Arnoldi multi-dot, 4 Arnoldi
 * update+norm, 5 pointwise ionic quadrature, 6 element/window maxima,
 * 7 banded mode products (constant part of the operator), 8 spline
 * expansion/projection at Gauss points, 9 dense eigenvector mode products of
 * the preconditioner, 10 fused coefficient terms.  Classes 100 + f + 32 q
 * select one kernel function f
 * (0 scalar gather, 1 4-wide gather, 2 LDS row gather, 3 time mixing,
 * 4 MFMA dense mode product, 5 arrowhead, 6 multi-dot, 7 update+norm,
 * 8 pointwise ionic, 9 maxima, 10 column-sweep gather, 11 fused coefficient
 * terms, 12 fused quadrature pass, 13 dual-table sweep, 14 fused time transforms and arrowhead
 * core of the preconditioner, counted in class 9) in storage precision q (0 FP64, 1 FP32,
 * 2 BF16; the reductions are FP64 only).  profile_read returns the summed duration (ms), the
 * launch count and the summed algorithmic bytes (each input and output array
 * counted once per launch), the summed algorithmic flops (recorded for the
 * time mixing, the fused coefficient kernel and the dense mode products, 0
 * elsewhere) since the last reset, and synchronizes the recorded events.  Any
 * output pointer may be NULL.  profile_record returns launch i (in launch
 * order since the last reset): function id f + 32 q, duration (ms),
 * algorithmic bytes and flops; EINVAL past the last launch. */
st_iga_status st_iga_profile(st_iga_ctx* ctx, int32_t enable);
st_iga_status st_iga_profile_read(st_iga_ctx* ctx, int32_t kernel_class, double* ms, int64_t* launches,
                                  double* bytes, double* flops, int32_t reset);
st_iga_status st_iga_profile_record(st_iga_ctx* ctx, int64_t i, int32_t* fn, double* ms, double* bytes,
                                    double* flops);

/* Lifted initial datum (N_s entries, HOST output) and the number of spatial
 * Greville points inside the stimulus. */
st_iga_status st_iga_lift(st_iga_ctx* ctx, const st_iga_stimulus* stim, double* c0, int64_t* count);

/* Sizes of a context: [d, n_1, n_2, n_3, n_t, N_s, N_t, unknowns(low), unknowns(high)]. */
st_iga_status st_iga_sizes(const st_iga_ctx* ctx, int64_t* out9);

st_iga_status st_iga_destroy(st_iga_ctx* ctx);
const char* st_iga_last_error(const st_iga_ctx* ctx);

/* Host-only queries of the setup (no device needed), for checks of the host
 * logic.  `what`: 0 Greville abscissae of direction dir (n); 1 mass matrix
 * (n*n, full basis); 2 stiffness; 3 time-derivative matrix W[i][j] = int b_j' b_i;
 * 4 tau_k at the time Gauss points (p_t*Q); 5 generalized eigenvalues of
 * (K_l, M_l) (n); 6 eigenvectors U_l (n*n, row-major); 7 time FD: U_t (N_t*N_t)
 * then block values (N_t-1), arrow l (N_t-1), sigma (1); 8 Gauss points of dir
 * (Q) then weights (Q); 9 first-basis index of each Gauss point of dir (Q, as
 * doubles); 10 support-extension element windows of dir ([e0, e1) pairs);
 * 11 plan of the fused coefficient kernel along the slowest spatial axis
 * (dir ignored): {enabled, time rows per slab, nchunk, then nchunk x
 * {first element, end element, first B-spline, end B-spline}}.
 * Writes at most `cap` doubles to out and the needed length to *len. */
st_iga_status st_iga_host_query(const st_iga_problem* prob, int32_t what, int32_t dir, double* out,
                                int64_t cap, int64_t* len);

/* Host-only check of the symmetric eigensolver used for the truncated SVDs of
 * eq. (3.9) (through the N_t x N_t Gram matrix): A (n x n, row-major,
 * symmetric, HOST) = Q diag(lam) Q^T with lam ascending and the eigenvectors
 * in the columns of the row-major Q (n*n, HOST).  ENOCONV if the QL
 * iteration fails. */
st_iga_status st_iga_host_symeig(int32_t n, const double* A, double* Q, double* lam);

#ifdef __cplusplus
}
#endif
#endif /* ST_IGA_H */
