/*
 * riot.h - C ABI of the RIOT inner loop of incremental 4D-Var on MI355X (gfx950).
 *
 * Method: Bousserez, Guerrette & Henze, "Enhanced parallelization of the
 * incremental 4D-Var data assimilation algorithm using the Randomized
 * Incremental Optimal Technique (RIOT)", arXiv 1906.01413.
 *
 * Problem statement (Section 2.1, eqs. 2-3): background x_b, B = L L^T with L
 * a symmetric circulant (banded half-kernel l_0..l_w on a periodic grid),
 * observations y of state variables at window steps with diagonal R, forecast
 * model = Lorenz-96 (Section 3.1.1) integrated with RK4. Control variable dz,
 * increment dx = L dz. The prior-preconditioned Hessian (minus I) is
 * A = L^T G^T R^{-1} G L where G stacks the tangent-linear observation
 * Jacobians of the window (Section 2.2, text after eq. 4).
 *
 * Conventions shared by every entry point:
 *  - Device pointers are caller-owned (for example torch tensors). Matrices are
 *    column-major with leading dimension n (state-sized) or m (m x m).
 *  - The caller allocates one device workspace of riot_workspace_bytes() bytes
 *    and passes it to riot_init; the library allocates no device memory of its
 *    own and never frees caller memory. riot_free releases host state only.
 *  - Every call enqueues work on the HIP stream given to riot_init and returns
 *    once enqueued, except where a host output pointer (J_host, dofs_host,
 *    info, used, mode_used) is non-NULL: then the call synchronises the stream
 *    to fill it; and except that the calls running CholeskyQR wait for its pass
 *    decisions (riot_set_pass_sync).
 *  - Errors are returned as riot_status; nothing aborts and no exception
 *    crosses the ABI. Argument errors are detected before any work is
 *    enqueued. Numerical failures detected on the device (breakdown,
 *    non-finite values) are reported by the calls that synchronise.
 *  - One handle per stream; a handle is not re-entrant.
 */
#ifndef RIOT_H
#define RIOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct riot_handle riot_handle;

typedef enum {
    RIOT_OK = 0,
    RIOT_E_ARG = -1,        /* invalid argument or size */
    RIOT_E_HIP = -2,        /* a HIP runtime call failed */
    RIOT_E_NOT_SPD = -3,    /* Cholesky breakdown even after the shifted retry */
    RIOT_E_SINGULAR = -4,   /* singular projected probe matrix Q^T Omega */
    RIOT_E_NONFINITE = -5,  /* NaN or Inf in a result */
    RIOT_E_NOCONV = -6,     /* iteration cap reached (eigen-solver) */
    RIOT_E_STATE = -7,      /* call order violated (e.g. no linearisation yet) */
    RIOT_E_WORKSPACE = -8,  /* workspace too small or misaligned */
    RIOT_E_SCRATCH = -9     /* problem too large for riot_sketch_eig_noalloc's static scratch */
} riot_status;

typedef enum {
    RIOT_FP64 = 0,        /* TL/AD in double precision */
    RIOT_FP32_TLAD = 1    /* TL/AD states in single precision; inputs, outputs and all
                             linear algebra stay double precision */
} riot_precision;

typedef enum {
    RIOT_ADAPTIVE = 0,    /* eq. 11: LRA if the last kept eigenvalue >= 1, else LRU */
    RIOT_LRA = 1,         /* eq. 9 */
    RIOT_LRU = 2          /* eq. 8 */
} riot_update;

/* Problem statement (eqs. 2-3). All pointers are HOST pointers, copied at init. */
typedef struct {
    int32_t n;                 /* state dimension, >= 4 */
    int32_t nsteps;            /* window length T in RK4 steps, >= 0 */
    double dt;                 /* RK4 step */
    double forcing;            /* Lorenz-96 forcing F */
    int32_t nobs;              /* number of observations p, >= 0 */
    const int32_t *obs_step;   /* [nobs] window step of each observation, 0..nsteps */
    const int32_t *obs_idx;    /* [nobs] observed state variable, 0..n-1 */
    const double *y;           /* [nobs] observed values */
    const double *rinv;        /* [nobs] diagonal of R^{-1}, > 0 */
    int32_t l_halfwidth;       /* w >= 0: L has taps at offsets -w..w */
    const double *l_taps;      /* [w+1] half-kernel l_0..l_w of the symmetric circulant L */
    int32_t m_max;             /* largest probe block used with this handle, >= 1 */
    riot_precision prec;       /* precision of the TL/AD integrations */
    int32_t elems_per_lane;    /* 0 = choose automatically, else 1, 2, 4, 8 or 16
                                  (n must be divisible by it; n / it <= 512 for 8 and 16,
                                  <= 1024 otherwise) */
    int32_t ckpt_stride;       /* 0 = the handle stores the whole window's trajectory (every
                                  call); c > 0 = it stores c steps at a time and only the
                                  riot_ckpt_* calls (plus forecast, apply_L, philox) apply */
} riot_desc;

/* Diagnostics of one randomized eigendecomposition (host struct). */
typedef struct {
    int32_t chol_shifts;       /* Cholesky factorisations that were shifted or had a pivot
                                  replaced, over the whole call */
    int32_t qr_passes;         /* CholeskyQR passes applied to the final block Y */
    double k_asym;             /* ||K - K^T||_F / ||K||_F before symmetrisation */
    double orth_err;           /* ||Q^T Q - I||_F after the last pass */
    double kappa_est;          /* (1 + lambda_1) / (1 + max(lambda_m, 0)): condition of I + A on
                                  the sketch's subspace (what an FP64 solve there loses) */
    double resid_est;          /* ||K (Q^T Omega) - Q^T Y||_F / ||Q^T Y||_F with the symmetrised K:
                                  how far the symmetric K is from solving Alg. 3's equation */
} riot_rsvd_info;

/* Bytes of device workspace needed for this problem (0 if the descriptor is invalid). */
size_t riot_workspace_bytes(const riot_desc *desc);

/* Create a handle. `workspace` is a device buffer of at least riot_workspace_bytes(desc)
 * bytes aligned to 256 bytes; it must stay allocated until riot_free. `hip_stream` is a
 * hipStream_t (NULL = default stream). The observation and covariance data are copied to
 * the workspace on that stream. */
riot_status riot_init(const riot_desc *desc, void *workspace, size_t bytes,
                      void *hip_stream, riot_handle **out);

/* Release host state (the workspace stays the caller's). NULL is accepted. */
void riot_free(riot_handle *h);

/* CholeskyQR pass control (the adaptive passes of the orthonormalisation in Alg. 3, see
 * riot_rsvd). on != 0 (the default): the calls that orthonormalise a block (riot_rsvd,
 * riot_orth, riot_block_lanczos) launch the passes that always run, then each further pass
 * only once the previous pass's Cholesky has reported, through a word of pinned host memory
 * that riot_init allocates, that it is needed: the call waits on the device for those
 * reports (not for the pass's triangular solve), so it returns later than the rest of its
 * work is enqueued, and no unneeded pass is launched. on == 0, or while the handle's stream
 * is being captured into a graph: every pass is launched and the unneeded ones return at
 * once on the device; the calls then only enqueue. Results are the same either way.
 * Returns RIOT_E_ARG for a NULL handle. */
riot_status riot_set_pass_sync(riot_handle *h, int32_t on);

/* Human-readable name of a status code (static string). */
const char *riot_status_str(riot_status s);

/* Replace the observed values y (eq. 2) for the next assimilation cycle; locations, error
 * variances and the prior stay. y [nobs] device, in the descriptor's order. The handle
 * must be linearised again before the calls that need it (RIOT_E_STATE otherwise). */
riot_status riot_set_obs(riot_handle *h, const double *y);

/* Outer-loop linearisation at state x (Alg. 3: integrate and store the trajectory,
 * innovation; gradient of eq. 3 at dz = 0).
 *   x    [n]     device, state x_{k-1} to linearise about
 *   v    [n]     device, accumulated control increment v_{k-1}, or NULL for v = 0
 *   d    [nobs]  device out, innovation y - H(M(x)) in the descriptor's order (eq. 3 sign)
 *   grad [n]     device out, g = v - L^T G^T R^{-1} d
 *   J_host       host out or NULL: 1/2 v^T v + 1/2 d^T R^{-1} d (eq. 2 in control variables)
 * Stores the RK4 trajectory in the workspace for the calls below. */
riot_status riot_linearize(riot_handle *h, const double *x, const double *v,
                           double *d, double *grad, double *J_host);

/* riot_linearize with the gradient's adjoint sweep and its L on a second stream of the
 * handle (created on first use, default priority), so that they run beside the calls
 * enqueued next: riot_rsvd and riot_hess_apply need only the trajectory, not the gradient
 * (Alg. 3 uses g only in the increment). d and J_host are complete as for riot_linearize;
 * grad is complete in the handle's stream order after riot_join(h). riot_rsvd,
 * riot_hess_apply, riot_proj_residual and riot_philox_normal do not join; every other call
 * on the handle joins first. v and grad must stay allocated and unmodified until the join. */
riot_status riot_linearize_deferred(riot_handle *h, const double *x, const double *v,
                                    double *d, double *grad, double *J_host);
/* The handle's stream waits for a deferred gradient (no-op when none is pending). */
riot_status riot_join(riot_handle *h);

/* Batched Hessian-probe products (Alg. 3: y_i = A w_i for all probes at once).
 *   m        number of columns, 1..m_max
 *   W [n x m] device, probes (column-major, ld n)
 *   Y [n x m] device out, A W (+ W when add_identity != 0); may not alias W.
 * Requires riot_linearize first (RIOT_E_STATE otherwise). */
riot_status riot_hess_apply(riot_handle *h, int32_t m, const double *W, double *Y,
                            int32_t add_identity);

/* Randomized eigendecomposition of A (Alg. 3 with precond = false).
 * m = k + p_os probes, 1 <= m <= min(m_max, n). Omega [n x m] device or NULL: NULL draws
 * N(0,1) probes with Philox4x32-10 keyed by `seed` (stream 0). q >= 0 power steps:
 * Q0 = orth(Y), Omega_eff = Q0, Y = A Q0 (Halko et al. subspace iteration).
 * Then Q = orth(Y) by CholeskyQR: a shifted first pass, then passes that replace pivots
 * below the shift, repeated on the device until two consecutive passes replace none (at
 * most 8), so that graded or numerically rank-deficient sketches still give an orthonormal
 * Q. K solves K (Q^T Omega_eff) = Q^T Y through the same adaptive CholeskyQR of
 * Q^T Omega_eff carrying Q^T Y, K <- (K + K^T)/2, K = Z diag(lambda) Z^T, V = Q Z.
 *   lambda [m]     device out, Ritz values in descending order
 *   V      [n x m] device out, Ritz vectors
 *   info           host out or NULL (synchronises)
 * Requires riot_linearize first. */
riot_status riot_rsvd(riot_handle *h, int32_t k, int32_t p_os, int32_t q,
                      const double *Omega, uint64_t seed,
                      double *lambda, double *V, riot_rsvd_info *info);

/* Projected residual of a sketch (the quality check of a probe basis, Section 2.2's view of
 * RIOT as finding the dominant invariant subspace of A):
 *   rho = ||A Q - Q (Q^T A Q)||_F / ||A Q||_F
 *   Q  [n x m] device, orthonormal columns (e.g. the Ritz vectors V of riot_rsvd)
 *   AQ [n x m] device, A Q (riot_hess_apply with add_identity = 0)
 *   rho_host   host out (synchronises). 1 <= m <= min(m_max, n). */
riot_status riot_proj_residual(riot_handle *h, int32_t m, const double *Q, const double *AQ,
                               double *rho_host);

/* Adaptive increment (eqs. 8-11 used in eq. 10; Alg. 3 update) from the k leading Ritz pairs:
 *   LRA: dz = -sum_i (1 + l_i)^{-1} v_i v_i^T g
 *   LRU: dz = -(I - sum_i l_i / (1 + l_i) v_i v_i^T) g
 *   lambda [>=k] device, V [n x >=k] device, grad [n] device
 *   dz [n], dx [n] device out (dx = L dz), distinct buffers
 *   dofs_host  host out or NULL: sum_i l_i / (1 + l_i) (degrees of freedom for signal)
 *   mode_used  host out or NULL: RIOT_LRA or RIOT_LRU as applied */
riot_status riot_increment(riot_handle *h, int32_t k, const double *lambda, const double *V,
                           const double *grad, riot_update mode, double *dz, double *dx,
                           double *dofs_host, int32_t *mode_used);

/* Deterministic choice between the two updates (Section 3.2.1, the first-inner-loop
 * discussion of the small black-carbon problem): with the rank-k approximation at hand, form
 * both the LRA and the LRU increment (as riot_increment), integrate the nonlinear model over
 * the window from both updated states x + L dz_c in one launch (one workgroup each), evaluate
 * the non-quadratic cost of eq. 2 in control variables, J_c = 1/2 |v + dz_c|^2
 * + 1/2 (y - H(M(x + L dz_c)))^T R^{-1} (...), and keep the increment with the lower J (LRA on
 * a tie). x must be the state of the current linearisation (x = x_b + L v).
 *   lambda [>=k], V [n x >=k], grad [n], x [n] device; v [n] device or NULL (v = 0)
 *   dz [n], dx [n] device out (dx = L dz), distinct from the inputs
 *   J_host  host out [2] or NULL: J of the LRA and of the LRU candidate (synchronises)
 *   mode_used host out or NULL: RIOT_LRA or RIOT_LRU as kept (synchronises)
 * The handle's stored trajectory is not touched. */
riot_status riot_increment_select(riot_handle *h, int32_t k, const double *lambda,
                                  const double *V, const double *grad, const double *x,
                                  const double *v, double *dz, double *dx, double *J_host,
                                  int32_t *mode_used);

/* Low-rank posterior error covariance in state space (eqs. 8-9, L symmetric):
 *   LRU: P_a = B + W diag(coef) W^T, coef_i = -l_i / (1 + l_i)
 *   LRA: P_a = W diag(coef) W^T,     coef_i = 1 / (1 + l_i)
 * with W = L V[:, :k].
 *   W [n x k] device out, not V; coef [k] device out
 *   diag  [n] device out or NULL: diagonal of P_a
 *   dense [n x n] device out or NULL: P_a itself
 *   mode_used host out or NULL (synchronises when mode is RIOT_ADAPTIVE) */
riot_status riot_posterior_cov(riot_handle *h, int32_t k, const double *lambda, const double *V,
                               riot_update mode, double *W, double *coef, double *diag,
                               double *dense, int32_t *mode_used);

/* Plain conjugate gradients on (I + A) dz = -g from dz = 0 (the iterative baseline of
 * eq. 4 / Alg. 1), all iterations in one device-resident launch.
 *   grad [n] device; iters >= 0; stops early once ||r|| <= rtol ||r_0|| (rtol <= 0: never)
 *   dz [n] device out; iterates [n x iters] device out or NULL (iterate j in column j)
 *   used host out or NULL: iterations performed (synchronises)
 * Requires riot_linearize first. */
riot_status riot_cg(riot_handle *h, const double *grad, int32_t iters, double rtol,
                    double *dz, double *iterates, int32_t *used);

/* Tangent-linear observation operator of the window (Section 2.1: the inner loop needs the
 * TL and AD integrations only, never the full Jacobian): Z = G X, i.e. column j holds H_t M_{0->t} X[:, j] at every
 * observation, in the descriptor's observation order.
 *   X [n x m] device (state space, no L applied), Z [nobs x m] device out (ld nobs).
 * Requires riot_linearize first. 1 <= m <= m_max. */
riot_status riot_tl_apply(riot_handle *h, int32_t m, const double *X, double *Z);

/* Adjoint of riot_tl_apply: X = G^T Fo.
 *   Fo [nobs x m] device (ld nobs), X [n x m] device out. Requires riot_linearize first. */
riot_status riot_ad_apply(riot_handle *h, int32_t m, const double *Fo, double *X);

/* State-space Gauss-Newton product Y = G^T R^{-1} G X (A = L^T (G^T R^{-1} G) L without the
 * L factors): one TL and one AD integration per column, all columns in one launch.
 *   X, Y [n x m] device (may not alias). Requires riot_linearize first. */
riot_status riot_gn_apply(riot_handle *h, int32_t m, const double *X, double *Y);

/* ------------------------------------------------------------------------------------
 * Spectral preconditioner with rotation across outer loops (Alg. 3, precond and rotation
 * branches; eqs. 6-7). After outer loop j the Ritz pairs (V_j, lambda_j) of that loop's
 * preconditioned Hessian define the factor P'_j = I + V_j ((1 + lambda_j)^{-1/2} - 1) V_j^T
 * (inverse: exponent +1/2; V_j orthonormal), and loop k uses P_k = P'_1 ... P'_{k-1}:
 *   A_hat_k = P_k^T (I + A) P_k - I,  b = P_k^T g,  dv = P_k dw,  x_k = x_{k-1} + L dv.
 * Ritz values below zero (rounding: A_hat_k is positive semi-definite) are taken as zero in
 * the factors. The rotation draws the probes as P_k^{-1} (I - U_k U_k^T) omega with U_k an
 * orthonormal basis of [P_1 V_1, ..., P_{k-1} V_{k-1}] (riot_orth, riot_project_out).
 * A level list is nlev host entries: V[j] [n x mj[j]] and lambda[j] [mj[j]] device pointers
 * (mj[j] <= min(n, m_max)); the caller keeps them allocated across the loops.
 * ---------------------------------------------------------------------------------- */
/* X [n x m] device, in place: op 0 = P_k X, 1 = P_k^T X, 2 = P_k^{-1} X (nlev = 0: identity). */
riot_status riot_precond_apply(riot_handle *h, int32_t nlev, const double *const *V,
                               const int32_t *mj, const double *const *lambda, int32_t op,
                               int32_t m, double *X);
/* Y = A_hat_k W = P_k^T (I + A) P_k W - W for m columns (W, Y [n x m] device, distinct);
 * needs riot_linearize first. */
riot_status riot_precond_hess_apply(riot_handle *h, int32_t nlev, const double *const *V,
                                    const int32_t *mj, const double *const *lambda, int32_t m,
                                    const double *W, double *Y);
/* Q [n x m] device out: orthonormal basis of X [n x m] by the adaptive shifted CholeskyQR of
 * riot_rsvd (1 <= m <= min(n, m_max)). */
riot_status riot_orth(riot_handle *h, int32_t m, const double *X, double *Q);
/* X <- (I - U U^T) X in place (two classical Gram-Schmidt passes) for orthonormal U [n x r],
 * X [n x m] device. */
riot_status riot_project_out(riot_handle *h, int32_t r, const double *U, int32_t m, double *X);
/* Outer-loop update: v += dv, x += L dv ([n] device each, distinct). */
riot_status riot_outer_update(riot_handle *h, const double *dv, double *v, double *x);

/* ------------------------------------------------------------------------------------
 * VarBL (Alg. 2): block Lanczos started from l realisations of the gradient.
 * ---------------------------------------------------------------------------------- */
/* One gradient realisation: x_j = x + L eps_b, v_j = v + eps_b (eps_b NULL: the unperturbed
 * sample), observations y_j = y - R^{1/2} eps_o (eq. 3's sign of d), and
 * grad = v_j - L G_j^T R^{-1} (y_j - H(M(x_j))) with G_j at x_j.
 *   x [n], v [n] or NULL (v = 0), eps_b [n] or NULL, eps_o [nobs] device; grad [n] device out.
 * The call integrates the window at x_j in the handle's trajectory storage, so the handle
 * must be linearised again (riot_linearize at x) before the products (RIOT_E_STATE). */
riot_status riot_gradient_sample(riot_handle *h, const double *x, const double *v,
                                 const double *eps_b, const double *eps_o, double *grad);
/* The block Lanczos inner loop of Alg. 2 on A at the current linearisation: Q_1 = orth(B),
 * iters blocks of l Hessian-probe products (one batched launch each), block three-term
 * recurrence with full reorthogonalisation, QR of each residual block (CholeskyQR), the
 * (l iters) x (l iters) block tridiagonal T = Z diag(lambda) Z^T, U = Q Z, and the increment
 * dz = -sum_i (1 + lambda_i)^{-1} u_i u_i^T g, dx = L dz (the LRA form Alg. 2 uses; g is the
 * gradient of the current linearisation).
 *   B [n x l] device: gradient samples; grad [n] device; l iters <= min(n, m_max)
 *   lambda [l iters], U [n x l iters], dz [n], dx [n] device out. */
riot_status riot_block_lanczos(riot_handle *h, int32_t l, int32_t iters, const double *B,
                               const double *grad, double *lambda, double *U, double *dz,
                               double *dx);

/* ------------------------------------------------------------------------------------
 * RIOT-PSAS (Appendix algorithm): the randomized solve in observation space, for windows
 * with fewer observations than controls. A_hat = R^{-1/2} G B G^T R^{-1/2} (p x p, B = L L^T)
 * has the nonzero spectrum of A; the dual increment is
 *   dw = R^{-1/2} M R^{-1/2} (d - b'),  b' = G (x_b - x),  dx = B G^T dw,  x_new = x_b + dx,
 * M = sum (1 + l)^{-1} u u^T (LRA) or I - sum l / (1 + l) u u^T (LRU) from the Ritz pairs of
 * A_hat (eq. 11's rule). The algorithm as printed updates x_{k-1} + B H^T dw; since dw
 * already carries b', that is the Gauss-Newton step only from x_b, which these calls use
 * (the two agree at the first outer loop). The Ritz pairs come from the sketch handle on
 * p-vectors: Y = riot_psas_hess_apply(Omega), riot_sketch_eig(p, m, Omega, Y, ...).
 * All three need riot_linearize first (RIOT_E_STATE otherwise) and nobs >= 1.
 * ---------------------------------------------------------------------------------- */
/* Y = A_hat W for m observation-space probes: W, Y [nobs x m] device (ld nobs), distinct;
 * one AD and one TL integration per column, 1 <= m <= m_max. */
riot_status riot_psas_hess_apply(riot_handle *h, int32_t m, const double *W, double *Y);
/* rhs = R^{-1/2} (d - G (x_b - x)) [nobs] device out; d [nobs] the innovation of the current
 * linearisation (riot_linearize's d); xb_minus_x [n] device, or NULL when x = x_b (b' = 0). */
riot_status riot_psas_rhs(riot_handle *h, const double *d, const double *xb_minus_x,
                          double *rhs);
/* dw [nobs] and dx [n] device out (dx = B G^T dw; the new state is x_b + dx) from the k
 * leading Ritz pairs lambda [>=k], U [nobs x >=k] of A_hat, k <= min(nobs, m_max);
 * mode_used host out or NULL (synchronises). */
riot_status riot_psas_increment(riot_handle *h, int32_t k, const double *lambda, const double *U,
                                const double *rhs, riot_update mode, double *dw, double *dx,
                                int32_t *mode_used);

/* Nonlinear forecast x(nsteps) from x0 with the handle's model (RK4, dt, F).
 * Used to build twin experiments and to cycle analyses. x0, xout [n] device. */
riot_status riot_forecast(riot_handle *h, const double *x0, int32_t nsteps, double *xout);

/* Y = L X for m columns (X, Y [n x m] device; may not alias). */
riot_status riot_apply_L(riot_handle *h, int32_t m, const double *X, double *Y);

/* Philox4x32-10 standard normals: out [n x m] device, entry e = col*n + row; pair j of
 * entries (2j, 2j+1) uses counter (j, stream) and key `seed` (Salmon et al. 2011). */
riot_status riot_philox_normal(riot_handle *h, int32_t n, int32_t m, uint64_t seed,
                               uint64_t stream, double *out);

/* ------------------------------------------------------------------------------------
 * Batches of independent inner-loop problems.
 *
 * Many Lorenz-96 4D-Var problems of different sizes (n a multiple of 8, n <= 2048; window
 * length, observations and B per problem; m = m_max probes per problem, m <= min(n, 278))
 * run the inner loop of Alg. 3 (first outer loop: v = 0, no power steps, all m Ritz pairs,
 * adaptive LRA/LRU update) together:
 *   - trajectories, innovations and gradients: one launch each over all problems;
 *   - the Hessian-probe products of all probes of all problems: one persistent launch
 *     whose workgroups take (problem, member) tiles, longest integrations first; problems
 *     with n <= 512 can run one member per wave instead of one per workgroup;
 *   - CholeskyQR, projections, K, eigen-solve, Ritz vectors, increment: batched launches;
 *   - the whole sequence can be captured once into a HIP graph and replayed.
 * Problem j's data live in batch-owned packed device buffers: vectors (x, grad, dz, dx) at
 * offset sum_{i<j} n_i, lambda at sum_{i<j} m_i, Ritz vectors V (n_j x m_j column-major) at
 * sum_{i<j} n_i m_i, innovations d at sum_{i<j} max(nobs_i, 1). Probes are Philox normals
 * keyed by the run's seed, stream j for problem j (the same draws as riot_philox_normal with
 * that seed and stream).
 * ---------------------------------------------------------------------------------- */
typedef struct riot_batch riot_batch;

typedef struct {
    double *x;       /* [sum n] device in: linearisation state of every problem */
    double *grad;    /* [sum n] device out: gradient g_j (eq. 3, v = 0) */
    double *lambda;  /* [sum m] device out: Ritz values, descending per problem */
    double *V;       /* [sum n m] device out: Ritz vectors */
    double *dz;      /* [sum n] device out: control increment */
    double *dx;      /* [sum n] device out: state increment L dz */
    double *d;       /* [sum max(nobs,1)] device out: innovations */
} riot_batch_io;

/* ------------------------------------------------------------------------------------
 * Checkpointed model derivatives (handles with ckpt_stride = c > 0): the observation map
 * x_0 -> y(x_0) = {H_t M_{0->t} x_0}, its tangent and its adjoint over the window, with the
 * trajectory kept only at every c-th step. The adjoint recomputes each segment's RK4 stage
 * states from its checkpoint, last segment first, and runs the exact discrete adjoint
 * through it; an observation at a segment boundary belongs to the earlier segment.
 *   ckpt   [n x (nseg+1)] device, nseg = ceil(nsteps / c): column s = x at step s c,
 *          the last column = x at step nsteps (written by riot_ckpt_forward)
 *   obs    [nobs] observed values H_t x_t (forward)
 *   dX0, gX0 [n x m] and dObs, gObs [nobs x m] device, column-major
 * m <= m_max. Calls are stream-ordered.
 * ---------------------------------------------------------------------------------- */
riot_status riot_ckpt_forward(riot_handle *h, const double *x0, double *ckpt, double *obs);
/* dObs = G dX0 (G = stacked H_t M_{0->t} tangent-linear maps at the checkpointed trajectory) */
riot_status riot_ckpt_tangent(riot_handle *h, int32_t m, const double *ckpt, const double *dX0,
                              double *dObs);
/* gX0 = G^T gObs (vector-Jacobian product of the observation map) */
riot_status riot_ckpt_adjoint(riot_handle *h, int32_t m, const double *ckpt, const double *gObs,
                              double *gX0);

/* ------------------------------------------------------------------------------------
 * Sketch handle: the steps of Alg. 3 after the Hessian-probe products, for an operator
 * whose products the caller computes (e.g. riot_tracer_hess_apply, or a learned probe
 * basis). Device pointers, column-major, leading dimension n.
 * ---------------------------------------------------------------------------------- */
typedef struct riot_sketch riot_sketch;
size_t riot_sketch_workspace_bytes(int32_t n, int32_t m_max);  /* 0: invalid (m_max <= n, 1088) */
riot_status riot_sketch_init(int32_t n, int32_t m_max, void *workspace, size_t bytes,
                             void *hip_stream, riot_sketch **out);
void riot_sketch_free(riot_sketch *s);
/* From Y = A Omega [n x m]: Q = orth(Y) (adaptive CholeskyQR), K solves
 * K (Q^T Omega) = Q^T Y, K <- (K + K^T)/2 = Z diag(lambda) Z^T, V = Q Z (lambda descending). */
riot_status riot_sketch_eig(riot_sketch *s, int32_t m, const double *Omega, const double *Y,
                            double *lambda, double *V, riot_rsvd_info *info);
/* dz from the k leading Ritz pairs: LRA -sum (1+l)^{-1} v v^T g, LRU -(I - sum l/(1+l) v v^T) g,
 * adaptive = eq. 11 (no L applied: the caller maps dz to its own space). */
/* riot_proj_residual on the sketch handle's workspace (any operator A). */
riot_status riot_sketch_residual(riot_sketch *s, int32_t m, const double *Q, const double *AQ,
                                 double *rho_host);
riot_status riot_sketch_increment(riot_sketch *s, int32_t k, const double *lambda,
                                  const double *V, const double *grad, riot_update mode,
                                  double *dz, double *dofs_host, int32_t *mode_used);

/* riot_sketch_eig for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid hipMalloc): no handle and no workspace.
 * The scratch regions (basis Q, Gram and projected matrices, eigen-solver work, split-K
 * partial products, flags) live in one static device array of
 * riot_sketch_noalloc_max_bytes() = 32 MiB, which each device the library runs on holds
 * until the process ends. Same arguments and results as riot_sketch_eig:
 *   n >= 1 rows, 1 <= m <= min(n, 1088) columns; Omega, Y [n x m] device (ld n);
 *   lambda [m], V [n x m] device out; hip_stream a hipStream_t of the current device (NULL =
 *   default stream); info host out or NULL (synchronises).
 * Returns RIOT_E_SCRATCH when riot_sketch_workspace_bytes(n, m) exceeds the array (e.g.
 * n = 4096 fits up to m = 316). The call allocates nothing: no hipMalloc, hipFree or
 * allocating library routine. Every call on one device shares that device's array, which
 * keeps the last call's contents; calls that overlap on one device (two streams, two host
 * threads) race and must be serialised by the caller. */
size_t riot_sketch_noalloc_max_bytes(void);
riot_status riot_sketch_eig_noalloc(int32_t n, int32_t m, const double *Omega, const double *Y,
                                    double *lambda, double *V, void *hip_stream,
                                    riot_rsvd_info *info);

/* ------------------------------------------------------------------------------------
 * Tracer source inversion on a periodic 2-D grid (the character of the paper's
 * black-carbon inversions, Sec. 3.2: a transport model, emissions through a lognormal
 * transform of the controls, point observations along aircraft tracks, p << n).
 * Concentration c on an N x N periodic grid (index [y][x], x fastest, dx = 1), c_0 = 0:
 *   c_{t+1} = A c_t + dt E * exp(up(s_tau(t))),
 * A = explicit upwind advection by u(y) = u0 + u1 sin(2 pi y / N) along x and v along y
 * (both >= 0) plus 5-point diffusion K; Courant number dt (u0 + |u1| + v) + 4 K dt <= 1.
 * Controls s: ntb time blocks (nsteps / ntb steps each) x (N/block)^2 spatial blocks,
 * [tau][by][bx]; up() repeats a block value over its block x block cells (block 1, 2, 4).
 * Observations: c_{t_o}[y_o][x_o], t_o in 1..nsteps. B = sigma^2 (C1 kron C1) per time
 * block, L = sigma (L1 kron L1) with L1 the caller's symmetric square root of the 1-D
 * correlation (N/block x N/block). The inner loop's operator is A_s = L G^T R^{-1} G L with
 * G the Jacobian of the observations at the base controls (Alg. 3 with this model).
 * ---------------------------------------------------------------------------------- */
typedef struct riot_tracer riot_tracer;
typedef struct {
    int32_t N;                 /* grid side, a multiple of 64 */
    int32_t nsteps;            /* window steps, a multiple of ntb */
    double dt, u0, u1, v, K;   /* step, wind, diffusion */
    int32_t block, ntb;        /* control block side in cells; time blocks */
    const double *E;           /* [N*N] host: prior emission field */
    int32_t nobs;
    const int32_t *obs_t, *obs_y, *obs_x;  /* [nobs] host: step (1..nsteps) and cell */
    const double *y, *rinv;    /* [nobs] host: observed values, diagonal of R^{-1} */
    const double *L1;          /* [(N/block)^2] host, symmetric */
    double sigma;
    int32_t m_max;             /* largest member block of tangent / adjoint / Hessian calls */
} riot_tracer_desc;

/* Host helper: the symmetric square root L1 [n x n] of the periodic 1-D exponential
 * correlation C1[i,j] = exp(-min(|i-j|, n-|i-j|) / ell), from the circulant's cosine
 * spectrum (eigenvalues clipped at 0). */
riot_status riot_exp_corr_sqrt(int32_t n, double ell, double *L1);

size_t riot_tracer_workspace_bytes(const riot_tracer_desc *desc);
riot_status riot_tracer_init(const riot_tracer_desc *desc, void *workspace, size_t bytes,
                             void *hip_stream, riot_tracer **out);
void riot_tracer_free(riot_tracer *h);
/* obs [nobs] = H(M(s)) for controls s [ncontrol] (device); s becomes the base of the
 * derivatives below. */
riot_status riot_tracer_forward(riot_tracer *h, const double *s, double *obs);
/* dObs [nobs x m] = G dS [ncontrol x m]; gS [ncontrol x m] = G^T gObs [nobs x m] */
riot_status riot_tracer_tangent(riot_tracer *h, int32_t m, const double *dS, double *dObs);
riot_status riot_tracer_adjoint(riot_tracer *h, int32_t m, const double *gObs, double *gS);
/* S = L Z [ncontrol x m] (S must not alias Z) */
riot_status riot_tracer_apply_L(riot_tracer *h, int32_t m, const double *Z, double *S);
/* Y = L G^T R^{-1} G L W [ncontrol x m] at the base (Y must not alias W) */
riot_status riot_tracer_hess_apply(riot_tracer *h, int32_t m, const double *W, double *Y);
/* grad = v - L G^T R^{-1} d, d = y - H(M(s_b)) (eq. 3), v nullable (zero); d_out [nobs]
 * device or NULL; J_host = 1/2 v^T v + 1/2 d^T R^{-1} d or NULL (synchronises). */
riot_status riot_tracer_gradient(riot_tracer *h, const double *v, double *grad, double *d_out,
                                 double *J_host);

/* Half-kernel taps l_0 .. l_w of the Gaussian square root used for B (host function):
 * l_d = c exp(-d^2 / ell^2), w = ceil(6.25 ell), c such that sum_{|d|<=w} l_d^2 = sigma_b^2,
 * so that B = L L^T has the correlation exp(-d^2 / (2 ell^2)) (the paper asks for Gaussian
 * correlations, Sec. 3.1, without fixing a square root). Returns w (with taps = NULL: the
 * half-width only), or -1 for invalid arguments or max_taps < w + 1. */
int32_t riot_gaussian_taps(double ell, double sigma_b, int32_t max_taps, double *taps);

/* Workspace bytes for a batch (0 if a descriptor is unusable in a batch). Every
 * descriptor's elems_per_lane is ignored (8 is used); all must share `prec`. */
size_t riot_batch_workspace_bytes(int32_t nprob, const riot_desc *descs);

/* Create a batch in a caller-allocated device workspace (256-byte aligned). Synchronises
 * `hip_stream` (uploads of the per-problem tables). Graph capture needs a stream other than
 * the legacy default stream. */
riot_status riot_batch_init(int32_t nprob, const riot_desc *descs, void *workspace,
                            size_t bytes, void *hip_stream, riot_batch **out);
void riot_batch_free(riot_batch *b);

/* Device pointers of the packed buffers (valid until riot_batch_free). */
riot_status riot_batch_buffers(riot_batch *b, riot_batch_io *io);

/* One inner loop for every problem (stream-ordered, no synchronisation): reads io.x,
 * writes grad, d, lambda, V, dz, dx. RIOT_E_STATE once a graph has been captured. */
riot_status riot_batch_run(riot_batch *b, uint64_t seed);

/* Layout of the persistent TL/AD launch: `workgroups` resident workgroups of 256 threads;
 * problems whose n / 8 <= wave_max_threads (<= 64) run one member per wave, the others one
 * member per workgroup (0: none per wave). */
riot_status riot_batch_set_layout(riot_batch *b, int32_t workgroups, int32_t wave_max_threads);

/* Autotuner: times the probe-product launch of this batch for workgroups in {1, 2, 3} x
 * compute units and member-per-wave on or off, keeps the fastest and reports it (host
 * pointers may be NULL). Synchronises; overwrites the batch's probe buffers. */
riot_status riot_batch_autotune(riot_batch *b, int32_t *workgroups_out,
                                int32_t *wave_max_threads_out, float *ms_out);

/* Capture riot_batch_run(b, seed) into a HIP graph; riot_batch_replay launches it. */
riot_status riot_batch_capture(riot_batch *b, uint64_t seed);
riot_status riot_batch_replay(riot_batch *b);

/* One timed probe-product launch of the batch (current probes) with per-tile device
 * clocks: ms = its duration (HIP events), busy_frac = the slots' busy time over the
 * slots available for the whole launch (load balance), tiles = number of tiles. Host
 * pointers may be NULL. Synchronises (not for use under graph capture); the clocks go to a
 * region of the batch's workspace. */
riot_status riot_batch_profile(riot_batch *b, float *ms, double *busy_frac, int32_t *tiles);

/* The handle of problem j inside the batch (owned by the batch: do not riot_free it). Its
 * single-problem calls work on the same workspace, e.g. for checks. */
riot_status riot_batch_problem(riot_batch *b, int32_t j, riot_handle **h);

/* ------------------------------------------------------------------------------------
 * Learned sketch proposal. Alg. 3 draws its probe block Omega at random; the sketch only
 * has to span the dominant eigenvectors of A (Section 2.2), so a network trained on the
 * eigenvectors of earlier cycles may propose most of the block. This network is a 1-D
 * periodic convolution stack on the state's grid (FP32 weights and activations):
 *   h_0[c] = (x[c] - mean(x[c])) / std(x[c])           (C0 input rows; none constant)
 *   z_l[c, i] = b_l[c] + sum_{c', j} W_l[c, c', j] h_{l-1}[c', (i + j - r) mod n]
 *   h_l = max(z_l, 0) for l < L                         (width 2 r + 1)
 *   N[i, c S + q] = z_L[c, i] if i lies in segment q, else 0   (localized output head)
 * An equivariant network alone gives fields over the whole grid; the head lets span(N)
 * hold structures at different places independently (S segments of n / S points).
 * Parameters: one flat FP32 array, per layer W_l [cout][cin][width] then b_l [cout]; layer
 * 1 has cin = C0, the last cout = k / S, the others cout = channels.
 * Training loss (eigenvalue-weighted subspace capture; a reading, the paper has no net):
 *   loss = -sum_i w_i v_i^T P v_i / sum_i w_i,  P = N (N^T N)^{-1} N^T,
 *   d loss / d N = -(2 / sum w) (I - P) V diag(w) V^T N (N^T N)^{-1},
 * evaluated in FP64 (Gram matrix, Cholesky, triangular solves on the FP64 MFMA GEMMs).
 * All data pointers are DEVICE pointers; a batch of inputs is [batch][C0][n], network outputs
 * [batch][k][n] (each sample an n x k column-major block), V [batch][k][n], w [batch][k].
 * The network keeps the activations of its last forward call for the backward call.
 * ---------------------------------------------------------------------------------- */
typedef struct riot_net riot_net;

typedef struct {
    int32_t n;          /* grid points, multiple of 64 */
    int32_t layers;     /* convolution layers L, 1..16 */
    int32_t channels;   /* hidden channels, 1..64 */
    int32_t k;          /* proposed basis vectors (output channels), 1..64, <= n */
    int32_t width;      /* kernel width 2 r + 1, odd, <= 11 */
    int32_t batch_max;  /* largest batch of states per call, >= 1 */
    int32_t segments;   /* S >= 1 (divides n and k): the last layer has k / S channels and
                           column c S + q of N is channel c on the q-th block of n / S
                           consecutive grid points, zero elsewhere (S = 1: N = z_L^T) */
    int32_t in_channels;/* C0, 1..64: fields per input sample (e.g. states along the window) */
} riot_net_desc;

size_t riot_net_workspace_bytes(const riot_net_desc *desc);  /* 0: invalid descriptor */
riot_status riot_net_init(const riot_net_desc *desc, void *workspace, size_t bytes,
                          void *hip_stream, riot_net **out);
void riot_net_free(riot_net *h);
int64_t riot_net_param_count(const riot_net *h);
/* Copy parameters and/or gradients in ([count] device each; either may be NULL), e.g. to
 * start from given weights or to apply Adam to gradients reduced elsewhere. */
riot_status riot_net_set_params(riot_net *h, const float *params, const float *grads);
/* Copy the parameters and/or the last gradients out (either pointer may be NULL). */
riot_status riot_net_get_params(riot_net *h, float *params, float *grads);
/* N = net(x) for a batch of inputs x [batch][C0][n] (FP64). N [batch][k][n] FP32 out or NULL;
 * N64 FP64 out or NULL: sample s, column c at N64 + (s * k + c) * ld64 (ld64 >= n), so a
 * single state's proposal can fill the first k columns of an n x m probe block. */
riot_status riot_net_forward(riot_net *h, int32_t batch, const double *x, float *N,
                             double *N64, int32_t ld64);
/* Parameter gradients (summed over the batch) of sum(gN * N) at the last forward call's
 * batch; gN [batch][k][n]. Overwrites the gradient buffer. */
riot_status riot_net_backward(riot_net *h, int32_t batch, const float *gN);
/* One Adam step (bias-corrected; step counts from 1, step 1 clears the moments). */
riot_status riot_net_adam(riot_net *h, float lr, float beta1, float beta2, float eps,
                          int32_t step);
/* Capture loss of each sample and its gradient gN [batch][k][n] (FP32 out) for network
 * outputs N, targets V (orthonormal columns) and weights w >= 0 (sum > 0). loss_host:
 * [batch] host out or NULL (synchronises). N must have full column rank (else NaN). */
riot_status riot_net_capture_loss(riot_net *h, int32_t batch, const float *N, const double *V,
                                  const double *w, double *loss_host, float *gN);
/* forward + capture loss + backward + Adam (beta1 0.9, beta2 0.999, eps 1e-8) on one batch. */
riot_status riot_net_train_step(riot_net *h, int32_t batch, const double *x, const double *V,
                                const double *w, float lr, int32_t step, double *loss_host);

#ifdef __cplusplus
}
#endif

#endif /* RIOT_H */
