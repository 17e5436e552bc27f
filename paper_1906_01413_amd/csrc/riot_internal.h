// Internal declarations shared by the HIP translation units of libriot.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "riot.h"

namespace riot {

// ---------------------------------------------------------------------------
// Lorenz-96 member layout.
//
// One probe ("member") of the batched TL/AD integration is owned by one
// workgroup of NT threads. Active thread l (l < A = n / E) owns the E
// contiguous state elements a = l*E .. a+E-1 and keeps them in registers.
// The base trajectory is stored per (step, RK4 stage) as a block of (E + 4)
// rows of NT values: row j < E holds x[l*E + j] in column l, rows E..E+3 hold
// the four halo values x[a-2], x[a-1], x[a+E], x[a+E+1] of thread l. Every row
// is read by a wave as one contiguous, coalesced segment.
// ---------------------------------------------------------------------------

struct ModelView {
  int n, T, E, NT, A;   // state size, window steps, elems/lane, threads, active threads
  double h, F;          // RK4 step and forcing
  int S, U;             // observed steps, unique observed (step, variable) pairs
  const void *xs;       // base stage blocks, (T+1)*4 blocks of (E+4)*NT Real
  const int *stepk;     // [T+1] observed-step ordinal or -1
  const int *ustart;    // [S*NT] first unique-obs index of thread l at observed step k
  const int *umask;     // [S*NT] bit j set when element l*E+j is observed at step k
  const void *wgt;      // [U] sum of R^{-1} over the observations of each unique pair (Real)
};

inline size_t stage_block_elems(int E, int NT) { return (size_t)(E + 4) * NT; }

// Launch helpers implemented in l96.hip -------------------------------------

// Nonlinear RK4 trajectory. When store != 0 the stage blocks of every step are
// written (FP64 and, when xs32 != nullptr, FP32 copies), plus block (T, 0) = x_T.
hipError_t launch_trajectory(const ModelView &mv, int nsteps, const double *x0, double *xout,
                             double *xs64, float *xs32, hipStream_t st);

// Innovation d = y - H(x) per observation and gradient forcing
// fgrad[u] = sum_{o in u} rinv_o d_o, from the stored trajectory.
hipError_t launch_innovation(const ModelView &mv, const double *xs64, int nobs, const int *obs_step,
                             const int *obs_idx, const double *y, const double *rinv,
                             const int *u_optr, const int *u_olist, double *d, void *fgrad,
                             bool fp32, hipStream_t st);

// 1/2 v^T v + 1/2 sum rinv d^2 -> out[0] (single workgroup, fixed reduction order).
hipError_t launch_cost(int n, const double *v, int nobs, const double *d, const double *rinv,
                       double *out, hipStream_t st);

// Member TL/AD integrations. mode: 0 = TL then AD with R^{-1}-weighted forcing from the TL
// pass (probe product), 1 = AD only with shared forcing `fsrc` (gradient), 2 = TL only
// (raw observed values into f), 3 = AD only with each member's own forcing f.
// dx0 [n x m] natural layout (already multiplied by L); lam0 [n x m] out.
// f: per-member forcing scratch [m x U] (Real). fp32 selects the Real type.
hipError_t launch_tlad(const ModelView &mv, int m, int mode, const double *dx0, double *lam0,
                       void *f, const void *fsrc, bool fp32, hipStream_t st);

// Observation-space values <-> per-member unique-pair buffers (caller order o).
hipError_t launch_obs_gather(int nobs, int U, int m, const int *u_of_o, const void *f, double *Z,
                             bool fp32, hipStream_t st);
hipError_t launch_obs_scatter(int nobs, int U, int m, const int *u_optr, const int *u_olist,
                              const double *Fo, void *f, bool fp32, hipStream_t st);

// Y = L X (mode 0), Y = L X + Z (mode 1), Y = Z - L X (mode 2); m columns.
hipError_t launch_apply_L(int n, int w, const double *taps, int m, const double *X, double *Y,
                          const double *Z, int mode, hipStream_t st);

// Conjugate gradients on (I + A) x = -g, one persistent workgroup.
hipError_t launch_cg(const ModelView &mv, int w, const double *taps, const double *g, int iters,
                     double rtol, double *x, double *iterates, double *vec_scratch, void *f,
                     int *used, bool fp32, hipStream_t st);

// Philox4x32-10 + Box-Muller standard normals.
hipError_t launch_philox_normal(long long total, uint64_t seed, uint64_t stream, double *out,
                                hipStream_t st);

// Linear algebra (linalg.hip) --------------------------------------------------

// C[M x N] = alpha * op(A) * op(B) + beta * C, column-major, FP64 MFMA.
// ta/tb: 0 = no transpose, 1 = transpose. For ta = 1 and tb = 0 (A^T B, the
// Gram/projection shape) the contraction is split over `splitk` partial
// buffers reduced in fixed order (partial must hold splitk * M * N doubles).
// run: optional device flag; when it holds 0 the launched kernels return at once
// (predicated launches that keep a data-dependent loop free of host synchronisation).
hipError_t gemm_f64(int ta, int tb, int M, int N, int K, double alpha, const double *A, int lda,
                    const double *B, int ldb, double beta, double *C, int ldc, double *partial,
                    int splitk, hipStream_t st, const int *run = nullptr);

// Upper Cholesky factor R of G + s I (R^T R). mode 0: s = 0; mode 1: s = shift_rel * ||G||_F;
// mode 2: s = 0 first, restarted with the shift on breakdown. flag[0] = 1 when the last
// attempt breaks down (non-positive or non-finite pivot); shifts[0] counts shifted attempts.
hipError_t launch_cholesky(int m, const double *G, double *R, double shift_rel, int mode,
                           int *flag, int *shifts, hipStream_t st);

// Blocked Cholesky G + s I = L L^T (lower), same modes as launch_cholesky.
hipError_t launch_chol_blocked(int m, const double *G, double *L, double shift_rel, int mode,
                               int *flag, int *shifts, hipStream_t st, const int *run = nullptr,
                               int *modflag = nullptr);
// CholeskyQR pass control (see cholqr in the API layer): reset, then one call per pass;
// count (optional) is incremented once per pass that ran.
hipError_t launch_cholqr_reset(int *cq, hipStream_t st);
hipError_t launch_cholqr_ctrl(int *cq, int pass_was_shifted, int *count, hipStream_t st);

// X <- X L^{-T} in place (X rows x m, leading dimension ldx; L lower m x m).
hipError_t launch_trsm_rlt(int rows, int m, double *X, int ldx, const double *L, hipStream_t st,
                           const int *run = nullptr);

// Blocked inverse of a lower-triangular L.
hipError_t launch_trinv_lower(int m, const double *L, double *X, hipStream_t st);

// Inverse of upper-triangular R (m x m).
hipError_t launch_trinv_upper(int m, const double *R, double *Rinv, hipStream_t st);

// Inverse of a general m x m matrix by Gauss-Jordan elimination with partial pivoting.
// work holds 2*m*m doubles; flag[0] = 1 when a zero pivot is met.
hipError_t launch_gj_inverse(int m, const double *M, double *Minv, double *work, int *flag,
                             hipStream_t st);

// K <- (K + K^T)/2 and asym[0] = ||K - K^T||_F / ||K||_F (before symmetrisation).
// part: 128 doubles of scratch.
hipError_t launch_symmetrize(int m, double *K, double *asym, double *part, hipStream_t st);

// ||Q^T Q - I||_F from the Gram matrix G = Q^T Q -> out[0].
hipError_t launch_orth_err(int m, const double *G, double *out, hipStream_t st);

// Symmetric eigendecomposition K = Z diag(lam) Z^T, eigenvalues descending.
// work must hold syev_work_doubles(m) doubles; flag[0] = 1 on non-convergence.
size_t syev_work_doubles(int m);
hipError_t launch_syev(int m, const double *K, double *lam, double *Z, double *work, int *flag,
                       hipStream_t st);

// Symmetric eigendecomposition (eig.hip): tridiagonalisation, relatively robust
// representation, multisection bisection, twisted-factorisation vectors, cluster
// Rayleigh-Ritz, back-transformation. Eigenvalues descending. flag[0] = 1 on failure.
size_t eig_work_doubles(int m);
hipError_t launch_eig(int m, const double *K, double *lam, double *Z, double *work, int *flag,
                      hipStream_t st);

// Increment helpers: c = V^T g handled by gemm_f64; these combine.
// dz = -(V (c .* a)) [lra] or dz = -(g - V (c .* a)) [lru], a = coefficient per pair.
hipError_t launch_increment_combine(int n, int k, const double *lam, const double *V,
                                    const double *c, const double *g, int mode_lru, double *dz,
                                    double *dofs, hipStream_t st);

// Mode selection on the device: out[0] = lam[k-1] >= 1 ? RIOT_LRA : RIOT_LRU.
hipError_t launch_choose_mode(int k, const double *lam, int *out, hipStream_t st);

// Posterior covariance coefficients and diagonal.
hipError_t launch_postcov_diag(int n, int k, const double *lam, const double *W, int mode_lru,
                               double base_diag, double *coef, double *diag, hipStream_t st);

// Dense B = L L^T (circulant with first column brow) into P: P = beta * P + B, skipped
// when mode != nullptr and *mode != RIOT_LRU.
hipError_t launch_dense_B(int n, const double *brow, double beta, double *P, const int *mode,
                          hipStream_t st);

// Scale columns: Y[:, j] = X[:, j] * s[j].
hipError_t launch_scale_cols(int n, int k, const double *X, const double *s, double *Y,
                             hipStream_t st);

// p[0..count) = 0 with a kernel (graph-capture safe, unlike a memset node).
hipError_t launch_zero_ints(int *p, int count, hipStream_t st);

// Non-finite check over `count` doubles: flag[0] |= 1 when any value is NaN or Inf.
hipError_t launch_check_finite(long long count, const double *x, int *flag, hipStream_t st);

}  // namespace riot
