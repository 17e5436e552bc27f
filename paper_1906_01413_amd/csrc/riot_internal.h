// Internal declarations shared by the HIP translation units of libriot.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "riot.h"

namespace riot {

// Every device buffer of the library is global memory, but a pointer that a kernel reads
// from a job table (or that is merged with one) is generic to the compiler, which then
// emits flat loads and stores. A flat access also counts against the LDS/scalar counter,
// so each LDS wait (every barrier of a halo exchange or reduction) would wait for the
// kernel's outstanding global stores and loads as well. Accessing such memory through
// gptr(p)[i] makes the compiler use global instructions.
template <typename T>
using gmem = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ gmem<T> *gptr(T *p) {
  return (gmem<T> *)p;
}

// ---------------------------------------------------------------------------
// Batched launches: one job per problem, the problem taken from a grid dimension,
// so that one launch serves a whole batch of independent, differently sized problems.
// ---------------------------------------------------------------------------
struct GemmJob {
  int M, N, K;
  const double *A;
  int lda;
  const double *B;
  int ldb;
  double *C;
  int ldc;
  const int *run;  // optional predicate (0: skip this problem)
};
struct CholJob {
  int m;
  const double *G;
  double *L;
  double shift_rel;
  int *flag, *shifts;
  const int *run;
  int *modflag;
};
struct TrsmJob {
  int rows, m;
  double *X;
  int ldx;
  const double *L;
  const int *run;
};
struct CqJob {
  int *cq;
  int *count;
};
// CholeskyQR pass control carried by the Cholesky of each pass: cq[p] is the run flag of
// pass 0 < p < npass (the launches of pass p return at once when it is 0; pass 0 always
// runs), cq[npass] counts consecutive clean passes (unshifted, no pivot replaced; pass 0
// starts the count). The Cholesky of pass p sets cq[p + 1]: 1 until two clean passes in a
// row (or a breakdown), and 0 when pass p itself did not run; count[0] (if given) counts
// the passes run.
struct CholQrCtl {
  int *cq = nullptr;
  int pass = 0, npass = 0;
  int *count = nullptr;
  // optional host-mapped word: the pass's Cholesky stores (seq << 1) | (next pass runs) there
  // with a system-scope release, for a host that launches passes only while they are needed
  int *host = nullptr;
  int seq = 0;
};
struct SymJob {
  int m;
  double *K;
};
struct EigJob {
  int m;
  const double *K;
  double *lam, *Z, *work;
  int *flag;
};
struct IncJob {
  int n, k;
  const double *lam, *V, *c, *g;
  double *dz, *dofs;
};
struct CopyJob {
  long long count;
  const double *src;
  double *dst;
};
struct PhiloxJob {
  long long total;
  unsigned long long stream;
  double *out;
};


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

// Batched model jobs (E = 8 for every problem of a batch).
struct TrajJob {
  ModelView mv;
  const double *x0;
  double *xs64;
  float *xs32;
};
struct InnovJob {
  ModelView mv;
  const double *xs64;
  const int *obs_step, *obs_idx, *u_optr, *u_olist;
  const double *y, *rinv;
  double *d;
  void *fgrad;
};
// One problem of a persistent TL/AD launch: members j = 0 .. m-1 read dx0 + j n, write
// lam0 + j n and use f + j U (mode 0/2/3); mode 1 reads the shared forcing fsrc.
struct TladProb {
  ModelView mv;
  const double *dx0;
  double *lam0;
  void *f;
  const void *fsrc;
};
// One tile of a persistent TL/AD launch: member `mem` of problem `prob`.
struct TladTile {
  int prob, mem;
};
struct ApplyLJobE {
  int n, w, m;
  const double *taps, *X;
  double *Y;
  const double *Z;
  int mode;
};

// Launch helpers implemented in l96.hip -------------------------------------

// Batched model launches. Persistent TL/AD: `nwg` workgroups of 256 threads first take
// whole-workgroup tiles (one member per workgroup) from wg_tiles through counters[0],
// then each wave takes wave tiles (one member per wave, problems with NT <= 64) from
// wave_tiles through counters[1]. Tiles are processed in list order (longest first).
hipError_t launch_trajectory_batched(int nprob, const TrajJob *jobs, hipStream_t st);
hipError_t launch_innovation_batched(int nprob, int maxU, const InnovJob *jobs, bool fp32,
                                     hipStream_t st);
// clk (optional): per tile, start and end of its integration on the device's constant-rate
// clock (wall_clock64), wg tiles first, then wave tiles.
hipError_t launch_tlad_persistent(int nwg, int mode, const TladProb *probs, const TladTile *wg_tiles,
                                  int n_wg, const TladTile *wave_tiles, int n_wave, int *counters,
                                  bool fp32, hipStream_t st, long long *clk = nullptr);
// Workgroups of the persistent TL/AD kernel that fit one compute unit at once.
int tlad_persistent_resident_per_cu(bool fp32);
hipError_t launch_apply_L_batched(int nprob, int maxm, int maxext, const ApplyLJobE *jobs,
                                  hipStream_t st);
hipError_t launch_philox_batched(int nprob, long long maxtotal, uint64_t seed,
                                 const PhiloxJob *jobs, hipStream_t st);

// Nonlinear RK4 trajectory. When store != 0 the stage blocks of every step are
// written (FP64 and, when xs32 != nullptr, FP32 copies), plus block (T, 0) = x_T.
// Dual (observation-space) right-hand side and increment scaling by R^{-1/2}.
hipError_t launch_psas_rhs(int nobs, const double *rinv, const double *d, const double *bp,
                           double *out, hipStream_t st);
hipError_t launch_psas_scale(int nobs, const double *rinv, const double *t, double *dw,
                             hipStream_t st);
// Perturbed observations y - R^{1/2} eps of a gradient sample.
hipError_t launch_obs_perturb(int nobs, const double *y, const double *rinv, const double *eps,
                              double *out, hipStream_t st);
// Deterministic LRA/LRU choice (nonlinear window from several states, costs, selection).
hipError_t launch_window_obs(const ModelView &mv, int nstates, const double *x0, double *xu,
                             hipStream_t st);
hipError_t launch_cand_state(int n, int nc, const double *x, const double *v, const double *dz,
                             const double *dx, double *xc, double *vc, hipStream_t st);
hipError_t launch_cand_cost(int n, int nc, const double *vc, int nobs, int U, const double *y,
                            const double *rinv, const int *u_of_o, const double *xu, double *J,
                            hipStream_t st);
hipError_t launch_cand_select(int n, int nc, const double *J, const double *dzc, const double *dxc,
                              double *dz, double *dx, int *mode_out, hipStream_t st);
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

// Flags or-ed into the TL/AD mode (see Member::run): skip step 0 of the window, start the
// AD from dx0, return the final tangent state of a TL-only sweep.
constexpr int kTladSkip0 = 8, kTladInitLam = 16, kTladOutState = 32;

// Member TL/AD integrations. mode: 0 = TL then AD with R^{-1}-weighted forcing from the TL
// pass (probe product), 1 = AD only with shared forcing `fsrc` (gradient), 2 = TL only
// (raw observed values into f), 3 = AD only with each member's own forcing f.
// dx0 [n x m] natural layout (already multiplied by L); lam0 [n x m] out.
// f: per-member forcing scratch [m x U] (Real). fp32 selects the Real type.
hipError_t launch_tlad(const ModelView &mv, int m, int mode, const double *dx0, double *lam0,
                       void *f, const void *fsrc, bool fp32, hipStream_t st);

// Observed values x_t[i] of a stored segment whose step 0 is window step lo (see kernel).
hipError_t launch_obs_value(const ModelView &mv, const double *xs64, int nobs, const int *obs_step,
                            const int *obs_idx, int lo, bool include_lo, double *out,
                            hipStream_t st);

// Observation-space values <-> per-member unique-pair buffers (caller order o).
hipError_t launch_obs_gather(int nobs, int U, int m, const int *u_of_o, const void *f, double *Z,
                             bool fp32, hipStream_t st, const double *rinv = nullptr);
hipError_t launch_obs_scatter(int nobs, int U, int m, const int *u_optr, const int *u_olist,
                              const double *Fo, void *f, bool fp32, hipStream_t st,
                              const double *rinv = nullptr);

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
// lower: for the symmetric A^T A shape (ta = 1, tb = 0, M = N), only C's lower triangle is
// formed; the strict upper triangle is left as it was.
// gram_sq (lower only, beta = 0): the strict upper triangle is set to zero and gram_sq[b],
// b < nb = gram_sq_blocks(M), receives a partial sum of ||C||_F^2; the 32 doubles after them
// are cleared (flags of the in-place Cholesky); gram_sq[nb + 32 + b] receives a partial sum
// of ||C - I||_F^2 (each sum in a fixed order). The input form of an in-place Cholesky
// (launch_chol_blocked with the same gram_sq).
// sym (M = N, beta = 0, partial given): C is written as (C + C^T) / 2 by the reduction.
// B2 and C2 (tb = 0, not lower, no gram_sq): the pair form [C C2] = alpha op(A) [B B2]
// + beta [C C2] in one launch (B2 with ldb and C2 with ldc, N columns each); the partial
// buffer then holds splitk * M * 2N doubles.
hipError_t gemm_f64(int ta, int tb, int M, int N, int K, double alpha, const double *A, int lda,
                    const double *B, int ldb, double beta, double *C, int ldc, double *partial,
                    int splitk, hipStream_t st, const int *run = nullptr, bool lower = false,
                    double *gram_sq = nullptr, const double *B2 = nullptr,
                    double *C2 = nullptr, bool sym = false);
inline int gram_sq_blocks(int m) { return (int)(((size_t)m * m + 255) / 256); }

// Blocked Cholesky G + s I = L L^T (lower, column-major). mode 0: s = 0; mode 1:
// s = shift_rel * ||G||_F; mode 2: s = 0 with every pivot not above shift_rel * ||G||_F
// replaced by that value (modflag[0] = 1 when one was). flag[0] = 1 on breakdown
// (non-positive or non-finite pivot); shifts[0] counts shifted or modified factorizations.
// dinv (with gram_sq, or null): receives the inverses of the factor's 32 x 32 diagonal
// blocks in the layout of launch_trsm_diag_inv. ctl.cq (with gram_sq, or null): the pass
// control of a CholeskyQR; the run flag is then ctl.cq[ctl.pass] and `run` is ignored.
// gram_sq: the partial sums of ||G||_F^2 and ||G - I||_F^2 written by the Gram GEMM
// (gemm_f64 with gram_sq); the factorization then runs in place, G == L holding the Gram
// matrix with a zero upper triangle, by one workgroup up to m = 288, beyond it by one
// workgroup per 32-column block (m <= 1536); in mode 2 a Gram with ||G - I||_F^2 <= u is
// factored to first order, L = I + (strict lower part of G - I) + (diagonal of G - I) / 2,
// whose L L^T is within ||G - I||_F^2 of G. Without gram_sq G is copied into L first and
// one workgroup factors.
hipError_t launch_chol_blocked(int m, const double *G, double *L, double shift_rel, int mode,
                               int *flag, int *shifts, hipStream_t st, const int *run = nullptr,
                               int *modflag = nullptr, const double *gram_sq = nullptr,
                               double *dinv = nullptr, CholQrCtl ctl = CholQrCtl());
// C_b = alpha op(A_b) op(B_b) + beta C_b for b < batch, with A_b = A + b sA (likewise B, C).
hipError_t gemm_f64_strided(int ta, int tb, int M, int N, int K, double alpha, const double *A,
                            int lda, long long sA, const double *B, int ldb, long long sB,
                            double beta, double *C, int ldc, long long sC, int batch,
                            hipStream_t st);

// Batched forms of the launches above (jobs: device array of nprob entries; max*: largest
// size over the batch, which sets the grid).
hipError_t launch_gemm_batched(int ta, int tb, int nprob, int maxM, int maxN, double alpha,
                               double beta, const GemmJob *jobs, hipStream_t st);
hipError_t launch_chol_batched(int nprob, int mode, const CholJob *jobs, hipStream_t st);
hipError_t launch_trsm_batched(int nprob, int maxrows, const TrsmJob *jobs, hipStream_t st);
hipError_t launch_cholqr_reset_batched(int nprob, const CqJob *jobs, hipStream_t st);
hipError_t launch_cholqr_ctrl_batched(int nprob, int pass_was_shifted, const CqJob *jobs,
                                      hipStream_t st);
hipError_t launch_symmetrize_batched(int nprob, const SymJob *jobs, hipStream_t st);
hipError_t launch_eig_batched(int nprob, int maxm, const EigJob *jobs, hipStream_t st);
hipError_t launch_increment_batched(int nprob, int maxn, int mode_lru, const IncJob *jobs,
                                    hipStream_t st);
hipError_t launch_copy_batched(int nprob, long long maxcount, const CopyJob *jobs, hipStream_t st);

// CholeskyQR pass control (see cholqr in the API layer): reset, then one call per pass;
// count (optional) is incremented once per pass that ran.
hipError_t launch_cholqr_reset(int *cq, hipStream_t st);
hipError_t launch_cholqr_ctrl(int *cq, int pass_was_shifted, int *count, hipStream_t st);

// X <- X L^{-T} in place (X rows x m, leading dimension ldx; L lower m x m), through the
// inverses of L's 32 x 32 diagonal blocks: launch_trsm_diag_inv (or the in-place Cholesky)
// writes them to dinv (ceil(m / 32) * 1024 doubles), launch_trsm_rlt_inv uses them. X2
// (rows2 x m, leading dimension ldx2, or null) is solved with the same L in the same launch.
hipError_t launch_trsm_diag_inv(int m, const double *L, double *dinv, hipStream_t st,
                                const int *run = nullptr);
// Xsrc (optional, not with run for m > 288): the first matrix's input, read from Xsrc
// (leading dimension ldx) and the solution written to X.
hipError_t launch_trsm_rlt_inv(int rows, int m, double *X, int ldx, const double *L,
                               const double *dinv, hipStream_t st, const int *run = nullptr,
                               int rows2 = 0, double *X2 = nullptr, int ldx2 = 1,
                               const double *Xsrc = nullptr);

// K <- (K + K^T)/2 and, if asym is given, asym[0] = ||K - K^T||_F / ||K||_F (before
// symmetrisation).
// part: 128 doubles of scratch.
hipError_t launch_symmetrize(int m, double *K, double *asym, double *part, hipStream_t st);

// out[0] = ||R||_F / ||A||_F over count contiguous doubles.
hipError_t launch_fro_ratio(long long count, const double *R, const double *A, double *out,
                            hipStream_t st);
// ||Q^T Q - I||_F from the Gram matrix G = Q^T Q -> out[0].
hipError_t launch_orth_err(int m, const double *G, double *out, hipStream_t st);

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
// Spectral preconditioner middle factor and Y = a Y + b X.
hipError_t launch_precond_scale(int mj, int m, const double *lam, double power, double *C,
                                hipStream_t st);
hipError_t launch_axpby(long long count, double a, double *Y, double b, const double *X,
                        hipStream_t st);
hipError_t launch_block_band_zero(int m, int l, double *T, hipStream_t st);

// Non-finite check over `count` doubles: flag[0] |= 1 when any value is NaN or Inf.
// flag[0] = 1 if x[0 .. count) or x2[0 .. count2) holds a NaN or an infinity.
hipError_t launch_check_finite(long long count, const double *x, int *flag, hipStream_t st,
                               long long count2 = 0, const double *x2 = nullptr);

}  // namespace riot
