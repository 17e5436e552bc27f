// Dense FP64 linear algebra of the RSVD stages (Alg. 3: orthonormal basis of Y,
// solve for K, eigendecomposition of K, Ritz vectors) for gfx950.
//
//  - gemm_f64: tall-skinny products (Y^T Y, Q^T Y, Q^T Omega, Y R^{-1}, Q Z, W C W^T)
//    on the FP64 matrix cores (v_mfma_f64_16x16x4_f64), split-K with a
//    fixed-order reduction for the A^T B shape.
//  - small m x m factorizations: one workgroup each (Cholesky with optional
//    diagonal shift, triangular inverse, Gauss-Jordan inverse with partial
//    pivoting, Householder tridiagonalisation + implicit QL eigen-solver).

#include "riot_internal.h"

namespace riot {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// GEMM on the FP64 matrix cores. One wave computes a 32 x 32 tile of C as a
// 2 x 2 grid of 16 x 16 MFMA tiles. Operand lane layout of
// v_mfma_f64_16x16x4_f64: lane l supplies A[i = l % 16][k = l / 16] and
// B[k = l / 16][j = l % 16]; result register r of lane l is
// C[l / 16 + 4 * r][l % 16] (checked on gfx950 with an exact-integer probe).
// ---------------------------------------------------------------------------

template <int TA, int TB>
__global__ void __launch_bounds__(64)
    gemm_mfma_kernel(int M, int N, int K, const double *__restrict__ A, int lda,
                     const double *__restrict__ B, int ldb, double *__restrict__ C, int ldc,
                     double alpha, double beta, int kchunk, double *__restrict__ partial,
                     const int *__restrict__ run) {
  if (run && run[0] == 0) return;  // predicated launch: the whole grid skips uniformly
  const int lane = threadIdx.x;
  const int li = lane & 15, lg = lane >> 4;
  const int m0 = blockIdx.x * 32, n0 = blockIdx.y * 32;
  const int kz = blockIdx.z;
  const int kbeg = kz * kchunk;
  const int kend = min(K, kbeg + kchunk);
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

  for (int k0 = kbeg; k0 < kend; k0 += 4) {
    const int kk = k0 + lg;
    const bool kin = kk < kend;
    double av[2], bv[2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const int row = m0 + 16 * rt + li;
      double v = 0.0;
      if (kin && row < M) v = TA ? A[(size_t)row * lda + kk] : A[(size_t)kk * lda + row];
      av[rt] = v;
    }
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int col = n0 + 16 * ct + li;
      double v = 0.0;
      if (kin && col < N) v = TB ? B[(size_t)kk * ldb + col] : B[(size_t)col * ldb + kk];
      bv[ct] = v;
    }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
        acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[rt], bv[ct], acc[rt][ct], 0, 0, 0);
  }

#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + 16 * rt + lg + 4 * r;
        const int col = n0 + 16 * ct + li;
        if (row < M && col < N) {
          const double v = acc[rt][ct][r];
          if (partial) {
            partial[(size_t)kz * M * N + (size_t)col * M + row] = v;
          } else {
            double out = alpha * v;
            if (beta != 0.0) out += beta * C[(size_t)col * ldc + row];
            C[(size_t)col * ldc + row] = out;
          }
        }
      }
}

__global__ void splitk_reduce_kernel(int M, int N, int splits, const double *__restrict__ partial,
                                     double alpha, double beta, double *__restrict__ C, int ldc,
                                     const int *__restrict__ run) {
  if (run && run[0] == 0) return;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t MN = (size_t)M * N;
  if (idx >= MN) return;
  double s = 0.0;
  for (int z = 0; z < splits; ++z) s += partial[(size_t)z * MN + idx];
  const int row = (int)(idx % M), col = (int)(idx / M);
  double out = alpha * s;
  if (beta != 0.0) out += beta * C[(size_t)col * ldc + row];
  C[(size_t)col * ldc + row] = out;
}

// ---------------------------------------------------------------------------
// Workgroup helpers
// ---------------------------------------------------------------------------

__device__ double wg_sum(double v, double *red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = (blockDim.x + 63) >> 6;
  for (int k = 0; k < nw; ++k) s += red[k];
  __syncthreads();
  return s;
}

// argmax of |v| with smallest index on ties; returns index (value via *best)
__device__ int wg_argmax_abs(double v, int idx, double *redv, int *redi, double *best) {
  double a = (idx >= 0) ? fabs(v) : -1.0;
  int bi = idx;
  for (int off = 32; off > 0; off >>= 1) {
    const double oa = __shfl_down(a, off, 64);
    const int oi = __shfl_down(bi, off, 64);
    if (oa > a || (oa == a && oi >= 0 && (bi < 0 || oi < bi))) {
      a = oa;
      bi = oi;
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    redv[wv] = a;
    redi[wv] = bi;
  }
  __syncthreads();
  double ba = -1.0;
  int bidx = -1;
  const int nw = (blockDim.x + 63) >> 6;
  for (int k = 0; k < nw; ++k) {
    if (redv[k] > ba || (redv[k] == ba && redi[k] >= 0 && (bidx < 0 || redi[k] < bidx))) {
      ba = redv[k];
      bidx = redi[k];
    }
  }
  __syncthreads();
  *best = ba;
  return bidx;
}

// ---------------------------------------------------------------------------
// 32 x 32 wave-level MFMA block product: acc += op(A)[0:32, 0:K] op(B)[0:K, 0:32],
// op(A)[i][k] = TA ? A[k + i*lda] : A[i + k*lda], op(B)[k][j] = TB ? B[j + k*ldb] : B[k + j*ldb].
// Rows >= mA and columns >= nB read as zero. The lane owning result register r
// of tile (rt, ct) holds element (16 rt + l/16 + 4 r, 16 ct + l%16).
// ---------------------------------------------------------------------------

template <bool TA, bool TB>
__device__ __forceinline__ void mma32_load(const double *__restrict__ A, int lda,
                                           const double *__restrict__ B, int ldb, int K, int mA,
                                           int nB, int k0, double (&av)[4][2], double (&bv)[4][2]) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lg = lane >> 4;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int kk = k0 + 4 * s + lg;
    const bool kin = kk < K;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const int row = 16 * rt + li;
      av[s][rt] = (kin && row < mA) ? (TA ? A[kk + (size_t)row * lda] : A[row + (size_t)kk * lda]) : 0.0;
    }
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int col = 16 * ct + li;
      bv[s][ct] = (kin && col < nB) ? (TB ? B[col + (size_t)kk * ldb] : B[kk + (size_t)col * ldb]) : 0.0;
    }
  }
}

// The contraction runs in chunks of 16 (four MFMA k-steps); the operands of the next
// chunk are loaded before the current chunk's MFMAs are issued.
template <bool TA, bool TB>
__device__ __forceinline__ void wave_mma32(const double *__restrict__ A, int lda,
                                           const double *__restrict__ B, int ldb, int K, int mA,
                                           int nB, d4 (&acc)[2][2]) {
  if (K <= 0) return;
  double av[4][2], bv[4][2], an[4][2], bn[4][2];
  mma32_load<TA, TB>(A, lda, B, ldb, K, mA, nB, 0, av, bv);
  for (int k0 = 0; k0 < K; k0 += 16) {
    const bool more = k0 + 16 < K;
    if (more) mma32_load<TA, TB>(A, lda, B, ldb, K, mA, nB, k0 + 16, an, bn);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
          acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s][rt], bv[s][ct], acc[rt][ct], 0, 0, 0);
    if (more) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          av[s][t] = an[s][t];
          bv[s][t] = bn[s][t];
        }
    }
  }
}

__device__ __forceinline__ void zero_acc(d4 (&acc)[2][2]) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
}

constexpr int kCholThreads = 512;
constexpr int kPB = 32;  // panel width of the blocked factorizations
constexpr int kStageRows = 320;  // panel rows staged in LDS by the Cholesky

// ---------------------------------------------------------------------------
// Blocked Cholesky G + s I = L L^T (lower, column-major), one workgroup.
// mode 0: s = 0; mode 1: s = shift_rel ||G||_F; mode 2: s = 0, restarted with the
// shift on breakdown. Per 32-column panel: the diagonal block is factored in LDS,
// the panel below by row-wise forward substitution, the trailing lower triangle
// updated with FP64 MFMA (one wave per 32 x 32 tile).
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kCholThreads)
    chol_blocked_kernel(int m, const double *__restrict__ G, double *__restrict__ L,
                        double shift_rel, int mode, int *__restrict__ flag,
                        int *__restrict__ shifts, const int *__restrict__ run,
                        int *__restrict__ modflag) {
  if (run && run[0] == 0) return;
  __shared__ double D[kPB][kPB + 1];
  __shared__ double Dinv[kPB];
  __shared__ double Pn[kPB * (kStageRows + 1)];
  __shared__ double red[16];
  __shared__ int bad;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int wave = tid >> 6, nwaves = nt >> 6;
  double fro = 0.0;
  if (mode != 0) {
    double part = 0.0;
    for (size_t idx = tid; idx < (size_t)m * m; idx += nt) part += G[idx] * G[idx];
    fro = sqrt(wg_sum(part, red));
  }
  // mode 2: a pivot below the shift is replaced by the shift (modified Cholesky), so a
  // nearly singular Gram matrix is factored in one pass instead of being restarted
  const double floor_piv = (mode == 2) ? shift_rel * fro : 0.0;
  __shared__ int modified;
  if (tid == 0) modified = 0;
  const int attempts = 1;
  for (int att = 0; att < attempts; ++att) {
    const bool shifted = (mode == 1);
    const double s = shifted ? shift_rel * fro : 0.0;
    if (shifted && tid == 0 && shifts) shifts[0] += 1;
    for (size_t idx = tid; idx < (size_t)m * m; idx += nt) {
      const int i = (int)(idx % m), j = (int)(idx / m);
      L[idx] = (i >= j) ? (G[idx] + (i == j ? s : 0.0)) : 0.0;
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int kb = 0; kb < m && !bad; kb += kPB) {
      const int nb = min(kPB, m - kb);
      // 1. diagonal block in LDS, factored by wave 0 alone (no workgroup barriers inside)
      for (int idx = tid; idx < nb * nb; idx += nt) {
        const int i = idx % nb, j = idx / nb;
        D[i][j] = (i >= j) ? L[(size_t)(kb + j) * m + kb + i] : 0.0;
      }
      __syncthreads();
      if (wave == 0) {
        // lane i keeps row i of the diagonal block in registers; column k is broadcast
        // through LDS once per step (independent reads, no read-modify-write chains)
        const int lane = tid & 63;
        double r[kPB];
#pragma unroll
        for (int j = 0; j < kPB; ++j) r[j] = (lane < nb && j <= lane) ? D[lane][j] : 0.0;
        bool fail = false;
#pragma unroll
        for (int k = 0; k < kPB; ++k) {
          if (k < nb && !fail) {
            double piv = __shfl(r[k], k, 64);
            if (!isfinite(piv)) fail = true;
            if (floor_piv > 0.0 && !(piv > floor_piv)) {
              piv = floor_piv;
              if (lane == 0) modified = 1;
            }
            if (!(piv > 0.0)) fail = true;
            if (!fail) {
              const double rkk = sqrt(piv), rinv = 1.0 / rkk;
              if (lane > k) r[k] *= rinv;
              if (lane == k) r[k] = rkk;
              if (lane < nb) D[lane][k] = r[k];  // column k for the other lanes
              asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
              if (lane > k && lane < nb) {
                const double lik = r[k];
#pragma unroll
                for (int j = k + 1; j < kPB; ++j)
                  if (j <= lane) r[j] -= lik * D[j][k];
              }
              asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            }
          }
        }
        if (fail && lane == 0) bad = 1;
        if (lane < nb) {
#pragma unroll
          for (int j = 0; j < kPB; ++j)
            if (j <= lane) D[lane][j] = r[j];
          Dinv[lane] = 1.0 / D[lane][lane];
        }
      }
      __syncthreads();
      if (bad) break;
      for (int idx = tid; idx < nb * nb; idx += nt) {
        const int i = idx % nb, j = idx / nb;
        if (i >= j) L[(size_t)(kb + j) * m + kb + i] = D[i][j];
      }
      // 2. panel rows below: x L11^T = a  (forward substitution per row)
      for (int i = kb + nb + tid; i < m; i += nt) {
        // keep the LDS reads of the diagonal block inside the row loop (no hoisting)
        asm volatile("" ::: "memory");
        double x[kPB];
#pragma unroll
        for (int j = 0; j < kPB; ++j) {
          if (j < nb) {
            double a = L[(size_t)(kb + j) * m + i];
#pragma unroll
            for (int t = 0; t < j; ++t) a -= x[t] * D[j][t];
            x[j] = a * Dinv[j];
          }
        }
#pragma unroll
        for (int j = 0; j < kPB; ++j)
          if (j < nb) L[(size_t)(kb + j) * m + i] = x[j];
      }
      __syncthreads();
      // 3. trailing update A22 -= L21 L21^T on the lower 32 x 32 tiles; the panel
      //    L21 is staged in LDS when it fits (MFMA operands then come from LDS)
      const int r0 = kb + nb;
      const int prow = m - r0;
      const bool staged = prow <= kStageRows;
      if (staged) {
        for (int idx = tid; idx < prow * nb; idx += nt) {
          const int i = idx % prow, j = idx / prow;
          Pn[j * (kStageRows + 1) + i] = L[(size_t)(kb + j) * m + r0 + i];
        }
      }
      __syncthreads();
      const int nt32 = (prow + 31) / 32;
      const int ntiles = nt32 * (nt32 + 1) / 2;
      for (int t = wave; t < ntiles; t += nwaves) {
        int I = 0, rem = t;
        while (rem > I) {
          rem -= I + 1;
          ++I;
        }
        const int J = rem;  // tile (I, J) with J <= I
        const int i0 = r0 + 32 * I, j0 = r0 + 32 * J;
        d4 acc[2][2];
        zero_acc(acc);
        if (staged)
          wave_mma32<false, true>(Pn + 32 * I, kStageRows + 1, Pn + 32 * J, kStageRows + 1, nb,
                                  m - i0, m - j0, acc);
        else
          wave_mma32<false, true>(L + (size_t)kb * m + i0, m, L + (size_t)kb * m + j0, m, nb,
                                  m - i0, m - j0, acc);
        const int lane = tid & 63, li = lane & 15, lg = lane >> 4;
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
          for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = i0 + 16 * rt + lg + 4 * r, col = j0 + 16 * ct + li;
              if (row < m && col < m && row >= col) L[(size_t)col * m + row] -= acc[rt][ct][r];
            }
      }
      __syncthreads();
    }
    __syncthreads();
    if (!bad) {
      if (tid == 0 && modified && shifts) shifts[0] += 1;
      if (tid == 0 && modified && modflag) modflag[0] = 1;
      return;
    }
    __syncthreads();
  }
  if (tid == 0) flag[0] = 1;
}

// ---------------------------------------------------------------------------
// X <- X L^{-T} for X (rows x m, leading dimension ldx) and lower-triangular L (m x m):
// the right-hand triangular solve of CholeskyQR (Q = Y R^{-1} with R = L^T). One wave
// per block of 32 rows; per 32-column block jb the wave forms
// B = X[:, jb] - Q[:, <jb] L[jb, <jb]^T with FP64 MFMA, then solves B = Q_jb L_jb^T
// row by row in LDS. Rows are independent, so X is overwritten in place.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64)
    trsm_rlt_kernel(int rows, int m, double *__restrict__ X, int ldx, const double *__restrict__ L,
                    const int *__restrict__ run) {
  if (run && run[0] == 0) return;
  __shared__ double B[32][33];
  __shared__ double Ld[32][33];
  const int lane = threadIdx.x, li = lane & 15, lg = lane >> 4;
  const int r0 = blockIdx.x * 32;
  const int nr = min(32, rows - r0);
  for (int jb = 0; jb * 32 < m; ++jb) {
    const int c0 = jb * 32, nc = min(32, m - c0);
    d4 acc[2][2];
    zero_acc(acc);
    if (c0 > 0)  // Q[:, 0:c0] L[c0:c0+32, 0:c0]^T
      wave_mma32<false, true>(X + r0 + (size_t)0 * ldx, ldx, L + c0, m, c0, nr, nc, acc);
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * rt + lg + 4 * r, col = 16 * ct + li;
          double v = 0.0;
          if (row < nr && col < nc) v = X[(size_t)(c0 + col) * ldx + r0 + row] - acc[rt][ct][r];
          B[row][col] = v;
        }
    for (int idx = lane; idx < 32 * 32; idx += 64) {
      const int i = idx & 31, j = idx >> 5;
      Ld[i][j] = (i < nc && j < nc && i >= j) ? L[(size_t)(c0 + j) * m + c0 + i] : 0.0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // lane = row: q L_jb^T = b  ->  q_j = (b_j - sum_{t<j} q_t L[j][t]) / L[j][j]
    if (lane < nr) {
      double q[32];
#pragma unroll
      for (int j = 0; j < 32; ++j) {
        if (j < nc) {
          double a = B[lane][j];
#pragma unroll
          for (int t = 0; t < j; ++t) a -= q[t] * Ld[j][t];
          q[j] = a / Ld[j][j];
        }
      }
#pragma unroll
      for (int j = 0; j < 32; ++j)
        if (j < nc) X[(size_t)(c0 + j) * ldx + r0 + lane] = q[j];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// ---------------------------------------------------------------------------
// Blocked inverse of a lower-triangular L (column-major): X = L^{-1}.
// Diagonal 32 x 32 blocks are inverted by substitution in LDS; then, block row
// by block row, X_ij = -X_ii (sum_{k=j}^{i-1} L_ik X_kj) with FP64 MFMA.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kCholThreads)
    trinv_lower_blocked_kernel(int m, const double *__restrict__ L, double *__restrict__ X) {
  __shared__ double S[kCholThreads / 64][kPB][kPB + 1];  // per-wave staging of one 32 x 32 block
  const int tid = threadIdx.x, nt = blockDim.x;
  const int wave = tid >> 6, nwaves = nt >> 6, lane = tid & 63;
  const int nbk = (m + kPB - 1) / kPB;
  for (size_t idx = tid; idx < (size_t)m * m; idx += nt) X[idx] = 0.0;
  __syncthreads();
  // diagonal blocks: staged in LDS; lane c of a half-wave solves column c of L_ii x = e_c
  for (int b0 = wave * 2; b0 < nbk; b0 += 2 * nwaves) {
    const int half = lane >> 5, c = lane & 31;
    const int b = b0 + half;
    if (b < nbk) {
      const int k0 = b * kPB, nb = min(kPB, m - k0);
      if (c < nb) {
        double x[kPB];
#pragma unroll
        for (int i = 0; i < kPB; ++i) {
          if (i < nb) {
            double a = (i == c) ? 1.0 : 0.0;
#pragma unroll
            for (int t = 0; t < i; ++t) a -= L[(size_t)(k0 + t) * m + k0 + i] * x[t];
            x[i] = (i < c) ? 0.0 : a / L[(size_t)(k0 + i) * m + k0 + i];
          }
        }
#pragma unroll
        for (int i = 0; i < kPB; ++i)
          if (i < nb && i >= c) X[(size_t)(k0 + c) * m + k0 + i] = x[i];
      }
    }
  }
  __syncthreads();
  const int li = lane & 15, lg = lane >> 4;
  for (int bi = 1; bi < nbk; ++bi) {
    const int i0 = bi * kPB, ni = min(kPB, m - i0);
    for (int bj = wave; bj < bi; bj += nwaves) {
      const int j0 = bj * kPB;
      d4 acc[2][2];
      zero_acc(acc);
      // T = sum_{k=j}^{i-1} L_ik X_kj  (rows i0.., cols j0.., K over rows j0..i0-1)
      wave_mma32<false, false>(L + (size_t)j0 * m + i0, m, X + (size_t)j0 * m + j0, m, i0 - j0, ni,
                               kPB, acc);
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
          for (int r = 0; r < 4; ++r) S[wave][16 * rt + lg + 4 * r][16 * ct + li] = acc[rt][ct][r];
      // the block is re-read by other lanes of the same wave
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // X_ij = -X_ii T : X_ii from global, T from LDS (row-major, stride kPB + 1)
      zero_acc(acc);
      wave_mma32<false, true>(X + (size_t)i0 * m + i0, m, &S[wave][0][0], kPB + 1, ni, ni, kPB,
                              acc);
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = i0 + 16 * rt + lg + 4 * r, col = j0 + 16 * ct + li;
            if (row < m && col < m) X[(size_t)col * m + row] = -acc[rt][ct][r];
          }
      // S[wave] is rewritten by this wave's next block
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Cholesky: G + s I = R^T R, R upper triangular (right-looking).
// ---------------------------------------------------------------------------

// mode 0: plain; mode 1: shifted (s = shift_rel * ||G||_F); mode 2: plain, and on
// breakdown restart from G with the shift. Each shifted attempt increments *shifts.
__global__ void __launch_bounds__(1024)
    cholesky_kernel(int m, const double *__restrict__ G, double *__restrict__ R, double shift_rel,
                    int mode, int *__restrict__ flag, int *__restrict__ shifts) {
  extern __shared__ double rowk[];
  __shared__ double red[16];
  double fro = 0.0;
  if (mode != 0) {
    double part = 0.0;
    for (size_t idx = threadIdx.x; idx < (size_t)m * m; idx += blockDim.x) part += G[idx] * G[idx];
    fro = sqrt(wg_sum(part, red));
  }
  const int attempts = (mode == 2) ? 2 : 1;
  for (int att = 0; att < attempts; ++att) {
    const bool shifted = (mode == 1) || (mode == 2 && att == 1);
    const double s = shifted ? shift_rel * fro : 0.0;
    if (shifted && threadIdx.x == 0 && shifts) shifts[0] += 1;
    for (size_t idx = threadIdx.x; idx < (size_t)m * m; idx += blockDim.x) {
      const int i = (int)(idx % m), j = (int)(idx / m);
      R[idx] = (i <= j) ? (G[idx] + (i == j ? s : 0.0)) : 0.0;
    }
    __syncthreads();
    bool ok = true;
    for (int k = 0; k < m; ++k) {
      const double piv = R[(size_t)k * m + k];
      if (!(piv > 0.0) || !isfinite(piv)) {
        ok = false;  // uniform: every thread read the same pivot
        break;
      }
      const double rkk = sqrt(piv);
      const double inv = 1.0 / rkk;
      for (int j = k + threadIdx.x; j < m; j += blockDim.x) {
        const double v = (j == k) ? rkk : R[(size_t)j * m + k] * inv;
        rowk[j] = v;
      }
      __syncthreads();
      for (int j = k + threadIdx.x; j < m; j += blockDim.x) R[(size_t)j * m + k] = rowk[j];
      const int len = m - k - 1;
      const size_t tot = (size_t)len * len;
      for (size_t idx = threadIdx.x; idx < tot; idx += blockDim.x) {
        const int i = k + 1 + (int)(idx % len), j = k + 1 + (int)(idx / len);
        if (i <= j) R[(size_t)j * m + i] -= rowk[i] * rowk[j];
      }
      __syncthreads();
    }
    if (ok) return;
    __syncthreads();
  }
  if (threadIdx.x == 0) flag[0] = 1;
}

// Upper-triangular inverse by column-oriented back substitution on all columns at once.
__global__ void __launch_bounds__(1024)
    trinv_upper_kernel(int m, const double *__restrict__ R, double *__restrict__ X) {
  extern __shared__ double colr[];
  for (size_t idx = threadIdx.x; idx < (size_t)m * m; idx += blockDim.x) {
    const int i = (int)(idx % m), j = (int)(idx / m);
    X[idx] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int i = m - 1; i >= 0; --i) {
    const double inv = 1.0 / R[(size_t)i * m + i];
    for (int r = threadIdx.x; r < i; r += blockDim.x) colr[r] = R[(size_t)i * m + r];
    // scale row i of X (columns j >= i)
    for (int j = i + threadIdx.x; j < m; j += blockDim.x) X[(size_t)j * m + i] *= inv;
    __syncthreads();
    // X[r, j] -= R[r, i] * X[i, j] for r < i <= j
    const size_t tot = (size_t)i * (m - i);
    for (size_t idx = threadIdx.x; idx < tot; idx += blockDim.x) {
      const int r = (int)(idx % i), j = i + (int)(idx / i);
      X[(size_t)j * m + r] -= colr[r] * X[(size_t)j * m + i];
    }
    __syncthreads();
  }
}

// Gauss-Jordan inverse with partial pivoting. work = [W | X] (2 m x m).
__global__ void __launch_bounds__(1024)
    gj_inverse_kernel(int m, const double *__restrict__ Min, double *__restrict__ Minv,
                      double *__restrict__ work, int *__restrict__ flag) {
  extern __shared__ double sh[];
  double *prow_w = sh;      // pivot row of W (m)
  double *prow_x = sh + m;  // pivot row of X (m)
  double *colk = sh + 2 * m;
  __shared__ double redv[16];
  __shared__ int redi[16];
  double *W = work, *X = Minv;
  for (size_t idx = threadIdx.x; idx < (size_t)m * m; idx += blockDim.x) {
    const int i = (int)(idx % m), j = (int)(idx / m);
    W[idx] = Min[idx];
    X[idx] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    // pivot search in column k, rows k..m-1
    double best = -1.0;
    int cand = -1;
    double cv = 0.0;
    for (int i = k + threadIdx.x; i < m; i += blockDim.x) {
      const double v = fabs(W[(size_t)k * m + i]);
      if (v > best || cand < 0) {
        best = v;
        cand = i;
        cv = v;
      }
    }
    double pv;
    const int p = wg_argmax_abs(cand >= 0 ? cv : 0.0, cand, redv, redi, &pv);
    if (!(pv > 0.0) || !isfinite(pv) || p < 0) {
      if (threadIdx.x == 0) flag[0] = 1;
      return;
    }
    // swap rows k and p (W columns k..m-1, X all columns), load pivot rows
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
      if (j >= k) {
        const double a = W[(size_t)j * m + k], b = W[(size_t)j * m + p];
        W[(size_t)j * m + k] = b;
        W[(size_t)j * m + p] = a;
      }
      const double c = X[(size_t)j * m + k], d = X[(size_t)j * m + p];
      X[(size_t)j * m + k] = d;
      X[(size_t)j * m + p] = c;
    }
    __syncthreads();
    const double inv = 1.0 / W[(size_t)k * m + k];
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
      const double wv = (j >= k) ? W[(size_t)j * m + k] * inv : 0.0;
      const double xv = X[(size_t)j * m + k] * inv;
      prow_w[j] = wv;
      prow_x[j] = xv;
      if (j >= k) W[(size_t)j * m + k] = wv;
      X[(size_t)j * m + k] = xv;
    }
    for (int i = threadIdx.x; i < m; i += blockDim.x) colk[i] = W[(size_t)k * m + i];
    __syncthreads();
    // eliminate column k from every other row
    const size_t tot = (size_t)m * m;
    for (size_t idx = threadIdx.x; idx < tot; idx += blockDim.x) {
      const int i = (int)(idx % m), j = (int)(idx / m);
      if (i == k) continue;
      const double c = colk[i];
      if (c == 0.0) continue;
      if (j > k) W[idx] -= c * prow_w[j];
      X[idx] -= c * prow_x[j];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += blockDim.x)
      if (i != k) W[(size_t)k * m + i] = 0.0;
    __syncthreads();
  }
}

// K <- (K + K^T)/2 over the strict lower triangle, many workgroups; per-block partial
// sums of ||K - K^T||^2 and ||K||^2 are reduced by symmetrize_norm_kernel in fixed order.
__global__ void __launch_bounds__(256) symmetrize_kernel(int m, double *__restrict__ K,
                                                         double *__restrict__ part) {
  __shared__ double red[16];
  const size_t tot = (size_t)m * m;
  double pa = 0.0, pk = 0.0;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % m), j = (int)(idx / m);
    const double a = K[idx];
    pk += a * a;
    if (i > j) {
      const double b = K[(size_t)i * m + j];
      pa += 2.0 * (a - b) * (a - b);
      const double v = 0.5 * (a + b);
      K[idx] = v;
      K[(size_t)i * m + j] = v;
    }
  }
  const double sa = wg_sum(pa, red);
  const double sk = wg_sum(pk, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sa;
    part[2 * blockIdx.x + 1] = sk;
  }
}

__global__ void symmetrize_norm_kernel(int nblk, const double *__restrict__ part,
                                       double *__restrict__ asym) {
  if (threadIdx.x != 0) return;
  double sa = 0.0, sk = 0.0;
  for (int b = 0; b < nblk; ++b) {
    sa += part[2 * b];
    sk += part[2 * b + 1];
  }
  asym[0] = sk > 0.0 ? sqrt(sa / sk) : 0.0;
}

__global__ void __launch_bounds__(1024) orth_err_kernel(int m, const double *__restrict__ G,
                                                        double *__restrict__ out) {
  __shared__ double red[16];
  double p = 0.0;
  for (size_t idx = threadIdx.x; idx < (size_t)m * m; idx += blockDim.x) {
    const int i = (int)(idx % m), j = (int)(idx / m);
    const double v = G[idx] - (i == j ? 1.0 : 0.0);
    p += v * v;
  }
  const double s = wg_sum(p, red);
  if (threadIdx.x == 0) out[0] = sqrt(s);
}

// ---------------------------------------------------------------------------
// Symmetric eigen-solver: Householder tridiagonalisation, implicit QL with
// Wilkinson-type shifts (the QL sweep's rotations are generated by one thread
// and applied to the rows of Z by all threads), back-transformation by the
// Householder reflectors (one wave per column) and a descending sort.
// ---------------------------------------------------------------------------

// work layout: Aw [m*m] | Hv [m*m] | Z [m*m] | d [m] | e [m]
__host__ __device__ size_t syev_layout(int m, size_t off[5]) {
  const size_t mm = (size_t)m * m;
  off[0] = 0;
  off[1] = mm;
  off[2] = 2 * mm;
  off[3] = 3 * mm;
  off[4] = 3 * mm + m;
  return 3 * mm + 2 * (size_t)m;
}

__global__ void __launch_bounds__(1024)
    tridiag_ql_kernel(int m, const double *__restrict__ K, double *__restrict__ work,
                      int *__restrict__ flag) {
  extern __shared__ double sh[];
  size_t off[5];
  syev_layout(m, off);
  double *Aw = work + off[0], *Hv = work + off[1], *Z = work + off[2];
  double *dg = work + off[3], *eg = work + off[4];
  double *vs = sh;          // Householder vector (m)
  double *ps = sh + m;      // p / w (m)
  double *cs = sh + 2 * m;  // rotation cosines (m)
  double *sn = sh + 3 * m;  // rotation sines (m)
  double *part = sh + 4 * m;  // symv partials (blockDim)
  __shared__ double red[16];
  __shared__ int ctl[4];
  const int tid = threadIdx.x, nt = blockDim.x;
  const size_t mm = (size_t)m * m;
  for (size_t idx = tid; idx < mm; idx += nt) {
    Aw[idx] = K[idx];
    Hv[idx] = 0.0;
  }
  __syncthreads();
  // ---- tridiagonalisation ----
  for (int k = 0; k + 2 < m; ++k) {
    const int R = m - k - 1;  // length of the trailing block
    double part_s = 0.0;
    for (int i = tid; i < R; i += nt) {
      const double x = Aw[(size_t)k * m + k + 1 + i];
      vs[i] = x;
      part_s += x * x;
    }
    const double sig2 = wg_sum(part_s, red);
    const double sig = sqrt(sig2);
    const double x0 = vs[0];
    __syncthreads();
    if (sig == 0.0) {
      if (tid == 0) {
        dg[k] = Aw[(size_t)k * m + k];
        eg[k] = 0.0;
      }
      __syncthreads();
      continue;
    }
    const double alpha = (x0 >= 0.0) ? -sig : sig;
    // v = x - alpha e1, normalised: ||v||^2 = sig^2 - 2 alpha x0 + alpha^2 = 2 (sig^2 - alpha x0)
    const double vn = sqrt(2.0 * (sig2 - alpha * x0));
    if (tid == 0) vs[0] = x0 - alpha;
    __syncthreads();
    for (int i = tid; i < R; i += nt) {
      const double v = vs[i] / vn;
      vs[i] = v;
      Hv[(size_t)k * m + k + 1 + i] = v;
    }
    __syncthreads();
    // p = S v with S = Aw[k+1:, k+1:] (thread groups split the column range)
    const int groups = max(1, nt / R);
    {
      const int i = tid % R, g = tid / R;
      double acc = 0.0;
      if (g < groups) {
        for (int j = g; j < R; j += groups)
          acc += Aw[(size_t)(k + 1 + j) * m + (k + 1 + i)] * vs[j];
      }
      if (tid < R * groups) part[tid] = acc;
      // rows beyond nt (R > nt) handled by the loop below
    }
    __syncthreads();
    if (R <= nt) {
      for (int i = tid; i < R; i += nt) {
        double s = 0.0;
        for (int g = 0; g < groups; ++g) s += part[g * R + i];
        ps[i] = s;
      }
    } else {
      for (int i = tid; i < R; i += nt) {
        double s = 0.0;
        for (int j = 0; j < R; ++j) s += Aw[(size_t)(k + 1 + j) * m + (k + 1 + i)] * vs[j];
        ps[i] = s;
      }
    }
    __syncthreads();
    double kp = 0.0;
    for (int i = tid; i < R; i += nt) kp += vs[i] * ps[i];
    const double Kv = wg_sum(kp, red);
    for (int i = tid; i < R; i += nt) ps[i] = ps[i] - Kv * vs[i];
    __syncthreads();
    const size_t tot = (size_t)R * R;
    for (size_t idx = tid; idx < tot; idx += nt) {
      const int i = (int)(idx % R), j = (int)(idx / R);
      Aw[(size_t)(k + 1 + j) * m + (k + 1 + i)] -= 2.0 * (vs[i] * ps[j] + ps[i] * vs[j]);
    }
    if (tid == 0) {
      dg[k] = Aw[(size_t)k * m + k];
      eg[k] = alpha;
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (m >= 2) {
      dg[m - 2] = Aw[(size_t)(m - 2) * m + m - 2];
      dg[m - 1] = Aw[(size_t)(m - 1) * m + m - 1];
      eg[m - 2] = Aw[(size_t)(m - 2) * m + m - 1];
    } else {
      dg[0] = Aw[0];
    }
    eg[m - 1] = 0.0;
  }
  // Z = I (eigenvectors of T, column-major)
  for (size_t idx = tid; idx < mm; idx += nt) {
    const int i = (int)(idx % m), j = (int)(idx / m);
    Z[idx] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  // ---- implicit QL on (d, e) ----
  const double eps = 0x1.0p-52;
  for (int l = 0; l < m; ++l) {
    int iter = 0;
    while (true) {
      if (tid == 0) {
        int mmi;
        for (mmi = l; mmi < m - 1; ++mmi) {
          const double dd = fabs(dg[mmi]) + fabs(dg[mmi + 1]);
          if (fabs(eg[mmi]) <= eps * dd) break;
        }
        ctl[0] = mmi;  // end of the unreduced block
        ctl[1] = -1;   // lowest rotation index applied (none)
        ctl[2] = 0;    // failure
        if (mmi != l) {
          if (iter >= 60) {
            ctl[2] = 1;
          } else {
            double g = (dg[l + 1] - dg[l]) / (2.0 * eg[l]);
            double r = hypot(g, 1.0);
            g = dg[mmi] - dg[l] + eg[l] / (g + copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            int i;
            bool under = false;
            for (i = mmi - 1; i >= l; --i) {
              double f = s * eg[i];
              const double b = c * eg[i];
              r = hypot(f, g);
              eg[i + 1] = r;
              if (r == 0.0) {
                dg[i + 1] -= p;
                eg[mmi] = 0.0;
                under = true;
                break;
              }
              s = f / r;
              c = g / r;
              g = dg[i + 1] - p;
              r = (dg[i] - g) * s + 2.0 * c * b;
              p = s * r;
              dg[i + 1] = g + p;
              g = c * r - b;
              cs[i] = c;
              sn[i] = s;
            }
            ctl[1] = under ? i + 1 : l;
            if (!under) {
              dg[l] -= p;
              eg[l] = g;
              eg[mmi] = 0.0;
            }
          }
        }
      }
      __syncthreads();
      const int mmi = ctl[0], lo = ctl[1], failed = ctl[2];
      __syncthreads();  // everyone has read ctl before thread 0 rewrites it
      if (failed) {
        if (tid == 0) flag[0] = 1;
        return;
      }
      if (mmi == l) break;
      ++iter;
      // apply rotations i = mmi-1 .. lo to columns (i, i+1) of every row of Z
      for (int row = tid; row < m; row += nt) {
        double carry = Z[(size_t)mmi * m + row];
        for (int i = mmi - 1; i >= lo; --i) {
          const double zi = Z[(size_t)i * m + row];
          Z[(size_t)(i + 1) * m + row] = sn[i] * zi + cs[i] * carry;
          carry = cs[i] * zi - sn[i] * carry;
        }
        Z[(size_t)lo * m + row] = carry;
      }
      __syncthreads();
    }
  }
}

// Back-transformation Z <- H_0 ... H_{m-3} Z and descending sort into (lam, Vout).
// One wave per column of Z.
__global__ void __launch_bounds__(256)
    syev_backtransform_kernel(int m, const double *__restrict__ work, double *__restrict__ lam,
                              double *__restrict__ Vout) {
  size_t off[5];
  syev_layout(m, off);
  const double *Hv = work + off[1], *Z = work + off[2], *dg = work + off[3];
  const int lane = threadIdx.x & 63;
  const int col = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (col >= m) return;
  constexpr int kMaxPer = 17;  // m <= 1088
  double z[kMaxPer];
#pragma unroll
  for (int q = 0; q < kMaxPer; ++q) {
    const int i = lane + 64 * q;
    z[q] = (i < m) ? Z[(size_t)col * m + i] : 0.0;
  }
  for (int k = m - 3; k >= 0; --k) {
    const double *v = Hv + (size_t)k * m;
    double dot = 0.0;
#pragma unroll
    for (int q = 0; q < kMaxPer; ++q) {
      const int i = lane + 64 * q;
      if (i > k && i < m) dot += v[i] * z[q];
    }
    for (int o = 32; o > 0; o >>= 1) dot += __shfl_xor(dot, o, 64);
#pragma unroll
    for (int q = 0; q < kMaxPer; ++q) {
      const int i = lane + 64 * q;
      if (i > k && i < m) z[q] -= 2.0 * dot * v[i];
    }
  }
  // rank in descending order (ties by index)
  const double dj = dg[col];
  int rank = 0;
  for (int i = lane; i < m; i += 64) {
    const double di = dg[i];
    rank += (di > dj || (di == dj && i < col)) ? 1 : 0;
  }
  for (int o = 32; o > 0; o >>= 1) rank += __shfl_xor(rank, o, 64);
  if (lane == 0) lam[rank] = dj;
#pragma unroll
  for (int q = 0; q < kMaxPer; ++q) {
    const int i = lane + 64 * q;
    if (i < m) Vout[(size_t)rank * m + i] = z[q];
  }
}

// ---------------------------------------------------------------------------
// Increment, covariance and utility kernels
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool use_lru(int mode_lru, const double *lam, int k) {
  if (mode_lru == 0) return false;
  if (mode_lru == 1) return true;
  return !(lam[k - 1] >= 1.0);  // adaptive (eq. 11)
}

__global__ void increment_kernel(int n, int k, const double *__restrict__ lam,
                                 const double *__restrict__ V, const double *__restrict__ c,
                                 const double *__restrict__ g, int mode_lru,
                                 double *__restrict__ dz, double *__restrict__ dofs) {
  const bool lru = use_lru(mode_lru, lam, k);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    double s = 0.0;
    for (int j = 0; j < k; ++j) {
      const double lj = lam[j];
      const double a = lru ? lj / (1.0 + lj) : 1.0 / (1.0 + lj);
      s += V[(size_t)j * n + i] * (c[j] * a);
    }
    dz[i] = lru ? -(g[i] - s) : -s;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && dofs) {
    double d = 0.0;
    for (int j = 0; j < k; ++j) d += lam[j] / (1.0 + lam[j]);
    dofs[0] = d;
  }
}

__global__ void choose_mode_kernel(int k, const double *__restrict__ lam, int *__restrict__ out) {
  if (threadIdx.x == 0) out[0] = (lam[k - 1] >= 1.0) ? (int)RIOT_LRA : (int)RIOT_LRU;
}

__global__ void postcov_diag_kernel(int n, int k, const double *__restrict__ lam,
                                    const double *__restrict__ W, int mode_lru, double base_diag,
                                    double *__restrict__ coef, double *__restrict__ diag) {
  const bool lru = use_lru(mode_lru, lam, k);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0 && coef) {
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
      const double lj = lam[j];
      coef[j] = lru ? -lj / (1.0 + lj) : 1.0 / (1.0 + lj);
    }
  }
  if (i < n && diag) {
    double s = lru ? base_diag : 0.0;
    for (int j = 0; j < k; ++j) {
      const double lj = lam[j];
      const double cj = lru ? -lj / (1.0 + lj) : 1.0 / (1.0 + lj);
      const double w = W[(size_t)j * n + i];
      s += cj * w * w;
    }
    diag[i] = s;
  }
}

__global__ void dense_B_kernel(int n, const double *__restrict__ brow, double beta,
                               double *__restrict__ P, const int *__restrict__ mode) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * n) return;
  if (mode && mode[0] != (int)RIOT_LRU) return;
  const int i = (int)(idx % n), j = (int)(idx / n);
  int d = i - j;
  if (d < 0) d += n;
  const double b = brow[d];
  P[idx] = (beta != 0.0 ? beta * P[idx] : 0.0) + b;
}

__global__ void scale_cols_kernel(int n, int k, const double *__restrict__ X,
                                  const double *__restrict__ s, double *__restrict__ Y) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * k) return;
  Y[idx] = X[idx] * s[idx / n];
}

__global__ void zero_ints_kernel(int *__restrict__ p, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0;
}

__global__ void check_finite_kernel(long long count, const double *__restrict__ x,
                                    int *__restrict__ flag) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  bool bad = false;
  for (; i < count; i += stride) bad |= !isfinite(x[i]);
  if (bad) flag[0] = 1;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t gemm_f64(int ta, int tb, int M, int N, int K, double alpha, const double *A, int lda,
                    const double *B, int ldb, double beta, double *C, int ldc, double *partial,
                    int splitk, hipStream_t st, const int *run) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (K <= 0) splitk = 1;
  if (splitk < 1 || !partial) splitk = 1;
  int kchunk = (K + splitk - 1) / splitk;
  kchunk = (kchunk + 3) / 4 * 4;
  if (kchunk <= 0) kchunk = 4;
  const int splits = K > 0 ? (K + kchunk - 1) / kchunk : 1;
  dim3 grid((M + 31) / 32, (N + 31) / 32, splits);
  double *part = splits > 1 ? partial : nullptr;
#define RIOT_GEMM(TA_, TB_)                                                                  \
  hipLaunchKernelGGL((gemm_mfma_kernel<TA_, TB_>), grid, dim3(64), 0, st, M, N, K, A, lda, B, \
                     ldb, C, ldc, alpha, beta, kchunk, part, run)
  if (ta == 0 && tb == 0)
    RIOT_GEMM(0, 0);
  else if (ta == 1 && tb == 0)
    RIOT_GEMM(1, 0);
  else if (ta == 0 && tb == 1)
    RIOT_GEMM(0, 1);
  else
    RIOT_GEMM(1, 1);
#undef RIOT_GEMM
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (splits > 1) {
    const size_t MN = (size_t)M * N;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((MN + 255) / 256)), dim3(256), 0, st,
                       M, N, splits, partial, alpha, beta, C, ldc, run);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_cholesky(int m, const double *G, double *R, double shift_rel, int mode,
                           int *flag, int *shifts, hipStream_t st) {
  hipLaunchKernelGGL(cholesky_kernel, dim3(1), dim3(1024), (size_t)m * sizeof(double), st, m, G, R,
                     shift_rel, mode, flag, shifts);
  return hipGetLastError();
}

hipError_t launch_chol_blocked(int m, const double *G, double *L, double shift_rel, int mode,
                               int *flag, int *shifts, hipStream_t st, const int *run,
                               int *modflag) {
  hipLaunchKernelGGL(chol_blocked_kernel, dim3(1), dim3(kCholThreads), 0, st, m, G, L, shift_rel,
                     mode, flag, shifts, run, modflag);
  return hipGetLastError();
}

hipError_t launch_trsm_rlt(int rows, int m, double *X, int ldx, const double *L, hipStream_t st,
                           const int *run) {
  if (rows <= 0 || m <= 0) return hipSuccess;
  hipLaunchKernelGGL(trsm_rlt_kernel, dim3((rows + 31) / 32), dim3(64), 0, st, rows, m, X, ldx, L,
                     run);
  return hipGetLastError();
}

// CholeskyQR pass control, one thread. cq[0]: further passes run; cq[1]: consecutive
// clean passes (plain Cholesky, no pivot replaced); cq[2]: a pivot was replaced in the
// pass just finished. Two clean passes in a row leave the block orthonormal to rounding.
__global__ void cholqr_ctrl_kernel(int *cq, int pass_was_shifted, int *count) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (cq[0] == 0) return;
  if (count) count[0] += 1;
  if (pass_was_shifted || cq[2])
    cq[1] = 0;
  else
    cq[1] += 1;
  cq[2] = 0;
  if (cq[1] >= 2) cq[0] = 0;
}

__global__ void cholqr_reset_kernel(int *cq) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    cq[0] = 1;
    cq[1] = 0;
    cq[2] = 0;
  }
}

hipError_t launch_cholqr_reset(int *cq, hipStream_t st) {
  hipLaunchKernelGGL(cholqr_reset_kernel, dim3(1), dim3(64), 0, st, cq);
  return hipGetLastError();
}

hipError_t launch_cholqr_ctrl(int *cq, int pass_was_shifted, int *count, hipStream_t st) {
  hipLaunchKernelGGL(cholqr_ctrl_kernel, dim3(1), dim3(64), 0, st, cq, pass_was_shifted, count);
  return hipGetLastError();
}

hipError_t launch_trinv_lower(int m, const double *L, double *X, hipStream_t st) {
  hipLaunchKernelGGL(trinv_lower_blocked_kernel, dim3(1), dim3(kCholThreads), 0, st, m, L, X);
  return hipGetLastError();
}

hipError_t launch_trinv_upper(int m, const double *R, double *Rinv, hipStream_t st) {
  hipLaunchKernelGGL(trinv_upper_kernel, dim3(1), dim3(1024), (size_t)m * sizeof(double), st, m, R,
                     Rinv);
  return hipGetLastError();
}

hipError_t launch_gj_inverse(int m, const double *M, double *Minv, double *work, int *flag,
                             hipStream_t st) {
  hipLaunchKernelGGL(gj_inverse_kernel, dim3(1), dim3(1024), (size_t)3 * m * sizeof(double), st, m,
                     M, Minv, work, flag);
  return hipGetLastError();
}

hipError_t launch_symmetrize(int m, double *K, double *asym, double *part, hipStream_t st) {
  const int nblk = 64;
  hipLaunchKernelGGL(symmetrize_kernel, dim3(nblk), dim3(256), 0, st, m, K, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(symmetrize_norm_kernel, dim3(1), dim3(64), 0, st, nblk, part, asym);
  return hipGetLastError();
}

hipError_t launch_orth_err(int m, const double *G, double *out, hipStream_t st) {
  hipLaunchKernelGGL(orth_err_kernel, dim3(1), dim3(1024), 0, st, m, G, out);
  return hipGetLastError();
}

size_t syev_work_doubles(int m) {
  size_t off[5];
  return syev_layout(m, off);
}

hipError_t launch_syev(int m, const double *K, double *lam, double *Z, double *work, int *flag,
                       hipStream_t st) {
  if (m > 1088) return hipErrorInvalidValue;
  const size_t lds = (size_t)(4 * m + 1024) * sizeof(double);
  hipLaunchKernelGGL(tridiag_ql_kernel, dim3(1), dim3(1024), lds, st, m, K, work, flag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int cols_per_block = 4;
  hipLaunchKernelGGL(syev_backtransform_kernel, dim3((m + cols_per_block - 1) / cols_per_block),
                     dim3(64 * cols_per_block), 0, st, m, work, lam, Z);
  return hipGetLastError();
}

hipError_t launch_increment_combine(int n, int k, const double *lam, const double *V,
                                    const double *c, const double *g, int mode_lru, double *dz,
                                    double *dofs, hipStream_t st) {
  hipLaunchKernelGGL(increment_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, k, lam, V, c, g,
                     mode_lru, dz, dofs);
  return hipGetLastError();
}

hipError_t launch_choose_mode(int k, const double *lam, int *out, hipStream_t st) {
  hipLaunchKernelGGL(choose_mode_kernel, dim3(1), dim3(64), 0, st, k, lam, out);
  return hipGetLastError();
}

hipError_t launch_postcov_diag(int n, int k, const double *lam, const double *W, int mode_lru,
                               double base_diag, double *coef, double *diag, hipStream_t st) {
  hipLaunchKernelGGL(postcov_diag_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, k, lam, W,
                     mode_lru, base_diag, coef, diag);
  return hipGetLastError();
}

hipError_t launch_dense_B(int n, const double *brow, double beta, double *P, const int *mode,
                          hipStream_t st) {
  const size_t tot = (size_t)n * n;
  hipLaunchKernelGGL(dense_B_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, brow,
                     beta, P, mode);
  return hipGetLastError();
}

hipError_t launch_scale_cols(int n, int k, const double *X, const double *s, double *Y,
                             hipStream_t st) {
  const size_t tot = (size_t)n * k;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(scale_cols_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, k,
                     X, s, Y);
  return hipGetLastError();
}

hipError_t launch_zero_ints(int *p, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, st, p, count);
  return hipGetLastError();
}

hipError_t launch_check_finite(long long count, const double *x, int *flag, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  long long blocks = (count + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(check_finite_kernel, dim3((unsigned)blocks), dim3(256), 0, st, count, x, flag);
  return hipGetLastError();
}

}  // namespace riot
