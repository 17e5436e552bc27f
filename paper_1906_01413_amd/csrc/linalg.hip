// Dense FP64 linear algebra of the RSVD stages (Alg. 3: orthonormal basis of Y,
// solve for K, eigendecomposition of K, Ritz vectors) for gfx950.
//
//  - gemm_f64: tall-skinny products (Y^T Y, Q^T Y, Q^T Omega, Q Z, W C W^T) on the
//    FP64 matrix cores (v_mfma_f64_16x16x4_f64), split-K with a fixed-order
//    reduction for the A^T B shape; a strided-batched form.
//  - the m x m Cholesky of CholeskyQR (one workgroup; shifted and modified-pivot
//    modes) and the right-hand triangular solve Q = Y L^{-T};
//  - CholeskyQR pass control, symmetrisation, increment and covariance kernels, and
//    their batched forms. The eigen-solver is in eig.hip.

#include "riot_internal.h"
#include "mfma_tile.h"

namespace riot {
namespace {


// ---------------------------------------------------------------------------
// GEMM on the FP64 matrix cores. One wave computes a 32 x 32 tile of C as a
// 2 x 2 grid of 16 x 16 MFMA tiles. Operand lane layout of
// v_mfma_f64_16x16x4_f64: lane l supplies A[i = l % 16][k = l / 16] and
// B[k = l / 16][j = l % 16]; result register r of lane l is
// C[l / 16 + 4 * r][l % 16] (checked on gfx950 with an exact-integer probe).
// ---------------------------------------------------------------------------

template <int TA, int TB, bool LOWER = false>
__global__ void __launch_bounds__(64)
    gemm_mfma_kernel(int M, int N, int K, const double *__restrict__ A, int lda,
                     const double *__restrict__ B, int ldb, double *__restrict__ C, int ldc,
                     double alpha, double beta, int kchunk, double *__restrict__ partial,
                     const int *__restrict__ run, const GemmJob *__restrict__ jobs,
                     long long sA = 0, long long sB = 0, long long sC = 0) {
  int kz = blockIdx.z;
  if (sA | sB | sC) {  // strided batch: blockIdx.z selects the matrices, no split over K
    A += sA * blockIdx.z;
    B += sB * blockIdx.z;
    C += sC * blockIdx.z;
    kchunk = K;
    partial = nullptr;
    kz = 0;
  }
  if (jobs) {  // batched: blockIdx.z selects the problem, no split over K
    const GemmJob &J = jobs[blockIdx.z];
    M = J.M, N = J.N, K = J.K, A = J.A, lda = J.lda, B = J.B, ldb = J.ldb, C = J.C, ldc = J.ldc;
    run = J.run;
    kchunk = K;
    partial = nullptr;
    kz = 0;
  }
  if (run && run[0] == 0) return;  // predicated launch: the whole grid skips uniformly
  const int lane = threadIdx.x;
  const int li = lane & 15, lg = lane >> 4;
  const int m0 = blockIdx.x * 32, n0 = blockIdx.y * 32;
  if (m0 >= M || n0 >= N) return;
  if (LOWER && blockIdx.y > blockIdx.x) return;  // symmetric result: tiles above the diagonal
  const int kbeg = kz * kchunk;
  const int kend = min(K, kbeg + kchunk);
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

  // the wave's share of the contraction, in chunks of 16 with the next chunk's operands in
  // flight while the current chunk's MFMAs issue
  if (kend > kbeg) {
    const double *Ab = TA ? A + (size_t)m0 * lda + kbeg : A + (size_t)kbeg * lda + m0;
    const double *Bb = TB ? B + (size_t)kbeg * ldb + n0 : B + (size_t)n0 * ldb + kbeg;
    wave_mma32<TA != 0, TB != 0>(gptr(Ab), lda, gptr(Bb), ldb, kend - kbeg, M - m0, N - n0, acc);
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
            gptr(partial)[(size_t)kz * M * N + (size_t)col * M + row] = v;
          } else {
            double out = alpha * v;
            if (beta != 0.0) out += beta * gptr(C)[(size_t)col * ldc + row];
            gptr(C)[(size_t)col * ldc + row] = out;
          }
        }
      }
}

// The same product with a 64 x 64 tile of C per workgroup (four waves, each a 32 x 32
// quarter) and the operands staged through LDS in chunks of 32 along K, double-buffered:
// every element of A and B comes from global memory once per workgroup, by loads in which
// consecutive lanes read consecutive addresses (along K for a transposed operand, along
// the rows otherwise), and the next chunk is in flight while the current one's MFMAs issue.
// Operand layouts in LDS: a transposed operand (A^T, or B as stored) by [row][k] with rows
// of 33 doubles, the others by [k][row] with rows of 65.
constexpr int kGT = 64;  // tile of C per workgroup
constexpr int kGK = 32;  // K chunk

// XCD-aware order (xcd_split > 0, a one-dimensional grid of tiles x splits workgroups):
// workgroup L runs on XCD L % 8 (the dispatcher deals workgroups to the eight XCDs in turn),
// and all workgroups of one K split go to the same XCD, so that the split's slices of A and
// B, shared by all its tiles, are read into that XCD's L2 once. Without splits (xcd_split
// < 0), the tiles of one 64-row block of C share an XCD (their common rows of A).
constexpr int kXcds = 8;

template <int TA, int TB, bool LOWER = false, bool PAIR = false>
__global__ void __launch_bounds__(256)
    gemm_lds_kernel(int M, int N, int K, const double *__restrict__ A, int lda,
                    const double *__restrict__ B, int ldb, double *__restrict__ C, int ldc,
                    double alpha, double beta, int kchunk, double *__restrict__ partial,
                    const int *__restrict__ run, int xcd_split, const double *__restrict__ B2,
                    double *__restrict__ C2, int N1) {
  if (run && run[0] == 0) return;
  int bx = blockIdx.x, by = blockIdx.y, kz = blockIdx.z;
  if (xcd_split != 0) {
    const int L = blockIdx.x, xcd = L % kXcds, slot = L / kXcds;
    const int tm = (M + kGT - 1) / kGT, tn = (N + kGT - 1) / kGT;
    if (xcd_split > 0) {  // LOWER: tiles numbered along the lower triangle
      const int tiles = LOWER ? tm * (tm + 1) / 2 : tm * tn;
      int t = slot % tiles;
      kz = (slot / tiles) * kXcds + xcd;
      if (LOWER) {
        bx = 0;
        while (t > bx) t -= ++bx;
        by = t;
      } else {
        bx = t % tm, by = t / tm;
      }
    } else {  // tm a multiple of 8
      bx = (slot / tn) * kXcds + xcd, by = slot % tn, kz = 0;
    }
  }
  const int m0 = bx * kGT, n0 = by * kGT;
  if (m0 >= M || n0 >= N) return;
  if (LOWER && by > bx) return;  // symmetric result: tiles above the diagonal
  // A tile: TA ? As[i][k] (ld 33) : As[k][i] (ld 65); B tile: TB ? Bs[k][j] (ld 65) : Bs[j][k] (ld 33)
  constexpr int kSz = kGT * (kGK + 1) > kGK * (kGT + 1) ? kGT * (kGK + 1) : kGK * (kGT + 1);
  __shared__ double As[2][kSz], Bs[2][kSz];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lg = lane >> 4;
  const int wr = wave >> 1, wc = wave & 1;  // this wave's 32 x 32 quarter
  const int kbeg = kz * kchunk, kend = min(K, kbeg + kchunk);
  d4 acc[2][2];
  zero_acc(acc);
  // eight elements of each operand per thread and chunk, two chunks in flight
  auto load = [&](double (&ra)[8], double (&rb)[8], int k0) {
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      // unconditional loads at a clamped address, the value selected (no branch per load)
      if (TA) {  // A[k + i lda]: lanes along k
        const int kk = tid & 31, i = (tid >> 5) + 8 * p;
        const bool in = m0 + i < M && k0 + kk < kend;
        const double v = A[in ? (size_t)(m0 + i) * lda + k0 + kk : 0];
        ra[p] = in ? v : 0.0;
      } else {  // A[i + k lda]: lanes along i
        const int i = tid & 63, kk = (tid >> 6) + 4 * p;
        const bool in = m0 + i < M && k0 + kk < kend;
        const double v = A[in ? (size_t)(k0 + kk) * lda + m0 + i : 0];
        ra[p] = in ? v : 0.0;
      }
      if (TB) {  // B[j + k ldb]: lanes along j
        const int j = tid & 63, kk = (tid >> 6) + 4 * p;
        const bool in = n0 + j < N && k0 + kk < kend;
        const double v = B[in ? (size_t)(k0 + kk) * ldb + n0 + j : 0];
        rb[p] = in ? v : 0.0;
      } else {  // B[k + j ldb]: lanes along k; columns from N1 on from B2 (pair form)
        const int kk = tid & 31, j = (tid >> 5) + 8 * p;
        const bool in = n0 + j < N && k0 + kk < kend;
        const bool second = PAIR && n0 + j >= N1;
        const double *bp = second ? B2 + (size_t)(n0 + j - N1) * ldb : B + (size_t)(n0 + j) * ldb;
        const double v = (in ? bp : B)[in ? k0 + kk : 0];
        rb[p] = in ? v : 0.0;
      }
    }
  };
  auto store = [&](const double (&ra)[8], const double (&rb)[8], int buf) {
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      if (TA) {
        const int kk = tid & 31, i = (tid >> 5) + 8 * p;
        As[buf][i * (kGK + 1) + kk] = ra[p];
      } else {
        const int i = tid & 63, kk = (tid >> 6) + 4 * p;
        As[buf][kk * (kGT + 1) + i] = ra[p];
      }
      if (TB) {
        const int j = tid & 63, kk = (tid >> 6) + 4 * p;
        Bs[buf][kk * (kGT + 1) + j] = rb[p];
      } else {
        const int kk = tid & 31, j = (tid >> 5) + 8 * p;
        Bs[buf][j * (kGK + 1) + kk] = rb[p];
      }
    }
  };
  auto compute = [&](int buf) {
    const double *as = As[buf], *bs = Bs[buf];
#pragma unroll
    for (int s = 0; s < kGK / 4; ++s) {
      const int kk = 4 * s + lg;
      double av[2], bv[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int i = 32 * wr + 16 * t + li, j = 32 * wc + 16 * t + li;
        av[t] = TA ? as[i * (kGK + 1) + kk] : as[kk * (kGT + 1) + i];
        bv[t] = TB ? bs[kk * (kGT + 1) + j] : bs[j * (kGK + 1) + kk];
      }
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
          acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[rt], bv[ct], acc[rt][ct], 0, 0, 0);
    }
  };
  const int nch = (kend - kbeg + kGK - 1) / kGK;
  if (nch > 0) {
    // chunk c is in LDS buffer c & 1; chunk c + 1 waits in registers; chunk c + 2 is loaded
    // while chunk c computes (the loop body is written out for even and odd c)
    double ra0[8], rb0[8], ra1[8], rb1[8];
    load(ra0, rb0, kbeg);
    if (nch > 1) load(ra1, rb1, kbeg + kGK);
    store(ra0, rb0, 0);
    __syncthreads();
    for (int c = 0; c < nch; c += 2) {
      if (c + 2 < nch) load(ra0, rb0, kbeg + (c + 2) * kGK);
      compute(0);
      if (c + 1 >= nch) break;
      store(ra1, rb1, 1);  // buffer 1's last readers passed the barrier below, one chunk ago
      __syncthreads();
      if (c + 3 < nch) load(ra1, rb1, kbeg + (c + 3) * kGK);
      compute(1);
      if (c + 2 >= nch) break;
      store(ra0, rb0, 0);
      __syncthreads();
    }
  }
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + 32 * wr + 16 * rt + lg + 4 * r;
        const int col = n0 + 32 * wc + 16 * ct + li;
        if (row < M && col < N) {
          const double v = acc[rt][ct][r];
          if (partial) {
            partial[(size_t)kz * M * N + (size_t)col * M + row] = v;
          } else {
            double *cp = (PAIR && col >= N1) ? C2 + (size_t)(col - N1) * ldc : C + (size_t)col * ldc;
            double out = alpha * v;
            if (beta != 0.0) out += beta * cp[row];
            cp[row] = out;
          }
        }
      }
}

// ints after the Gram's partial sums of squares used by the multi-workgroup Cholesky: one
// "panel published" flag per 32-column block, then the breakdown and modified words
constexpr int kCholMaxBlocks = 48;  // 1088 / 32 = 34 blocks at the largest sketch
constexpr int kCholSyncBad = kCholMaxBlocks, kCholSyncMod = kCholMaxBlocks + 1;
constexpr int kCholSyncInts = 64;

__global__ void __launch_bounds__(256)
    splitk_reduce_kernel(int M, int N, int splits, const double *__restrict__ partial,
                         double alpha, double beta, double *__restrict__ C, int ldc,
                         const int *__restrict__ run, int lower, double *__restrict__ gram_sq,
                         double *__restrict__ C2, int N1, int sym) {
  if (run && run[0] == 0) return;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t MN = (size_t)M * N;
  double sq = 0.0, dq = 0.0;
  if (idx < MN) {
    int row = (int)(idx % M), col = (int)(idx / M);
    if (C2 && col >= N1) C = C2, col -= N1;  // the pair form's second result
    if (sym) {
      // C <- (C + C^T) / 2 as it is formed (M == N): the thread of (row, col), row >= col,
      // sums both entries' splits in order and writes the mean to both
      if (row >= col) {
        const size_t mir = (size_t)row * M + col;
        double sa = 0.0, sb = 0.0;
        for (int z = 0; z < splits; ++z) {
          sa += partial[(size_t)z * MN + idx];
          sb += partial[(size_t)z * MN + mir];
        }
        const double a = alpha * sa, b = alpha * sb;
        const double v = (row == col) ? a : 0.5 * (a + b);
        C[(size_t)col * ldc + row] = v;
        C[(size_t)row * ldc + col] = v;
      }
    } else if (lower && row < col) {
      // not computed for a lower-triangle result; zeroed when the result is a Cholesky input
      if (gram_sq) C[(size_t)col * ldc + row] = 0.0;
    } else {
      // the splits summed in order, eight loads in flight at a time
      double s = 0.0;
      int z = 0;
      for (; z + 8 <= splits; z += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = partial[(size_t)(z + u) * MN + idx];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
      }
      for (; z < splits; ++z) s += partial[(size_t)z * MN + idx];
      double out = alpha * s;
      if (beta != 0.0) out += beta * C[(size_t)col * ldc + row];
      C[(size_t)col * ldc + row] = out;
      const double w = row > col ? 2.0 : 1.0;  // strict lower counts for both triangles
      const double dev = out - (row == col ? 1.0 : 0.0);
      sq = w * out * out;
      dq = w * dev * dev;
    }
  }
  if (gram_sq) {
    // this block's shares of ||C||_F^2 and ||C - I||_F^2, each summed in a fixed order
    __shared__ double red[2][4];
    for (int off = 32; off > 0; off >>= 1) {
      sq += __shfl_down(sq, off, 64);
      dq += __shfl_down(dq, off, 64);
    }
    if ((threadIdx.x & 63) == 0) red[0][threadIdx.x >> 6] = sq, red[1][threadIdx.x >> 6] = dq;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0, d = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[0][w], d += red[1][w];
      gram_sq[blockIdx.x] = t;
      gram_sq[gridDim.x + kCholSyncInts / 2 + blockIdx.x] = d;
    }
    // the flags the in-place Cholesky's workgroups exchange follow the partial sums; they
    // start each factorization cleared
    if (blockIdx.x == 0 && threadIdx.x < kCholSyncInts)
      reinterpret_cast<int *>(gram_sq + gridDim.x)[threadIdx.x] = 0;
  }
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


constexpr int kCholThreads = 512;
// A Gram matrix G = X^T X with ||G - I||_F^2 at most the unit roundoff is factored to first
// order: L = I + F, F = strict lower part of G - I plus half its diagonal, so that
// L L^T = G - F F^T, off by at most ||G - I||_F^2 <= u in the 2-norm (X L^{-T} is then
// orthonormal to rounding, as from the exact factor).
constexpr double kCholFirstOrderDev2 = 0x1.0p-53;

// End of a CholeskyQR pass (one thread): count it, update the clean-pass count and set the
// next pass's run flag.
__device__ __noinline__ void cholqr_notify(const CholQrCtl &c, int next) {
  if (c.host)
    __hip_atomic_store(c.host, (int)((unsigned)c.seq << 1) | next, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_SYSTEM);
}

// A pass that does not run (one thread): the next one does not either.
__device__ void cholqr_ctl_skip(const CholQrCtl &c) {
  if (c.pass + 1 < c.npass) c.cq[c.pass + 1] = 0;
  cholqr_notify(c, 0);
}

__device__ __noinline__ void cholqr_ctl_end(const CholQrCtl &c, bool shifted, bool modified, bool bad) {
  if (c.count) c.count[0] += 1;
  const int prev = (c.pass == 0) ? 0 : c.cq[c.npass];  // pass 0 starts the count
  const int clean = (!shifted && !modified && !bad) ? prev + 1 : 0;
  c.cq[c.npass] = clean;
  const int next = (c.pass + 1 < c.npass && clean < 2 && !bad) ? 1 : 0;
  if (c.pass + 1 < c.npass) c.cq[c.pass + 1] = next;
  cholqr_notify(c, next);
}

// Inverse of diagonal block b of the first-order factor L = I + F of G (F: strict lower
// part of G - I and half its diagonal): I - F_bb, off by at most ||F_bb||^2 <= u, in the
// layout of trsm_diag_inv_kernel (entry (t, c) at dinv[1024 b + 32 c + t], zero outside
// the block's nb x nb part), from G itself (before its diagonal becomes the factor's).
// Threads tid0, tid0 + nthr, ... of the caller.
__device__ void first_order_dinv(int m, int b, const double *G, double *dinv, int tid0, int nthr) {
  const int c0 = 32 * b, nb = min(32, m - c0);
  for (int idx = tid0; idx < 1024; idx += nthr) {
    const int c = idx >> 5, t = idx & 31;
    double v = 0.0;
    if (c < nb && t < nb) {
      const double g = G[(size_t)(c0 + c) * m + c0 + t];
      v = (t == c) ? 1.5 - 0.5 * g : (t > c ? -g : 0.0);  // 1 - (g - 1) / 2 on the diagonal
    }
    dinv[(size_t)b * 1024 + idx] = v;
  }
}

// The same for every block of an m <= kFoBlocks * 32 factor, by kCholThreads threads, every
// load issued before the first wait (kept out of line: the blocked Cholesky's main path
// keeps its register allocation).
constexpr int kFoBlocks = 9;
__device__ __noinline__ void first_order_dinv_all(int m, const double *G, double *dinv) {
  constexpr int kFoPer = kFoBlocks * 1024 / kCholThreads;
  const gmem<double> *Gg = gptr(G);
  const int tid = threadIdx.x;
  double gv[kFoPer];
#pragma unroll
  for (int t = 0; t < kFoPer; ++t) {
    const int e = tid + kCholThreads * t, b = e >> 10, c = (e >> 5) & 31, r = e & 31;
    const int c0 = 32 * b, nb = min(32, m - c0);
    const bool in = c0 < m && c < nb && r < nb;
    gv[t] = Gg[in ? (size_t)(c0 + c) * m + c0 + r : 0];
  }
#pragma unroll
  for (int t = 0; t < kFoPer; ++t) {
    const int e = tid + kCholThreads * t, b = e >> 10, c = (e >> 5) & 31, r = e & 31;
    const int c0 = 32 * b, nb = min(32, m - c0);
    if (c0 >= m) continue;
    const double g = gv[t];
    const double v =
        (c < nb && r < nb) ? ((r == c) ? 1.5 - 0.5 * g : (r > c ? -g : 0.0)) : 0.0;
    gptr(dinv)[e] = v;
  }
}

// Sum of the partial sums of ||G - I||_F^2 that the Gram's split-K reduction left after
// those of ||G||_F^2 and the 32 doubles of flags, in a fixed order (every caller in the
// grid gets the same value).
__device__ double gram_dev2(int m, const double *gram_sq, double *red) {
  const int nsq = (int)(((size_t)m * m + 255) / 256);
  const double *dev = gram_sq + nsq + kCholSyncInts / 2;
  double part = 0.0;
  for (int q = threadIdx.x; q < nsq; q += blockDim.x) part += dev[q];
  return wg_sum(part, red);
}
constexpr int kPB = 32;  // panel width of the blocked factorizations
constexpr int kStageRows = 256;  // panel rows staged in LDS by the Cholesky (two buffers)
// largest 1-norm condition of a 32 x 32 diagonal block whose panel the Cholesky solves as a
// product with the block's inverse (about one digit of the panel's residual given up)
constexpr double kCholInvCond = 16.0;

// Value of a double held by lane `src` of the wave (src uniform), via two v_readlane_b32.
__device__ __forceinline__ double readlane_d(double v, int src) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Maximum over the wave of a non-negative double, without LDS: DPP exchanges within each row
// of 16 lanes (xor 1, xor 2, mirror within 8, mirror within 16; lanes a pattern leaves without
// a source read 0, which cannot raise the maximum), then the four rows' values by v_readlane.
template <int CTRL>
__device__ __forceinline__ double dpp_nonneg(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_max_nonneg(double v) {
  v = fmax(v, dpp_nonneg<0xB1>(v));   // quad_perm [1, 0, 3, 2]
  v = fmax(v, dpp_nonneg<0x4E>(v));   // quad_perm [2, 3, 0, 1]
  v = fmax(v, dpp_nonneg<0x141>(v));  // row_half_mirror
  v = fmax(v, dpp_nonneg<0x140>(v));  // row_mirror
  return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}

// LDS of the diagonal-block factorization (one wave).
struct BlockLds {
  double D[kPB][kPB + 1];   // in: the block's lower triangle; out: L11 (upper part zero)
  double Di[kPB][kPB + 1];  // out: Di[c][t] = (L11^{-1})[t][c], zero outside nb x nb
  __align__(16) double colk[2][16];  // column k of L11 by row parity: colk[i & 1][i >> 1]
  __align__(16) double yrow[2][16];  // row k of the unscaled inverse by column parity
  double rdiag[kPB];                 // out without the inverse: about 1 / L11[i][i] (rsqrt)
};

// Cholesky of the SPD block held in S.D (rows and columns >= nb are ignored) and the inverse
// of its factor, by one wave, straight-line code without branches. fpiv > 0: a pivot not
// above fpiv is replaced by it (modified Cholesky). Returns through the references: fail
// (non-finite or non-positive pivot), modified (a pivot was replaced), use_inv (1-norm
// condition |L11|_1 |L11^{-1}|_1 <= kCholInvCond). Uniform across the wave.
//
// Lane (i, h) = (lane & 31, lane >> 5) keeps the block's row i at the columns j = 2 jj + h
// (jj < 16) in r[jj]: interleaving the columns over the two halves keeps both busy while
// the active part shrinks, and with the pivot index known at compile time the finished
// columns take no instructions. Rows and columns from nb on hold the identity, which
// factors to itself without touching the rest, so every pivot runs the same code. Pivot k:
// its value comes from the owning lane's register (v_readlane), the owning half publishes
// column k scaled (L11[i][k], i > k) and every lane reads back its row's entry and the
// entries of its columns (broadcast LDS reads), then updates its live columns.
// The inverse is built alongside as Y with X = L11^{-1} = diag(1 / L11[k][k]) Y: pivot k
// takes (L11[i][k] / L11[k][k]) Y[k, :] from every row i > k, where Y[k, :] is final and
// nonzero only in columns <= k; rows are scaled once at the end.
// INV = false: no inverse (Di, use_inv untouched); S.rdiag[i] receives the pivot's reciprocal
// square root, within about an ulp of 1 / L11[i][i], for a forward substitution.
// A separate function (not inlined into the Cholesky kernel, whose other live values would
// push it into spills) taking the LDS block by an address-space-3 reference, so that the
// accesses stay plain ds_read/ds_write with immediate offsets.
using LdsBlock = __attribute__((address_space(3))) BlockLds;
using lds_double = __attribute__((address_space(3))) double;
template <bool INV>
__device__ __attribute__((noinline)) void factor_block32(LdsBlock &S, int nb, double fpiv,
                                                         bool &fail_out, bool &mod_out,
                                                         bool &use_inv_out) {
  const int lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
  double r[16], y[16];
#pragma unroll
  for (int jj = 0; jj < 16; ++jj) {
    const int j = 2 * jj + h;
    const bool real = i < nb && j < nb;
    r[jj] = real ? (j <= i ? S.D[i][j] : 0.0) : (i == j ? 1.0 : 0.0);
    if constexpr (INV) y[jj] = (i == j) ? 1.0 : 0.0;
  }
  bool fail = false, modified = false;
  double myrinv = 1.0;  // 1 / L11[i][i]
  lds_double *const mycol = &S.colk[i & 1][i >> 1];
  // this half's entries of the published column and row, read as pairs (ds_read_b128)
  const lds_double *const colh = &S.colk[h][0];  // this half's entries, read in pairs
  const lds_double *const yrh = &S.yrow[h][0];
#pragma unroll
  for (int k = 0; k < kPB; ++k) {
    const int kh = k & 1, kk = k >> 1;  // column k is r[kk] of half kh
    const bool realk = k < nb;
    double piv = readlane_d(r[kk], k + 32 * kh);
    fail |= realk && !isfinite(piv);
    const bool repl = realk && fpiv > 0.0 && !(piv > fpiv);
    modified |= repl;
    piv = repl ? fpiv : piv;
    fail |= !(piv > 0.0);
    const double rinv = rsqrt(piv);
    myrinv = (i == k) ? rinv : myrinv;
    // the owning half publishes column k below the diagonal (zero at and above it) and
    // writes L11[i][k], i >= k, to D (rows from nb on are zero or the identity's and are
    // never read back)
    const double lown = r[kk] * rinv;
    if (h == kh) {
      *mycol = (i > k) ? lown : 0.0;
      if (i >= k) S.D[i][k] = (i == k) ? piv * rinv : lown;
    }
    // lanes (k, 0) and (k, 1) publish row k of Y (columns <= k; the pairs' second entry
    // beyond k is zero)
    if (INV && i == k) {
      lds_double *const ydst = &S.yrow[h][0];
#pragma unroll
      for (int q = 0; q <= kk / 2; ++q) {
        ydst[2 * q] = y[2 * q];
        ydst[2 * q + 1] = y[2 * q + 1];
      }
    }
    // a wave's LDS operations complete in order: the reads below see these writes
    __builtin_amdgcn_wave_barrier();
    const double lik = *mycol;  // L11[i][k] for i > k, else 0
    const int jlo = k >> 1;     // columns 2 jj + h > k have jj >= jlo
    double lj[16], yk[16];
#pragma unroll
    for (int q = jlo / 2; q < 8; ++q) {
      lj[2 * q] = colh[2 * q];
      lj[2 * q + 1] = colh[2 * q + 1];
    }
    if constexpr (INV) {
#pragma unroll
      for (int q = 0; q <= kk / 2; ++q) {
        yk[2 * q] = yrh[2 * q];
        yk[2 * q + 1] = yrh[2 * q + 1];
      }
    }
#pragma unroll
    for (int jj = jlo; jj < 16; ++jj) r[jj] = fma(-lik, lj[jj], r[jj]);
    if constexpr (INV) {
      const double t = lik * rinv;  // L11[i][k] / L11[k][k], zero for i <= k
#pragma unroll
      for (int jj = 0; jj <= kk; ++jj) y[jj] = fma(-t, yk[jj], y[jj]);
    }
    // the updates happen here: without this the compiler defers the FMAs of columns needed
    // only at later pivots and keeps all their operands live (register spills)
#pragma unroll
    for (int jj = jlo; jj < 16; ++jj) asm volatile("" : "+v"(r[jj]));
    if constexpr (INV) {
#pragma unroll
      for (int jj = 0; jj <= kk; ++jj) asm volatile("" : "+v"(y[jj]));
    }
  }
  if constexpr (!INV) {
    if (h == 0) S.rdiag[i] = (i < nb) ? myrinv : 0.0;
    fail_out = fail;
    mod_out = modified;
    use_inv_out = false;
    return;
  }
  // X = diag(1 / L11[i][i]) Y into Di (transposed), zero outside the nb x nb block
#pragma unroll
  for (int jj = 0; jj < 16; ++jj) {
    const int c = 2 * jj + h;
    S.Di[c][i] = (i < nb && c < nb) ? y[jj] * myrinv : 0.0;
  }
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_wave_barrier();
  // kappa = |L11|_1 |L11^{-1}|_1: lane c sums column c of the factor (D[t][c]) and of its
  // inverse (Di[c][t]); the loads are issued together
  double cl = 0.0, ci = 0.0;
  {
    const int c = i;
#pragma unroll
    for (int t = 0; t < kPB; ++t) {
      const double dv = S.D[t][c];
      const double xv = S.Di[c][t];
      const bool in = t >= c && t < nb && c < nb;
      cl += in ? fabs(dv) : 0.0;
      ci += in ? fabs(xv) : 0.0;
    }
  }
  cl = wave_max_nonneg(cl);
  ci = wave_max_nonneg(ci);
  // fail and modified are uniform: every lane took the same pivots
  fail_out = fail;
  mod_out = modified;
  use_inv_out = !fail && (cl * ci <= kCholInvCond);
}

// Inverse of the factored diagonal block D (LDS, rows of kPB + 1, nb x nb used) by column-oriented forward
// substitution, L11 x_c = e_c with one column per lane (lanes 0..31 of the calling wave;
// the others return), into out[32 c + t] = (L11^{-1})[t][c], zero outside the nb x nb part.
// Solving for the columns keeps the right residual L11 X - I at rounding level relative to
// |L11| |X|, which the right-hand solves X <- X L^{-T} that use it need (the inverse that
// factor_block32 builds alongside the pivots is row-oriented: its left residual is small,
// its right one up to the block's condition times larger). Each x_i takes its row's sum in
// two accumulators and the reciprocal of L11[i][i] (one correctly rounded division per lane,
// shared by v_readlane), so the 32 rows run without branches.
__device__ __attribute__((noinline)) void block_inverse_fs(const lds_double *D, int nb,
                                                           double *__restrict__ out) {
  const int c = threadIdx.x & 63;
  if (c >= 32) return;
  const double rd = (c < nb) ? 1.0 / D[c * (kPB + 1) + c] : 0.0;  // 1 / L11[c][c]
  double x[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    double a0 = (i == c) ? 1.0 : 0.0, a1 = 0.0;
#pragma unroll
    for (int t = 0; t < i; t += 2) {  // x[t] = 0 for t < c
      a0 = fma(-D[i * (kPB + 1) + t], x[t], a0);
      if (t + 1 < i) a1 = fma(-D[i * (kPB + 1) + t + 1], x[t + 1], a1);
    }
    const double v = (a0 + a1) * readlane_d(rd, i);
    x[i] = (i >= c && i < nb) ? v : 0.0;
  }
#pragma unroll
  for (int i = 0; i < 32; ++i) out[(size_t)c * 32 + i] = x[i];
}

// ---------------------------------------------------------------------------
// Blocked Cholesky G + s I = L L^T (lower, column-major), one workgroup.
// mode 0: s = 0; mode 1: s = shift_rel ||G||_F; mode 2: s = 0, and a pivot that is not
// above shift_rel ||G||_F is replaced by that value (modified Cholesky). Per 32-column
// panel: wave 0 factors the diagonal block in registers, inverts the factor and takes the
// block's condition; the panel below is X = A21 L11^{-T}, on the FP64 matrix cores with
// the inverse when the block is well conditioned, else by forward substitution; the
// trailing lower triangle is updated with FP64 MFMA (32 x 32 tiles), wave 0 taking the
// next diagonal tile and factoring it while the other waves update the rest.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kCholThreads)
    chol_blocked_kernel(int m, const double *G, double *L,
                        double shift_rel, int mode, int *__restrict__ flag,
                        int *__restrict__ shifts, const int *__restrict__ run,
                        int *__restrict__ modflag, const double *__restrict__ gram_sq,
                        double *__restrict__ dinv, CholQrCtl ctl,
                        const CholJob *__restrict__ jobs) {
  if (jobs) {  // batched: blockIdx.y selects the problem
    const CholJob &J = jobs[blockIdx.y];
    m = J.m, G = J.G, L = J.L, shift_rel = J.shift_rel, flag = J.flag, shifts = J.shifts;
    run = J.run, modflag = J.modflag;
    gram_sq = nullptr, dinv = nullptr, ctl = CholQrCtl();
  }
  // pass 0 of a CholeskyQR always runs; pass p > 0 runs when pass p - 1 set its flag
  if (ctl.cq) run = ctl.pass == 0 ? nullptr : ctl.cq + ctl.pass;
  if (run && run[0] == 0) {
    if (threadIdx.x == 0 && ctl.cq) cholqr_ctl_skip(ctl);
    return;
  }
  gmem<double> *const Lg = gptr(L);  // the factor's global accesses (see gptr)
  __shared__ BlockLds S;  // the diagonal block, its factor and inverse
  // the staged panel and the next one, which the trailing update writes (ping-pong)
  __shared__ double Pbuf[2][kPB * (kStageRows + 1)];
  __shared__ double Dc[kPB][kPB + 1];  // this block's factor, kept for its inverse
  __shared__ double red[16];
  __shared__ int bad, use_inv;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int wave = tid >> 6, nwaves = nt >> 6;
  // gram_sq given: the Gram GEMM wrote G into L (zero upper triangle) and the partial sums
  // of ||G||_F^2; the factorization runs in place
  const bool inplace = gram_sq != nullptr;
  if (inplace && mode == 2 && gram_dev2(m, gram_sq, red) <= kCholFirstOrderDev2) {
    // G within sqrt(u) of the identity: the first-order factor, in place (the diagonal is
    // the only change: L[i][i] = 1 + (G[i][i] - 1) / 2), and its blocks' inverses (as
    // first_order_dinv, with every load of the at most nine blocks issued before the first
    // wait)
    if (dinv && nt == kCholThreads && m <= kFoBlocks * kPB)
      first_order_dinv_all(m, L, dinv);
    else if (dinv)
      for (int b = 0; b * kPB < m; ++b) first_order_dinv(m, b, L, dinv, tid, nt);
    __syncthreads();
    for (int i = tid; i < m; i += nt) Lg[(size_t)i * m + i] = 0.5 + 0.5 * Lg[(size_t)i * m + i];
    if (tid == 0 && ctl.cq) cholqr_ctl_end(ctl, false, false, false);
    return;
  }
  double fro = 0.0;
  if (mode != 0) {
    double part = 0.0;
    if (inplace) {
      const int nsq = (int)(((size_t)m * m + 255) / 256);
      for (int q = tid; q < nsq; q += nt) part += gram_sq[q];
    } else {
      // from the lower triangle (the upper one need not be formed): diagonal + 2 x strict lower
      for (size_t idx = tid; idx < (size_t)m * m; idx += nt) {
        const int i = (int)(idx % m), j = (int)(idx / m);
        const double w = (i > j) ? 2.0 : ((i == j) ? 1.0 : 0.0);
        part += w * G[idx] * G[idx];
      }
    }
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
    if (inplace) {
      if (s != 0.0)
        for (int i = tid; i < m; i += nt) Lg[(size_t)i * m + i] += s;
    } else {
      // (i, j) of idx advanced by nt each iteration without a division per element
      const int step_i = nt % m, step_j = nt / m;
      int i = tid % m, j = tid / m;
#pragma unroll 4
      for (size_t idx = tid; idx < (size_t)m * m; idx += nt) {
        Lg[idx] = (i >= j) ? (G[idx] + (i == j ? s : 0.0)) : 0.0;
        i += step_i;
        j += step_j;
        if (i >= m) i -= m, ++j;
      }
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    // Factor the diagonal block held in S.D by wave 0 alone (factor_block32); no workgroup
    // barrier inside.
    // inv: the block's inverse for a panel too tall to stage (a staged panel is solved by
    // forward substitution, which needs only the pivots' reciprocals)
    auto factor_block = [&](int nb, bool inv) __attribute__((always_inline)) {
      bool f, md, ui;
      if (inv)
        factor_block32<true>(*(LdsBlock *)&S, nb, floor_piv, f, md, ui);
      else
        factor_block32<false>(*(LdsBlock *)&S, nb, floor_piv, f, md, ui);
      if ((tid & 63) == 0) {
        if (f) bad = 1;
        if (md) modified = 1;
        use_inv = ui;
      }
    };
    // first diagonal block
    {
      const int nb = min(kPB, m);
      for (int idx = tid; idx < nb * nb; idx += nt) {
        const int i = idx % nb, j = idx / nb;
        S.D[i][j] = (i >= j) ? Lg[(size_t)j * m + i] : 0.0;
      }
      __syncthreads();
      if (wave == 0) factor_block(nb, m - nb > kStageRows);
      __syncthreads();
    }
    int cur = 0;        // Pbuf[cur] holds this block's panel
    bool have = false;  // the previous trailing update left it there
    for (int kb = 0; kb < m && !bad; kb += kPB) {
      const int nb = min(kPB, m - kb);
      double *const Pn = Pbuf[cur];
      // 1. the diagonal block, factored (before the loop, or during the previous panel's
      //    trailing update), goes to L, and to Dc for its inverse (step 3)
      for (int idx = tid; idx < nb * nb; idx += nt) {
        const int i = idx % nb, j = idx / nb;
        if (i >= j) Lg[(size_t)(kb + j) * m + kb + i] = S.D[i][j];
      }
      if (dinv)
        for (int idx = tid; idx < kPB * kPB; idx += nt) Dc[idx >> 5][idx & 31] = S.D[idx >> 5][idx & 31];

      // 2. panel rows below: X L11^T = A21. A staged panel (in LDS) is solved by forward
      //    substitution along each row, one row per thread; the result goes to L and to the
      //    staged copy. A panel too tall to stage: X = A21 L11^{-T} on MFMA, one 32-row tile
      //    per wave, when the block is well conditioned (the product with the inverse leaves a
      //    residual of order kappa times rounding), else forward substitution per row in L.
      const int r0 = kb + nb;
      const int prow = m - r0;
      const bool staged = prow <= kStageRows;
      if (staged && !have) {
        // eight loads in flight per thread before any is stored (one memory latency per
        // round, not one per element)
        const int tot = nb * prow;
        for (int base = tid; base < tot; base += 8 * nt) {
          double v[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int e = base + u * nt;
            const int ec = e < tot ? e : 0;
            const int jj = ec / prow, ii = ec - jj * prow;
            v[u] = Lg[(size_t)(kb + jj) * m + r0 + ii];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int e = base + u * nt;
            if (e < tot) {
              const int jj = e / prow, ii = e - jj * prow;
              Pn[jj * (kStageRows + 1) + ii] = v[u];
            }
          }
        }
      }
      __syncthreads();
      if (staged) {
        // X L11^T = A by forward substitution along each row, one row per thread, from the
        // staged panel: backward stable for any condition of L11 (no refinement needed).
        // A panel below exists only under a full block (nb = 32).
        if (tid < prow) {
          const int ii = tid, ld = kStageRows + 1;
          double x[kPB];
#pragma unroll
          for (int j = 0; j < kPB; ++j) {
            double a0 = Pn[j * ld + ii], a1 = 0.0;
#pragma unroll
            for (int t = 0; t < j; t += 2) {
              a0 = fma(-x[t], S.D[j][t], a0);
              if (t + 1 < j) a1 = fma(-x[t + 1], S.D[j][t + 1], a1);
            }
            x[j] = (a0 + a1) * S.rdiag[j];
          }
#pragma unroll
          for (int j = 0; j < kPB; ++j) {
            Pn[j * ld + ii] = x[j];
            Lg[(size_t)(kb + j) * m + r0 + ii] = x[j];
          }
        }
      } else if (!use_inv) {
        // in place in the panel's own storage (global), row by row:
        // x_j = (a_j - sum_{t<j} x_t L11[j][t]) / L11[j][j]
        for (int i = tid; i < prow; i += nt) {
          double *col = L + (size_t)kb * m + r0 + i;  // element j at col[j m]
          for (int j = 0; j < nb; ++j) {
            double a = col[(size_t)j * m];
            for (int t = 0; t < j; ++t) a -= col[(size_t)t * m] * S.D[j][t];
            col[(size_t)j * m] = a * S.Di[j][j];  // Di[j][j] = 1 / L11[j][j]
          }
        }
      } else {
        const int lane = tid & 63, li = lane & 15, lg = lane >> 4;
        const int npt = (prow + 31) / 32;
        for (int I = wave; I < npt; I += nwaves) {
          const int i0 = 32 * I;
          d4 acc[2][2];
          zero_acc(acc);
          wave_mma32<false, true>(Lg + (size_t)kb * m + r0 + i0, m, &S.Di[0][0], kPB + 1, nb,
                                  prow - i0, nb, acc);
          // the MFMAs consumed every operand load of this wave's rows: overwrite them
#pragma unroll
          for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
#pragma unroll
              for (int rr = 0; rr < 4; ++rr) {
                const int row = i0 + 16 * rt + lg + 4 * rr, col = 16 * ct + li;
                if (row < prow && col < nb) Lg[(size_t)(kb + col) * m + r0 + row] = acc[rt][ct][rr];
              }
        }
      }
      __syncthreads();
      // 3. trailing update A22 -= L21 L21^T on the lower 32 x 32 tiles (MFMA operands
      //    from the staged panel when it fits), with look-ahead: wave 0 updates the next
      //    diagonal tile (tile 0) into L and D and factors it while the other waves update
      //    the remaining tiles, so the next panel starts with its diagonal block factored.
      const int nt32 = (prow + 31) / 32;
      const int ntiles = nt32 * (nt32 + 1) / 2;
      auto trailing_tile = [&](int t, bool to_D) {
        int I = 0, rem = t;
        while (rem > I) {
          rem -= I + 1;
          ++I;
        }
        const int J = rem;  // tile (I, J) with J <= I
        const int i0 = r0 + 32 * I, j0 = r0 + 32 * J;
        const int lane = tid & 63, li = lane & 15, lg = lane >> 4;
        // the tile's current values are loaded before the products (unconditional loads at a
        // clamped address, so they are all in flight together and overlap the MFMAs)
        double old[2][2][4];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
          for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = i0 + 16 * rt + lg + 4 * r, col = j0 + 16 * ct + li;
              const bool in = row < m && col < m && row >= col;
              old[rt][ct][r] = Lg[in ? (size_t)col * m + row : 0];
            }
        d4 acc[2][2];
        zero_acc(acc);
        if (staged)
          wave_mma32<false, true>(Pn + 32 * I, kStageRows + 1, Pn + 32 * J, kStageRows + 1, nb,
                                  m - i0, m - j0, acc);
        else
          wave_mma32<false, true>(Lg + (size_t)kb * m + i0, m, Lg + (size_t)kb * m + j0, m, nb,
                                  m - i0, m - j0, acc);
        // tiles below the next diagonal block in its column are the next panel: with a
        // staged panel they go to the other LDS buffer only (the panel's solve writes L)
        const bool to_next = staged && J == 0 && I > 0;
        double *const Pnext = Pbuf[cur ^ 1];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
          for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = i0 + 16 * rt + lg + 4 * r, col = j0 + 16 * ct + li;
              if (row < m && col < m && row >= col) {
                const double v = old[rt][ct][r] - acc[rt][ct][r];
                if (to_next)
                  Pnext[(col - r0) * (kStageRows + 1) + (row - r0 - kPB)] = v;
                else
                  Lg[(size_t)col * m + row] = v;
                if (to_D) S.D[row - i0][col - j0] = v;
              }
            }
      };
      if (wave == 0) {
        if (ntiles > 0) {
          // the critical path: wave 0's instructions go first when it shares its SIMD with a
          // wave of the trailing update
          __builtin_amdgcn_s_setprio(3);
          trailing_tile(0, true);
          asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
          __builtin_amdgcn_wave_barrier();
          factor_block(min(kPB, prow), prow - min(kPB, prow) > kStageRows);
          __builtin_amdgcn_s_setprio(0);
        }
      } else {
        // the block's inverse for the right-hand solves that follow the factorization, by
        // the last wave, which has the fewest tiles
        if (dinv && wave == nwaves - 1)
          block_inverse_fs((const lds_double *)&Dc[0][0], nb, dinv + (size_t)(kb / kPB) * 1024);
        for (int t = wave; t < ntiles; t += nwaves - 1) trailing_tile(t, false);
      }
      __syncthreads();
      have = staged;
      cur ^= 1;
    }
    __syncthreads();
    if (!bad) {
      if (tid == 0 && modified && shifts) shifts[0] += 1;
      if (tid == 0 && modified && modflag) modflag[0] = 1;
      if (tid == 0 && ctl.cq) cholqr_ctl_end(ctl, mode == 1, modified != 0, false);
      return;
    }
    __syncthreads();
  }
  if (tid == 0) flag[0] = 1;
  if (tid == 0 && ctl.cq) cholqr_ctl_end(ctl, mode == 1, modified != 0, true);
}

// ---------------------------------------------------------------------------
// Blocked Cholesky G + s I = L L^T in place, one workgroup per 32-column block J (the
// same modes and flags as chol_blocked_kernel). G == L is the Gram matrix as the Gram GEMM
// left it (zero upper triangle) with the partial sums of ||G||_F^2 in gram_sq and cleared
// flags after them. Right-looking: workgroup J applies the update of every panel p < J to
// its own column block as soon as panel p is published (tiles (I, J), I >= J, on FP64
// MFMA, operands from L2), then factors its diagonal block (factor_block32) and solves its
// panel X = A21 L11^{-T} (with one refinement step for a badly conditioned block), and
// publishes it: stores, agent-scope release fence, flag. Waiting is acquire on the flag,
// by one thread, with a bounded number of polls (a timeout counts as a breakdown). Only
// lower-numbered workgroups are waited for, and they are dispatched first.
// ---------------------------------------------------------------------------
constexpr int kCholMaxPolls = 1 << 22;

__global__ void __launch_bounds__(kCholThreads)
    chol_mwg_kernel(int m, double *L, double shift_rel, int mode, int *__restrict__ flag,
                    int *__restrict__ shifts, const int *__restrict__ run,
                    int *__restrict__ modflag, double *__restrict__ gram_sq,
                    double *__restrict__ dinv, CholQrCtl ctl) {
  if (ctl.cq) run = ctl.pass == 0 ? nullptr : ctl.cq + ctl.pass;
  if (run && run[0] == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0 && ctl.cq) cholqr_ctl_skip(ctl);
    return;
  }
  const int nblk = (m + kPB - 1) / kPB;
  const int J = blockIdx.x;
  if (J >= nblk) return;
  const int nsq = (int)(((size_t)m * m + 255) / 256);
  int *const sync = reinterpret_cast<int *>(gram_sq + nsq);
  __shared__ BlockLds S;
  __shared__ double W[kCholThreads / 64][kPB * (kPB + 1)];  // per-wave refinement tile
  __shared__ double red[16];
  __shared__ int bad, modified, use_inv, timed_out;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int wave = tid >> 6, nwaves = nthr >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  if (mode == 2 && gram_dev2(m, gram_sq, red) <= kCholFirstOrderDev2) {
    // first-order factor (every workgroup takes the same decision): this block's diagonal
    // and its inverse
    if (dinv) first_order_dinv(m, J, L, dinv, tid, nthr);
    __syncthreads();
    for (int t = kPB * J + tid; t < min(m, kPB * (J + 1)); t += nthr)
      L[(size_t)t * m + t] = 0.5 + 0.5 * L[(size_t)t * m + t];
    if (J == 0 && tid == 0 && ctl.cq) cholqr_ctl_end(ctl, false, false, false);
    return;
  }
  // ||G||_F from the partial sums, in the same order in every workgroup
  double fro = 0.0;
  if (mode != 0) {
    double part = 0.0;
    for (int q = tid; q < nsq; q += nthr) part += gram_sq[q];
    fro = sqrt(wg_sum(part, red));
  }
  const double floor_piv = (mode == 2) ? shift_rel * fro : 0.0;
  const double s = (mode == 1) ? shift_rel * fro : 0.0;
  if (mode == 1 && J == 0 && tid == 0 && shifts) shifts[0] += 1;
  const int c0 = kPB * J, nb = min(kPB, m - c0);
  if (tid == 0) bad = 0, modified = 0, use_inv = 1, timed_out = 0;
  // the diagonal block's upper triangle (and rows from nb on) stay zero: S.D is an MFMA
  // operand of the refinement
  for (int idx = tid; idx < kPB * (kPB + 1); idx += nthr) (&S.D[0][0])[idx] = 0.0;
  if (s != 0.0)
    for (int t = tid; t < nb; t += nthr) L[(size_t)(c0 + t) * m + c0 + t] += s;
  __syncthreads();

  auto factor_diag = [&]() {
    bool f, md, ui;
    factor_block32<true>(*(LdsBlock *)&S, nb, floor_piv, f, md, ui);
    if (lane == 0) {
      if (f) bad = 1;
      if (md) modified = 1;
      use_inv = ui;
    }
  };
  // tile (I, J) -= L[I, p] L[J, p]^T with the old values loaded ahead of the MFMAs; the
  // diagonal tile keeps its lower triangle only, and with to_D also goes to S.D
  auto update_tile = [&](int p, int I, bool to_D) {
    const int i0 = kPB * I, k0 = kPB * p;
    double old[2][2][4];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = i0 + 16 * rt + lg + 4 * r, col = c0 + 16 * ct + li;
          const bool in = row < m && col < m && row >= col;
          old[rt][ct][r] = L[in ? (size_t)col * m + row : 0];
        }
    d4 acc[2][2];
    zero_acc(acc);
    wave_mma32<false, true>(L + (size_t)k0 * m + i0, m, L + (size_t)k0 * m + c0, m,
                            min(kPB, m - k0), m - i0, m - c0, acc);
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = i0 + 16 * rt + lg + 4 * r, col = c0 + 16 * ct + li;
          if (row < m && col < m && row >= col) {
            const double v = old[rt][ct][r] - acc[rt][ct][r];
            L[(size_t)col * m + row] = v;
            if (to_D) S.D[row - i0][col - c0] = v;
          }
        }
  };

  // updates from the published panels p < J
  for (int p = 0; p < J; ++p) {
    if (tid == 0) {
      int polls = 0;
      while (__hip_atomic_load(&sync[p], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != 1) {
        if (++polls > kCholMaxPolls) {
          timed_out = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __syncthreads();
    // every thread sees panel p's stores (its own L1 may hold older lines)
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (timed_out) break;
    const int ntile = nblk - J;  // tiles I = J .. nblk - 1
    if (p == J - 1) {
      // last update: wave 0 takes the diagonal tile and factors it while the other waves
      // update the tiles below
      if (wave == 0) {
        __builtin_amdgcn_s_setprio(3);  // the critical path goes first on its SIMD
        update_tile(p, J, true);
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        __builtin_amdgcn_wave_barrier();
        factor_diag();
        __builtin_amdgcn_s_setprio(0);
      } else {
        for (int t = wave; t < ntile; t += nwaves - 1) update_tile(p, J + t, false);
      }
    } else {
      for (int t = wave; t < ntile; t += nwaves) update_tile(p, J + t, false);
    }
  }
  if (J == 0) {
    for (int idx = tid; idx < kPB * kPB; idx += nthr) {
      const int i = idx % kPB, j = idx / kPB;
      if (i >= j && i < nb && j < nb) S.D[i][j] = L[(size_t)j * m + i];
    }
    __syncthreads();
    if (wave == 0) factor_diag();
  }
  __syncthreads();

  if (!timed_out) {
    // the factor's diagonal block, then the panel below: X L11^T = A21, by 32-row tiles
    for (int idx = tid; idx < nb * nb; idx += nthr) {
      const int i = idx % nb, j = idx / nb;
      if (i >= j) L[(size_t)(c0 + j) * m + c0 + i] = S.D[i][j];
    }
    double *const Wt = W[wave];
    for (int I = J + 1 + wave; I < nblk; I += nwaves) {
      const int i0 = kPB * I, rows = m - i0;
      const double *A = L + (size_t)c0 * m + i0;
      double a[2][2][4];  // the panel tile A21, loaded ahead
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * rt + lg + 4 * r, col = 16 * ct + li;
            const bool in = row < rows && col < nb;
            a[rt][ct][r] = A[in ? (size_t)col * m + row : 0];
          }
      d4 x0[2][2];
      zero_acc(x0);
      wave_mma32<false, true>(A, m, &S.Di[0][0], kPB + 1, nb, rows, nb, x0);
      {
        // one refinement step for every block: residual R = A - X0 L11^T and
        // X = X0 + R L11^{-T} (the product with the inverse alone leaves a residual of order
        // the block's condition times rounding), operands through this wave's LDS tile
        // (column-major, leading dimension kPB + 1)
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
          for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = 16 * rt + lg + 4 * r, col = 16 * ct + li;
              Wt[col * (kPB + 1) + row] = (row < rows && col < nb) ? x0[rt][ct][r] : 0.0;
            }
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        __builtin_amdgcn_wave_barrier();
        d4 t1[2][2];
        zero_acc(t1);
        wave_mma32<false, false>(Wt, kPB + 1, &S.D[0][0], kPB + 1, nb, rows, nb, t1);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
          for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = 16 * rt + lg + 4 * r, col = 16 * ct + li;
              Wt[col * (kPB + 1) + row] =
                  (row < rows && col < nb) ? a[rt][ct][r] - t1[rt][ct][r] : 0.0;
            }
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        __builtin_amdgcn_wave_barrier();
        d4 t2[2][2];
        zero_acc(t2);
        wave_mma32<false, true>(Wt, kPB + 1, &S.Di[0][0], kPB + 1, nb, rows, nb, t2);
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
          for (int ct = 0; ct < 2; ++ct) x0[rt][ct] += t2[rt][ct];
        __builtin_amdgcn_wave_barrier();
      }
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * rt + lg + 4 * r, col = 16 * ct + li;
            if (row < rows && col < nb) L[(size_t)(c0 + col) * m + i0 + row] = x0[rt][ct][r];
          }
    }
  }
  // publish: the breakdown and modified words first, then (after every thread's stores are
  // released) the panel flag
  if (tid == 0) {
    if (bad || timed_out) __hip_atomic_store(&sync[kCholSyncBad], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (modified) __hip_atomic_store(&sync[kCholSyncMod], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (tid == 0) __hip_atomic_store(&sync[J], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  // the block's inverse for the right-hand solves after the factorization, once published
  // (off the chain of workgroups waiting on each other)
  if (dinv && !timed_out && wave == nwaves - 1)
    block_inverse_fs((const lds_double *)&S.D[0][0], nb, dinv + (size_t)J * 1024);
  // the last block has waited for every other one: it reports for the factorization
  if (J == nblk - 1 && tid == 0) {
    const int b = __hip_atomic_load(&sync[kCholSyncBad], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    const int md = __hip_atomic_load(&sync[kCholSyncMod], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    if (b) flag[0] = 1;
    if (md && shifts) shifts[0] += 1;
    if (md && modflag) modflag[0] = 1;
    if (ctl.cq) cholqr_ctl_end(ctl, mode == 1, md != 0, b != 0);
  }
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
                    const int *__restrict__ run, const TrsmJob *__restrict__ jobs) {
  if (jobs) {  // batched: blockIdx.y selects the problem
    const TrsmJob &J = jobs[blockIdx.y];
    rows = J.rows, m = J.m, X = J.X, ldx = J.ldx, L = J.L, run = J.run;
  }
  if (run && run[0] == 0) return;
  if ((int)blockIdx.x * 32 >= rows) return;
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
// The same X <- X L^{-T} through the inverses of L's 32 x 32 diagonal blocks, so that
// every step is a matrix-core product instead of a row-by-row substitution.
// trsm_diag_inv_kernel: block b of L (rows and columns 32 b ...) staged in LDS; lane c
// solves L_bb x = e_c by forward substitution; dinv + 1024 b holds L_bb^{-1}
// column-major (ld 32), zero outside the block.
// trsm_rlt_inv_kernel: four waves per 32-row block of X; per column block jb the waves
// split the contraction X[:, <c0] L[jb, <c0]^T four ways, wave 0 adds the partial
// products, forms B = X[:, jb] - (sum) in LDS and writes X[:, jb] = B L_jb^{-T}.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64)
    trsm_diag_inv_kernel(int m, const double *__restrict__ L, double *__restrict__ dinv,
                         const int *__restrict__ run) {
  if (run && run[0] == 0) return;
  __shared__ double Lb[32][33];
  const int lane = threadIdx.x, b = blockIdx.x, c0 = 32 * b, nb = min(32, m - c0);
  for (int idx = lane; idx < 32 * 32; idx += 64) {
    const int i = idx & 31, t = idx >> 5;
    Lb[i][t] = (i < nb && t <= i) ? L[(size_t)(c0 + t) * m + c0 + i] : 0.0;
  }
  __syncthreads();
  if (lane >= 32) return;
  const int c = lane;
  double x[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    double acc = (i == c) ? 1.0 : 0.0;
#pragma unroll
    for (int t = 0; t < i; ++t) acc -= Lb[i][t] * x[t];  // x[t] = 0 for t < c
    x[i] = (i >= c && i < nb) ? acc / Lb[i][i] : 0.0;
  }
  double *o = dinv + (size_t)b * 1024 + (size_t)c * 32;
#pragma unroll
  for (int i = 0; i < 32; ++i) o[i] = x[i];
}

__global__ void __launch_bounds__(256)
    trsm_rlt_inv_kernel(int rows, int m, double *__restrict__ X, int ldx,
                        const double *__restrict__ L, const double *__restrict__ dinv,
                        const int *__restrict__ run, int rows2, double *__restrict__ X2,
                        int ldx2) {
  if (run && run[0] == 0) return;
  __shared__ double red[4][32][33];
  __shared__ double Bm[32 * 33];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lg = lane >> 4;
  int r0 = blockIdx.x * 32;
  const int nblk1 = (rows + 31) / 32;
  if ((int)blockIdx.x >= nblk1) {  // a block of the second matrix
    r0 = ((int)blockIdx.x - nblk1) * 32, rows = rows2, X = X2, ldx = ldx2;
  }
  if (r0 >= rows) return;
  const int nr = min(32, rows - r0);
  for (int jb = 0; jb * 32 < m; ++jb) {
    const int c0 = jb * 32, nc = min(32, m - c0);
    // 1. wave w: X[r0:, k0:k1] L[c0:, k0:k1]^T over its quarter of [0, c0)
    const int k0 = (c0 * wave) / 4, k1 = (c0 * (wave + 1)) / 4;
    d4 acc[2][2];
    zero_acc(acc);
    if (k1 > k0)
      wave_mma32<false, true>(X + r0 + (size_t)k0 * ldx, ldx, L + c0 + (size_t)k0 * m, m, k1 - k0,
                              nr, nc, acc);
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[wave][16 * rt + lg + 4 * r][16 * ct + li] = acc[rt][ct][r];
    __syncthreads();
    if (wave == 0) {
      // 2. B = X[:, jb] - sum of the partial products, column-major in LDS
      for (int idx = lane; idx < 32 * 32; idx += 64) {
        const int i = idx & 31, j = idx >> 5;
        double v = 0.0;
        if (i < nr && j < nc)
          v = X[(size_t)(c0 + j) * ldx + r0 + i] - (red[0][i][j] + red[1][i][j] + red[2][i][j] +
                                                     red[3][i][j]);
        Bm[i + 33 * j] = v;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // 3. X[:, jb] = B L_jb^{-T}
      d4 q[2][2];
      zero_acc(q);
      wave_mma32<false, true>(Bm, 33, dinv + (size_t)jb * 1024, 32, nc, nr, nc, q);
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * rt + lg + 4 * r, col = 16 * ct + li;
            if (row < nr && col < nc) X[(size_t)(c0 + col) * ldx + r0 + row] = q[rt][ct][r];
          }
    }
    __syncthreads();
  }
}

// The same solve with the workgroup's 16-row strip of X held in LDS for m <= kStripM: the
// strip is read once and written once, and the solved column blocks that every later
// block's contraction needs are LDS operands instead of global re-reads. Four waves: wave
// (kh, ct) forms the 16 x 16 tile ct of B = X[:, jb] - X[:, <jb] L[jb, <jb]^T over the
// contraction's chunks of 16 with parity kh (two accumulators, so consecutive MFMAs are
// independent); the kh = 1 partial goes through LDS to its kh = 0 partner, which completes
// B; then each kh = 0 wave multiplies the strip's B by its column tile of L_jb^{-T}. Sixteen
// rows per workgroup give a 4096-row block 256 workgroups, one per CU, and the k split
// halves each wave's chain of MFMAs.
constexpr int kStripM = 288;
constexpr int kSR = 16;           // rows per strip
constexpr int kXsLd = kSR + 1;    // LDS stride of the strip's columns

__global__ void __launch_bounds__(256)
    trsm_rlt_inv_strip_kernel(int rows, int m, double *__restrict__ X, int ldx,
                              const double *__restrict__ L, const double *__restrict__ dinv,
                              const int *__restrict__ run, int rows2, double *__restrict__ X2,
                              int ldx2, const double *__restrict__ Xsrc) {
  if (run && run[0] == 0) return;
  __shared__ double xs[kStripM * kXsLd];  // xs[j kXsLd + i] = X[r0 + i][j]
  __shared__ double Bm[32 * kXsLd];       // B, column-major
  __shared__ double part[2][4 * 64];      // the kh = 1 partial sums, per tile and lane
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lg = lane >> 4;
  int r0 = blockIdx.x * kSR;
  const int nblk1 = (rows + kSR - 1) / kSR;
  // the first matrix's values come from Xsrc when given (same leading dimension)
  const double *src = Xsrc ? Xsrc : X;
  if ((int)blockIdx.x >= nblk1) {  // a block of the second matrix
    r0 = ((int)blockIdx.x - nblk1) * kSR, rows = rows2, X = X2, ldx = ldx2, src = X2;
  }
  if (r0 >= rows) return;
  const int nr = min(kSR, rows - r0);
  {
    // every load of the strip issued before the first wait (at a clamped address where the
    // strip ends; those values are dropped), then the LDS writes
    constexpr int kPer = kSR * kStripM / 256;
    const int i = tid & (kSR - 1), ic = min(i, nr - 1);
    double v[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const int j = min((tid >> 4) + 16 * t, m - 1);
      v[t] = src[(size_t)j * ldx + r0 + ic];
    }
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const int j = (tid >> 4) + 16 * t;
      if (j < m) xs[j * kXsLd + i] = (i < nr) ? v[t] : 0.0;
    }
  }
  __syncthreads();
  const int ct = wave & 1, kh = wave >> 1;
  constexpr int kChunks = (kStripM - 32) / 16;
  for (int jb = 0; jb * 32 < m; ++jb) {
    const int c0 = jb * 32, nc = min(32, m - c0);
    const int bcol = c0 + 16 * ct + li;  // B-operand column (a row of L) of this lane
    const bool bin = bcol < m;
    // this wave's column tile of L_jb^{-T}: op[k][j] = dinv[1024 jb + 32 k + 16 ct + j]
    double dv[8];
    if (kh == 0) {
#pragma unroll
      for (int s = 0; s < 8; ++s)
        dv[s] = dinv[(size_t)jb * 1024 + 32 * (4 * s + lg) + 16 * ct + li];
    }
    // 1. this wave's share of X[:, 0:c0] L[c0 + 16 ct.., 0:c0]^T: chunks q = kh, kh + 2, ..
    //    below c0, every L operand loaded at once
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
    if (c0 > 0) {
      constexpr int kMine = (kChunks + 1) / 2;
      double bl[4 * kMine];
#pragma unroll
      for (int h = 0; h < kMine; ++h)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int k = 16 * (2 * h + kh) + 4 * s + lg;
          bl[4 * h + s] = (bin && k < c0) ? L[(size_t)k * m + bcol] : 0.0;
        }
      d4 acc1 = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int h = 0; h < kMine; ++h) {
        const int q = 2 * h + kh;
        if (16 * q < c0) {
#pragma unroll
          for (int s = 0; s < 4; s += 2) {
            const double a0 = xs[(16 * q + 4 * s + lg) * kXsLd + li];
            const double a1 = xs[(16 * q + 4 * s + 4 + lg) * kXsLd + li];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bl[4 * h + s], acc, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bl[4 * h + s + 1], acc1, 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] += acc1[r];
      if (kh == 1) {
#pragma unroll
        for (int r = 0; r < 4; ++r) part[ct][r * 64 + lane] = acc[r];
      }
    }
    __syncthreads();
    // 2. the kh = 0 waves complete their tile of B into LDS (rows >= nr and columns >= nc
    //    zero)
    if (kh == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = lg + 4 * r, col = 16 * ct + li;
        const double p = (c0 > 0) ? part[ct][r * 64 + lane] : 0.0;
        Bm[row + kXsLd * col] =
            (row < nr && col < nc) ? xs[(c0 + col) * kXsLd + row] - (acc[r] + p) : 0.0;
      }
    }
    __syncthreads();
    // 3. X[:, c0 + 16 ct..] = B L_jb^{-T}[:, 16 ct..], into the strip
    if (kh == 0) {
      d4 q = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 8; ++s)
        q = __builtin_amdgcn_mfma_f64_16x16x4f64(Bm[li + kXsLd * (4 * s + lg)], dv[s], q, 0, 0,
                                                 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = lg + 4 * r, col = 16 * ct + li;
        if (row < nr && col < nc) xs[(c0 + col) * kXsLd + row] = q[r];
      }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < kSR * m; idx += 256) {
    const int i = idx & (kSR - 1), j = idx >> 4;
    if (i < nr) X[(size_t)j * ldx + r0 + i] = xs[j * kXsLd + i];
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

// out[0] = ||R||_F / ||A||_F over count elements (one workgroup, fixed summation order).
__global__ void __launch_bounds__(1024) fro_ratio_kernel(long long count,
                                                         const double *__restrict__ R,
                                                         const double *__restrict__ A,
                                                         double *__restrict__ out) {
  __shared__ double red[16];
  double pr = 0.0, pa = 0.0;
  for (long long idx = threadIdx.x; idx < count; idx += blockDim.x) {
    pr += R[idx] * R[idx];
    pa += A[idx] * A[idx];
  }
  const double sr = wg_sum(pr, red);
  const double sa = wg_sum(pa, red);
  if (threadIdx.x == 0) out[0] = sqrt(sr) / sqrt(sa);
}

// ---------------------------------------------------------------------------
// Increment, covariance and utility kernels
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool use_lru(int mode_lru, const double *lam, int k) {
  if (mode_lru == 0) return false;
  if (mode_lru == 1) return true;
  return !(lam[k - 1] >= 1.0);  // adaptive (eq. 11)
}

// Rows are split four ways: a workgroup takes 64 rows, wave w sums the columns j = w (mod 4)
// of each row, and the four partial sums are added in a fixed order through LDS, so a row's
// dependent chain is k / 4 long (and deterministic). The per-column factors (a division
// each) are formed once per workgroup into LDS, kCoefChunk columns at a time.
constexpr int kRowsPerWg = 64;
constexpr int kCoefChunk = 1024;

__global__ void __launch_bounds__(256)
    increment_kernel(int n, int k, const double *__restrict__ lam,
                     const double *__restrict__ V, const double *__restrict__ c,
                     const double *__restrict__ g, int mode_lru,
                     double *__restrict__ dz, double *__restrict__ dofs,
                     const IncJob *__restrict__ jobs) {
  if (jobs) {  // batched: blockIdx.y selects the problem
    const IncJob &J = jobs[blockIdx.y];
    n = J.n, k = J.k, lam = J.lam, V = J.V, c = J.c, g = J.g, dz = J.dz, dofs = J.dofs;
  }
  __shared__ double part[4][kRowsPerWg];
  __shared__ double cf[kCoefChunk];  // c_j times the filter factor, a chunk of j at a time
  __shared__ double red[16];
  const bool lru = use_lru(mode_lru, lam, k);
  const int r = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = blockIdx.x * kRowsPerWg + r;
  double s = 0.0;
  for (int j0 = 0; j0 < k; j0 += kCoefChunk) {
    const int jn = min(kCoefChunk, k - j0);
    __syncthreads();
    for (int t = threadIdx.x; t < jn; t += blockDim.x) {
      const double lj = lam[j0 + t];
      const double a = lru ? lj / (1.0 + lj) : 1.0 / (1.0 + lj);
      cf[t] = c[j0 + t] * a;
    }
    __syncthreads();
    if (i < n) {
      const gmem<double> *Vg = gptr(V);
#pragma unroll 8
      for (int j = w; j < jn; j += 4) s += Vg[(size_t)(j0 + j) * n + i] * cf[j];
    }
  }
  part[w][r] = s;
  __syncthreads();
  if (w == 0 && i < n) {
    const double t = (part[0][r] + part[1][r]) + (part[2][r] + part[3][r]);
    dz[i] = lru ? -(g[i] - t) : -t;
  }
  if (blockIdx.x == 0 && dofs) {  // sum of lambda / (1 + lambda), fixed order
    double d = 0.0;
    for (int j = threadIdx.x; j < k; j += blockDim.x) d += lam[j] / (1.0 + lam[j]);
    d = wg_sum(d, red);
    if (threadIdx.x == 0) dofs[0] = d;
  }
}

__global__ void choose_mode_kernel(int k, const double *__restrict__ lam, int *__restrict__ out) {
  if (threadIdx.x == 0) out[0] = (lam[k - 1] >= 1.0) ? (int)RIOT_LRA : (int)RIOT_LRU;
}

// The same four-way split of each row's sum over the k columns of W.
__global__ void __launch_bounds__(256)
    postcov_diag_kernel(int n, int k, const double *__restrict__ lam,
                        const double *__restrict__ W, int mode_lru, double base_diag,
                        double *__restrict__ coef, double *__restrict__ diag) {
  __shared__ double part[4][kRowsPerWg];
  __shared__ double cf[kCoefChunk];
  const bool lru = use_lru(mode_lru, lam, k);
  if (blockIdx.x == 0 && coef) {
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
      const double lj = lam[j];
      coef[j] = lru ? -lj / (1.0 + lj) : 1.0 / (1.0 + lj);
    }
  }
  if (!diag) return;
  const int r = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = blockIdx.x * kRowsPerWg + r;
  double s = 0.0;
  for (int j0 = 0; j0 < k; j0 += kCoefChunk) {
    const int jn = min(kCoefChunk, k - j0);
    __syncthreads();
    for (int t = threadIdx.x; t < jn; t += blockDim.x) {
      const double lj = lam[j0 + t];
      cf[t] = lru ? -lj / (1.0 + lj) : 1.0 / (1.0 + lj);
    }
    __syncthreads();
    if (i < n) {
      const gmem<double> *Wg = gptr(W);
#pragma unroll 8
      for (int j = w; j < jn; j += 4) {
        const double x = Wg[(size_t)(j0 + j) * n + i];
        s += cf[j] * x * x;
      }
    }
  }
  part[w][r] = s;
  __syncthreads();
  if (w == 0 && i < n)
    diag[i] = (lru ? base_diag : 0.0) + ((part[0][r] + part[1][r]) + (part[2][r] + part[3][r]));
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
                                    int *__restrict__ flag, long long count2,
                                    const double *__restrict__ x2) {
  const long long i0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  bool bad = false;
  for (long long i = i0; i < count; i += stride) bad |= !isfinite(x[i]);
  for (long long i = i0; i < count2; i += stride) bad |= !isfinite(x2[i]);
  if (bad) flag[0] = 1;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

// y = alpha A^T x + beta y for A (K x M, leading dimension lda): one workgroup per output,
// its 256 threads reading the column A[:, c] and x coalesced (eight loads in flight each),
// the partial sums reduced in a fixed order (wave trees, then the four waves in turn).
__global__ void __launch_bounds__(256)
    gemv_t_kernel(int M, int K, const double *__restrict__ A, int lda,
                  const double *__restrict__ x, double *__restrict__ y, double alpha,
                  double beta) {
  const int c = blockIdx.x;
  if (c >= M) return;
  const double *a = A + (size_t)c * lda;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double acc = 0.0;
  for (int kb = 0; kb < K; kb += 8 * 256) {
    double av[8], xv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = kb + u * 256 + tid;
      const int kc = k < K ? k : 0;
      av[u] = a[kc];
      xv[u] = x[kc];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = (kb + u * 256 + tid < K) ? fma(av[u], xv[u], acc) : acc;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  __shared__ double red[4];
  if (lane == 0) red[wave] = acc;
  __syncthreads();
  if (tid == 0) {
    const double sum = (red[0] + red[1]) + (red[2] + red[3]);
    double out = alpha * sum;
    if (beta != 0.0) out += beta * y[c];
    y[c] = out;
  }
}

hipError_t gemm_f64(int ta, int tb, int M, int N, int K, double alpha, const double *A, int lda,
                    const double *B, int ldb, double beta, double *C, int ldc, double *partial,
                    int splitk, hipStream_t st, const int *run, bool lower, double *gram_sq,
                    const double *B2, double *C2, bool sym) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (lower && !(ta == 1 && tb == 0 && M == N)) return hipErrorInvalidValue;
  if (N == 1 && ta == 1 && tb == 0 && !lower && !gram_sq && !B2 && !run && K > 0) {
    // a matrix-vector product: one workgroup per output instead of a 32-wide MFMA tile
    hipLaunchKernelGGL(gemv_t_kernel, dim3(M), dim3(256), 0, st, M, K, A, lda, B, C, alpha,
                       beta);
    return hipGetLastError();
  }
  // pair form: [C C2] = alpha op(A)^T [B B2] + beta [C C2], two results of N columns each
  const bool pair = B2 != nullptr;
  if (pair && (!C2 || tb != 0 || lower || gram_sq)) return hipErrorInvalidValue;
  if (sym && (M != N || lower || gram_sq || pair || beta != 0.0 || !partial))
    return hipErrorInvalidValue;
  // two products instead when too small for the LDS kernel, or when one product's tiles
  // already fill the chip (no split over K to share)
  if (pair && (!(M >= kGT && 2 * N >= kGT) ||
               ((M + kGT - 1) / kGT) * ((N + kGT - 1) / kGT) >= 256)) {
    hipError_t e = gemm_f64(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, partial,
                            splitk, st, run);
    if (e != hipSuccess) return e;
    return gemm_f64(ta, tb, M, N, K, alpha, A, lda, B2, ldb, beta, C2, ldc, partial, splitk, st,
                    run);
  }
  const int N1 = N;
  if (pair) N = 2 * N;
  if (gram_sq && (!lower || !partial || K <= 0 || beta != 0.0)) return hipErrorInvalidValue;
  if (K <= 0) splitk = 1;
  if (splitk < 1 || !partial) splitk = 1;
  // 64 x 64 tiles through LDS when both sides span a tile, else one wave per 32 x 32 tile
  const bool big = M >= kGT && N >= kGT;
  const int kround = big ? kGK : 4;
  const int tm = (M + kGT - 1) / kGT, tn = (N + kGT - 1) / kGT;
  const int tiles = lower ? tm * (tm + 1) / 2 : tm * tn;
  // about one workgroup per CU: no more K splits than fill 256 CUs with the tiles (when that
  // is a multiple of 8, each split's workgroups share an XCD, see gemm_lds_kernel)
  // (the pair form: two workgroups per CU, which hide each other's latencies)
  if (big && splitk > 1) splitk = std::max(1, std::min(splitk, (pair ? 512 : 256) / tiles));
  int kchunk = (K + splitk - 1) / splitk;
  kchunk = (kchunk + kround - 1) / kround * kround;
  if (kchunk <= 0) kchunk = kround;
  const int splits = K > 0 ? (K + kchunk - 1) / kchunk : 1;
  // the Gram-with-squares form always goes through the reduction, which writes them
  double *part = (splits > 1 || gram_sq || sym) ? partial : nullptr;
  if (big) {
    dim3 grid(tm, tn, splits);
    int xs = 0;
    if (splits % kXcds == 0) {
      xs = 1, grid = dim3((unsigned)(tiles * splits), 1, 1);
    } else if (splits == 1 && !lower && tm % kXcds == 0) {
      xs = -1, grid = dim3((unsigned)(tm * tn), 1, 1);
    }
#define RIOT_GEMM_LDS(TA_, TB_, LO_)                                                            \
  hipLaunchKernelGGL((gemm_lds_kernel<TA_, TB_, LO_>), grid, dim3(256), 0, st, M, N, K, A, lda, B, \
                     ldb, C, ldc, alpha, beta, kchunk, part, run, xs, nullptr, nullptr, N)
    if (pair && ta == 1)
      hipLaunchKernelGGL((gemm_lds_kernel<1, 0, false, true>), grid, dim3(256), 0, st, M, N, K, A,
                         lda, B, ldb, C, ldc, alpha, beta, kchunk, part, run, xs, B2, C2, N1);
    else if (pair)
      hipLaunchKernelGGL((gemm_lds_kernel<0, 0, false, true>), grid, dim3(256), 0, st, M, N, K, A,
                         lda, B, ldb, C, ldc, alpha, beta, kchunk, part, run, xs, B2, C2, N1);
    else if (ta == 0 && tb == 0)
      RIOT_GEMM_LDS(0, 0, false);
    else if (ta == 1 && tb == 0 && lower)
      RIOT_GEMM_LDS(1, 0, true);
    else if (ta == 1 && tb == 0)
      RIOT_GEMM_LDS(1, 0, false);
    else if (ta == 0 && tb == 1)
      RIOT_GEMM_LDS(0, 1, false);
    else
      RIOT_GEMM_LDS(1, 1, false);
#undef RIOT_GEMM_LDS
  } else {
    if (pair) return hipErrorInvalidValue;  // the pair form runs on the LDS kernel only
    dim3 grid((M + 31) / 32, (N + 31) / 32, splits);
#define RIOT_GEMM(TA_, TB_)                                                                  \
  hipLaunchKernelGGL((gemm_mfma_kernel<TA_, TB_>), grid, dim3(64), 0, st, M, N, K, A, lda, B, \
                     ldb, C, ldc, alpha, beta, kchunk, part, run, nullptr, 0, 0, 0)
    if (ta == 0 && tb == 0)
      RIOT_GEMM(0, 0);
    else if (ta == 1 && tb == 0 && lower)
      hipLaunchKernelGGL((gemm_mfma_kernel<1, 0, true>), grid, dim3(64), 0, st, M, N, K, A, lda, B,
                         ldb, C, ldc, alpha, beta, kchunk, part, run, nullptr, 0, 0, 0);
    else if (ta == 1 && tb == 0)
      RIOT_GEMM(1, 0);
    else if (ta == 0 && tb == 1)
      RIOT_GEMM(0, 1);
    else
      RIOT_GEMM(1, 1);
#undef RIOT_GEMM
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (part) {
    const size_t MN = (size_t)M * N;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((MN + 255) / 256)), dim3(256), 0, st,
                       M, N, splits, partial, alpha, beta, C, ldc, run, lower ? 1 : 0, gram_sq,
                       C2, N1, sym ? 1 : 0);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_chol_blocked(int m, const double *G, double *L, double shift_rel, int mode,
                               int *flag, int *shifts, hipStream_t st, const int *run,
                               int *modflag, const double *gram_sq, double *dinv,
                               CholQrCtl ctl) {
  if (gram_sq && G != L) return hipErrorInvalidValue;
  if (!gram_sq && (dinv || ctl.cq)) return hipErrorInvalidValue;
  if (ctl.cq && (ctl.pass < 0 || ctl.pass >= ctl.npass)) return hipErrorInvalidValue;
  // up to the staged panel height one workgroup is faster (the critical path is the chain of
  // diagonal blocks either way); beyond it the trailing updates dominate and are spread
  if (gram_sq && m > kStageRows + kPB) {
    if ((m + kPB - 1) / kPB > kCholMaxBlocks) return hipErrorInvalidValue;
    hipLaunchKernelGGL(chol_mwg_kernel, dim3((m + kPB - 1) / kPB), dim3(kCholThreads), 0, st, m,
                       L, shift_rel, mode, flag, shifts, run, modflag, const_cast<double *>(gram_sq),
                       dinv, ctl);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(chol_blocked_kernel, dim3(1), dim3(kCholThreads), 0, st, m, G, L, shift_rel,
                     mode, flag, shifts, run, modflag, gram_sq, dinv, ctl,
                     static_cast<const CholJob *>(nullptr));
  return hipGetLastError();
}

hipError_t launch_trsm_diag_inv(int m, const double *L, double *dinv, hipStream_t st,
                                const int *run) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(trsm_diag_inv_kernel, dim3((m + 31) / 32), dim3(64), 0, st, m, L, dinv, run);
  return hipGetLastError();
}

hipError_t launch_trsm_rlt_inv(int rows, int m, double *X, int ldx, const double *L,
                               const double *dinv, hipStream_t st, const int *run, int rows2,
                               double *X2, int ldx2, const double *Xsrc) {
  if (!X2) rows2 = 0;
  if (rows < 0 || rows2 < 0 || m <= 0 || rows + rows2 == 0) return hipSuccess;
  if (Xsrc == X) Xsrc = nullptr;
  if (Xsrc && m > kStripM) {  // the general kernel solves in place: copy first
    if (run) return hipErrorInvalidValue;  // the copy could not be predicated
    const hipError_t e = hipMemcpyAsync(X, Xsrc, (size_t)ldx * m * sizeof(double),
                                        hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    Xsrc = nullptr;
  }
  if (m <= kStripM)
    hipLaunchKernelGGL(trsm_rlt_inv_strip_kernel,
                       dim3((rows + kSR - 1) / kSR + (rows2 + kSR - 1) / kSR), dim3(256), 0, st,
                       rows, m, X, ldx, L, dinv, run, rows2, X2, ldx2, Xsrc);
  else
    hipLaunchKernelGGL(trsm_rlt_inv_kernel, dim3((rows + 31) / 32 + (rows2 + 31) / 32), dim3(256),
                       0, st, rows, m, X, ldx, L, dinv, run, rows2, X2, ldx2);
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

hipError_t launch_symmetrize(int m, double *K, double *asym, double *part, hipStream_t st) {
  const int nblk = 64;
  hipLaunchKernelGGL(symmetrize_kernel, dim3(nblk), dim3(256), 0, st, m, K, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !asym) return e;
  hipLaunchKernelGGL(symmetrize_norm_kernel, dim3(1), dim3(64), 0, st, nblk, part, asym);
  return hipGetLastError();
}

hipError_t launch_orth_err(int m, const double *G, double *out, hipStream_t st) {
  hipLaunchKernelGGL(orth_err_kernel, dim3(1), dim3(1024), 0, st, m, G, out);
  return hipGetLastError();
}

hipError_t launch_fro_ratio(long long count, const double *R, const double *A, double *out,
                            hipStream_t st) {
  hipLaunchKernelGGL(fro_ratio_kernel, dim3(1), dim3(1024), 0, st, count, R, A, out);
  return hipGetLastError();
}

hipError_t launch_increment_combine(int n, int k, const double *lam, const double *V,
                                    const double *c, const double *g, int mode_lru, double *dz,
                                    double *dofs, hipStream_t st) {
  hipLaunchKernelGGL(increment_kernel, dim3((n + kRowsPerWg - 1) / kRowsPerWg), dim3(256), 0, st, n,
                     k, lam, V, c, g, mode_lru, dz, dofs, nullptr);
  return hipGetLastError();
}

hipError_t launch_choose_mode(int k, const double *lam, int *out, hipStream_t st) {
  hipLaunchKernelGGL(choose_mode_kernel, dim3(1), dim3(64), 0, st, k, lam, out);
  return hipGetLastError();
}

hipError_t launch_postcov_diag(int n, int k, const double *lam, const double *W, int mode_lru,
                               double base_diag, double *coef, double *diag, hipStream_t st) {
  hipLaunchKernelGGL(postcov_diag_kernel, dim3((n + kRowsPerWg - 1) / kRowsPerWg), dim3(256), 0, st,
                     n, k, lam, W, mode_lru, base_diag, coef, diag);
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

hipError_t launch_check_finite(long long count, const double *x, int *flag, hipStream_t st,
                               long long count2, const double *x2) {
  if (!x2) count2 = 0;
  if (count <= 0 && count2 <= 0) return hipSuccess;
  long long blocks = (std::max(count, count2) + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(check_finite_kernel, dim3((unsigned)blocks), dim3(256), 0, st, count, x, flag,
                     count2, x2);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Batched launches (one job per problem; see the job structs in the internal header)
// ---------------------------------------------------------------------------

__global__ void cholqr_reset_batched_kernel(const CqJob *__restrict__ jobs) {
  if (threadIdx.x == 0) {
    int *cq = jobs[blockIdx.x].cq;
    cq[0] = 1;
    cq[1] = 0;
    cq[2] = 0;
  }
}

__global__ void cholqr_ctrl_batched_kernel(const CqJob *__restrict__ jobs, int pass_was_shifted) {
  if (threadIdx.x != 0) return;
  int *cq = jobs[blockIdx.x].cq;
  if (cq[0] == 0) return;
  int *count = jobs[blockIdx.x].count;
  if (count) count[0] += 1;
  if (pass_was_shifted || cq[2])
    cq[1] = 0;
  else
    cq[1] += 1;
  cq[2] = 0;
  if (cq[1] >= 2) cq[0] = 0;
}

// K <- (K + K^T) / 2, one workgroup per problem.
__global__ void __launch_bounds__(256) symmetrize_batched_kernel(const SymJob *__restrict__ jobs) {
  const int m = jobs[blockIdx.x].m;
  double *K = jobs[blockIdx.x].K;
  for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
    const int i = idx % m, j = idx / m;
    if (i > j) {
      const double a = 0.5 * (K[(size_t)j * m + i] + K[(size_t)i * m + j]);
      K[(size_t)j * m + i] = a;
      K[(size_t)i * m + j] = a;
    }
  }
}

__global__ void copy_batched_kernel(const CopyJob *__restrict__ jobs) {
  const CopyJob &J = jobs[blockIdx.y];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < J.count;
       i += (long long)gridDim.x * blockDim.x)
    J.dst[i] = J.src[i];
}

hipError_t launch_gemm_batched(int ta, int tb, int nprob, int maxM, int maxN, double alpha,
                               double beta, const GemmJob *jobs, hipStream_t st) {
  if (nprob <= 0 || maxM <= 0 || maxN <= 0) return hipSuccess;
  dim3 grid((maxM + 31) / 32, (maxN + 31) / 32, nprob);
#define RIOT_GEMMB(TA_, TB_)                                                                    \
  hipLaunchKernelGGL((gemm_mfma_kernel<TA_, TB_>), grid, dim3(64), 0, st, 0, 0, 0, nullptr, 0,   \
                     nullptr, 0, nullptr, 0, alpha, beta, 0, nullptr, nullptr, jobs, 0, 0, 0)
  if (ta == 0 && tb == 0)
    RIOT_GEMMB(0, 0);
  else if (ta == 1 && tb == 0)
    RIOT_GEMMB(1, 0);
  else if (ta == 0 && tb == 1)
    RIOT_GEMMB(0, 1);
  else
    RIOT_GEMMB(1, 1);
#undef RIOT_GEMMB
  return hipGetLastError();
}

hipError_t launch_chol_batched(int nprob, int mode, const CholJob *jobs, hipStream_t st) {
  if (nprob <= 0) return hipSuccess;
  hipLaunchKernelGGL(chol_blocked_kernel, dim3(1, nprob), dim3(kCholThreads), 0, st, 0, nullptr,
                     nullptr, 0.0, mode, nullptr, nullptr, nullptr, nullptr, nullptr,
                     static_cast<double *>(nullptr), CholQrCtl(), jobs);
  return hipGetLastError();
}

hipError_t launch_trsm_batched(int nprob, int maxrows, const TrsmJob *jobs, hipStream_t st) {
  if (nprob <= 0 || maxrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(trsm_rlt_kernel, dim3((maxrows + 31) / 32, nprob), dim3(64), 0, st, 0, 0,
                     nullptr, 0, nullptr, nullptr, jobs);
  return hipGetLastError();
}

hipError_t launch_cholqr_reset_batched(int nprob, const CqJob *jobs, hipStream_t st) {
  if (nprob <= 0) return hipSuccess;
  hipLaunchKernelGGL(cholqr_reset_batched_kernel, dim3(nprob), dim3(64), 0, st, jobs);
  return hipGetLastError();
}

hipError_t launch_cholqr_ctrl_batched(int nprob, int pass_was_shifted, const CqJob *jobs,
                                      hipStream_t st) {
  if (nprob <= 0) return hipSuccess;
  hipLaunchKernelGGL(cholqr_ctrl_batched_kernel, dim3(nprob), dim3(64), 0, st, jobs,
                     pass_was_shifted);
  return hipGetLastError();
}

hipError_t launch_symmetrize_batched(int nprob, const SymJob *jobs, hipStream_t st) {
  if (nprob <= 0) return hipSuccess;
  hipLaunchKernelGGL(symmetrize_batched_kernel, dim3(nprob), dim3(256), 0, st, jobs);
  return hipGetLastError();
}

hipError_t launch_increment_batched(int nprob, int maxn, int mode_lru, const IncJob *jobs,
                                    hipStream_t st) {
  if (nprob <= 0 || maxn <= 0) return hipSuccess;
  hipLaunchKernelGGL(increment_kernel, dim3((maxn + kRowsPerWg - 1) / kRowsPerWg, nprob), dim3(256), 0,
                     st, 0, 0, nullptr, nullptr, nullptr, nullptr, mode_lru, nullptr, nullptr, jobs);
  return hipGetLastError();
}

hipError_t launch_copy_batched(int nprob, long long maxcount, const CopyJob *jobs,
                               hipStream_t st) {
  if (nprob <= 0 || maxcount <= 0) return hipSuccess;
  const long long blocks = std::min<long long>((maxcount + 255) / 256, 64);
  hipLaunchKernelGGL(copy_batched_kernel, dim3((unsigned)blocks, nprob), dim3(256), 0, st, jobs);
  return hipGetLastError();
}


hipError_t gemm_f64_strided(int ta, int tb, int M, int N, int K, double alpha, const double *A,
                            int lda, long long sA, const double *B, int ldb, long long sB,
                            double beta, double *C, int ldc, long long sC, int batch,
                            hipStream_t st) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if (!(sA | sB | sC)) return hipErrorInvalidValue;
  dim3 grid((M + 31) / 32, (N + 31) / 32, batch);
#define RIOT_GEMMS(TA_, TB_)                                                                  \
  hipLaunchKernelGGL((gemm_mfma_kernel<TA_, TB_>), grid, dim3(64), 0, st, M, N, K, A, lda, B, \
                     ldb, C, ldc, alpha, beta, K, nullptr, nullptr, nullptr, sA, sB, sC)
  if (ta == 0 && tb == 0)
    RIOT_GEMMS(0, 0);
  else if (ta == 1 && tb == 0)
    RIOT_GEMMS(1, 0);
  else if (ta == 0 && tb == 1)
    RIOT_GEMMS(0, 1);
  else
    RIOT_GEMMS(1, 1);
#undef RIOT_GEMMS
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Spectral preconditioner factors (eq. 7) and small vector updates of the outer loop.
// ---------------------------------------------------------------------------

namespace {

// C[i, c] *= (1 + max(lam_i, 0))^power - 1 for an m_j x m block (ld m_j): the middle factor of
// I + V ((lam + 1)^power - 1) V^T (power -1/2: the preconditioner factor, +1/2: its inverse).
// Ritz values of the positive semi-definite preconditioned Hessian below zero are rounding and
// are taken as zero.
__global__ void precond_scale_kernel(int mj, int m, const double *__restrict__ lam, double power,
                                     double *__restrict__ C) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)mj * m) return;
  const int i = (int)(e % mj);
  const double lt = 1.0 + fmax(lam[i], 0.0);
  C[e] *= pow(lt, power) - 1.0;
}

// Zero the entries of an m x m matrix (ld m) outside the block band |bi - bj| <= 1 of l x l
// blocks (the never-written blocks of a block tridiagonal matrix).
__global__ void block_band_zero_kernel(int m, int l, double *__restrict__ T) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)m * m) return;
  const int i = (int)(e % m), j = (int)(e / m);
  const int d = i / l - j / l;
  if (d > 1 || d < -1) T[e] = 0.0;
}

// Y[e] = a Y[e] + b X[e]
__global__ void axpby_kernel(long long count, double a, double *__restrict__ Y, double b,
                             const double *__restrict__ X) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) Y[e] = a * Y[e] + b * X[e];
}

}  // namespace

hipError_t launch_precond_scale(int mj, int m, const double *lam, double power, double *C,
                                hipStream_t st) {
  const long long tot = (long long)mj * m;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(precond_scale_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                     mj, m, lam, power, C);
  return hipGetLastError();
}

hipError_t launch_block_band_zero(int m, int l, double *T, hipStream_t st) {
  const long long tot = (long long)m * m;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(block_band_zero_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                     m, l, T);
  return hipGetLastError();
}

hipError_t launch_axpby(long long count, double a, double *Y, double b, const double *X,
                        hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(axpby_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count,
                     a, Y, b, X);
  return hipGetLastError();
}

}  // namespace riot
