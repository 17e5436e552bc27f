// FP64 matrix-core tile helpers shared by the dense kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace riot {

typedef double d4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// 32 x 32 wave-level MFMA block product: acc += op(A)[0:32, 0:K] op(B)[0:K, 0:32],
// op(A)[i][k] = TA ? A[k + i*lda] : A[i + k*lda], op(B)[k][j] = TB ? B[j + k*ldb] : B[k + j*ldb].
// Rows >= mA and columns >= nB read as zero. The lane owning result register r
// of tile (rt, ct) holds element (16 rt + l/16 + 4 r, 16 ct + l%16). NCT = 1 computes only the
// first 16 columns (half the MFMAs, for operands 16 columns wide).
// ---------------------------------------------------------------------------

// PA, PB: pointers to double, in the generic or the global address space.
template <bool TA, bool TB, int NCT = 2, typename PA, typename PB>
__device__ __forceinline__ void mma32_load(PA A, int lda, PB B, int ldb, int K, int mA, int nB,
                                           int k0, double (&av)[4][2], double (&bv)[4][NCT]) {
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
    for (int ct = 0; ct < NCT; ++ct) {
      const int col = 16 * ct + li;
      bv[s][ct] = (kin && col < nB) ? (TB ? B[col + (size_t)kk * ldb] : B[kk + (size_t)col * ldb]) : 0.0;
    }
  }
}

// The contraction runs in chunks of 16 (four MFMA k-steps); the operands of the next
// chunk are loaded before the current chunk's MFMAs are issued.
template <bool TA, bool TB, int NCT = 2, typename PA, typename PB>
__device__ __forceinline__ void wave_mma32(PA A, int lda, PB B, int ldb, int K, int mA, int nB,
                                           d4 (&acc)[2][NCT]) {
  if (K <= 0) return;
  double av[4][2], bv[4][NCT], an[4][2], bn[4][NCT];
  mma32_load<TA, TB, NCT>(A, lda, B, ldb, K, mA, nB, 0, av, bv);
  for (int k0 = 0; k0 < K; k0 += 16) {
    const bool more = k0 + 16 < K;
    if (more) mma32_load<TA, TB, NCT>(A, lda, B, ldb, K, mA, nB, k0 + 16, an, bn);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
          acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s][rt], bv[s][ct], acc[rt][ct], 0, 0, 0);
    if (more) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
#pragma unroll
        for (int t = 0; t < 2; ++t) av[s][t] = an[s][t];
#pragma unroll
        for (int t = 0; t < NCT; ++t) bv[s][t] = bn[s][t];
      }
    }
  }
}

template <int NCT = 2>
__device__ __forceinline__ void zero_acc(d4 (&acc)[2][NCT]) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < NCT; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
}

}  // namespace riot
