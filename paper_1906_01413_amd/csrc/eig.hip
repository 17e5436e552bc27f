// Symmetric eigen-solver for the m x m matrix K of the randomized eigendecomposition
// (Alg. 3: K = Z Lambda Z^T), FP64, for gfx950.
//
//  1. Householder tridiagonalisation Q^T K Q = T (one workgroup; reflectors kept).
//  2. Root representation: T - sigma I = L D L^T positive definite, sigma just below
//     the smallest eigenvalue (found by bisection with Sturm counts).
//  3. Eigenvalues of L D L^T to high relative accuracy: one wave per eigenvalue,
//     64-way multisection with negative counts from the stationary qd transform
//     (geometric brackets first, then uniform ones).
//  4. Eigenvectors: twisted factorisation of L D L^T - mu I (stationary and
//     progressive qd transforms, twist index of the smallest gamma) with two
//     Rayleigh-quotient corrections; one thread per eigenvalue.
//  5. Eigenvalues closer than a relative gap of 1e-3 are treated as a cluster:
//     their vectors are re-orthonormalised and rotated by a small Rayleigh-Ritz
//     (Jacobi) solve on T restricted to the cluster.
//  6. Back-transformation by the reflectors and descending order.
//
// Steps 2-4 follow the relatively-robust-representation approach of Dhillon &
// Parlett (2004) for the tridiagonal eigenproblem.

#include "riot_internal.h"
#include "mfma_tile.h"

namespace riot {
namespace {

__device__ double wsum(double v, double *red) {
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

// work layout (doubles): Aw[m*m] Hv[m*m] Z[m*m] d[m] e[m] D[m] Ls[m] LLD[m] mu[m] misc[16]
//                        scratch for the vector kernel: 4 * m * m (at least one 32 x 32
//                        block per 32 reflectors for the back-transform)
struct EigLayout {
  size_t Aw, Hv, Z, d, e, D, Ls, LLD, mu, misc, scr, total;
  __host__ __device__ EigLayout(int m) {
    const size_t mm = (size_t)m * m;
    Aw = 0;
    Hv = mm;
    Z = 2 * mm;
    d = 3 * mm;
    e = d + m;
    D = e + m;
    Ls = D + m;
    LLD = Ls + m;
    mu = LLD + m;
    misc = mu + m;
    scr = misc + 16;
    // the scratch also holds the blocked back-transform's 32 x 32 factors, one per 32 reflectors
    const size_t wy = (size_t)((m + 31) / 32) * 32 * 32;
    total = scr + (4 * mm > wy ? 4 * mm : wy);
  }
};

constexpr int kTriThreads = 512;
constexpr int kEigMaxM = 1088;  // largest m of the eigen-solver

// ---------------------------------------------------------------------------
// 1. Householder tridiagonalisation (full storage, one workgroup).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kTriThreads)
    tridiag_kernel(int m, const double *__restrict__ K, double *__restrict__ work,
                   const EigJob *__restrict__ jobs) {
  if (jobs) m = jobs[blockIdx.y].m, K = jobs[blockIdx.y].K, work = jobs[blockIdx.y].work;
  extern __shared__ double sh[];
  EigLayout Lw(m);
  double *Aw = work + Lw.Aw, *Hv = work + Lw.Hv, *dg = work + Lw.d, *eg = work + Lw.e;
  double *vs = sh, *ps = sh + m, *part = sh + 2 * m;
  __shared__ double red[16];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (size_t idx = tid; idx < (size_t)m * m; idx += nt) {
    Aw[idx] = K[idx];
    Hv[idx] = 0.0;
  }
  __syncthreads();
  for (int k = 0; k + 2 < m; ++k) {
    const int R = m - k - 1;
    double part_s = 0.0;
    for (int i = tid; i < R; i += nt) {
      const double x = Aw[(size_t)k * m + k + 1 + i];
      vs[i] = x;
      part_s += x * x;
    }
    const double sig2 = wsum(part_s, red);
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
    const double vn = sqrt(2.0 * (sig2 - alpha * x0));
    if (tid == 0) vs[0] = x0 - alpha;
    __syncthreads();
    for (int i = tid; i < R; i += nt) {
      const double v = vs[i] / vn;
      vs[i] = v;
      Hv[(size_t)k * m + k + 1 + i] = v;
    }
    __syncthreads();
    // p = S v: thread groups split the column range of each row
    const int groups = max(1, nt / R);
    if (R <= nt) {
      const int i = tid % R, g = tid / R;
      double acc = 0.0;
      if (g < groups)
        for (int j = g; j < R; j += groups)
          acc += Aw[(size_t)(k + 1 + j) * m + (k + 1 + i)] * vs[j];
      if (tid < R * groups) part[tid] = acc;
      __syncthreads();
      for (int ii = tid; ii < R; ii += nt) {
        double s = 0.0;
        for (int gg = 0; gg < groups; ++gg) s += part[gg * R + ii];
        ps[ii] = s;
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
    const double Kv = wsum(kp, red);
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
}

// Grid variant, for m beyond the register tiles: a persistent grid of kTriGridWG workgroups
// and two grid-wide barriers per step. Workgroup g owns a contiguous block of columns of
// the symmetric working matrix (full storage in Aw) for the rank-2 updates and a contiguous
// block of the trailing rows for the product p = S v. Step k:
//   every workgroup forms the reflector v of column k itself (the same data and the same
//   reduction order everywhere, so all hold the same v); workgroup 0 stores it;
//   p = S v by row blocks (reads of S coalesced along its columns) and the block's share
//   of v^T p into a per-workgroup slot;                                   -- barrier
//   w = p - (v^T p) v with v^T p summed over the slots in order, and the rank-2 update
//   S -= 2 (v w^T + w v^T) of the owned columns;                          -- barrier
// A barrier is a release fence and an arrival on a counter (cleared before the launch), then
// acquire polls until every workgroup of this barrier has arrived; the polls are bounded, and
// a workgroup that gives up raises an abort word the others see and the eigen-solver's flag.
constexpr int kTriGridWG = 64;
constexpr int kTriGridThreads = 256;
constexpr int kTriGridMaxPolls = 1 << 22;

__device__ bool grid_barrier(int *ctr, int *abort_w, int target, int *ok_lds) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    int polls = 0, ok = 1;
    while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(abort_w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
          ++polls > kTriGridMaxPolls) {
        __hip_atomic_store(abort_w, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    *ok_lds = ok;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return *ok_lds != 0;
}

__global__ void __launch_bounds__(kTriGridThreads)
    tridiag_grid_kernel(int m, const double *__restrict__ K, double *__restrict__ work,
                        int *__restrict__ gsync, int *__restrict__ flag) {
  EigLayout Lw(m);
  double *Aw = work + Lw.Aw, *Hv = work + Lw.Hv, *dg = work + Lw.d, *eg = work + Lw.e;
  double *pg = work + Lw.scr, *partg = pg + m;  // p, and the per-workgroup shares of v^T p
  int *const ctr = gsync, *const abort_w = gsync + 1;
  __shared__ double vs[kEigMaxM];
  __shared__ double red[16];
  __shared__ double psum[kTriGridThreads];
  __shared__ int ok;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int G = gridDim.x, g = blockIdx.x;
  const int cper = (m + G - 1) / G, clo = min(m, g * cper), chi = min(m, clo + cper);
  int nbar = 0;
  // copy of K (owned columns) and cleared reflector columns
  for (int j = clo; j < chi; ++j)
    for (int i = tid; i < m; i += nt) {
      Aw[(size_t)j * m + i] = K[(size_t)j * m + i];
      Hv[(size_t)j * m + i] = 0.0;
    }
  if (!grid_barrier(ctr, abort_w, ++nbar * G, &ok)) {
    if (tid == 0) flag[0] = 1;
    return;
  }
  for (int k = 0; k + 2 < m; ++k) {
    const int R = m - k - 1, r0 = k + 1;
    // reflector of column k, in every workgroup
    double part = 0.0;
    for (int i = tid; i < R; i += nt) {
      const double x = Aw[(size_t)k * m + r0 + i];
      vs[i] = x;
      part += x * x;
    }
    const double sig2 = wsum(part, red);
    const double sig = sqrt(sig2);
    const double x0 = vs[0];
    __syncthreads();
    if (sig == 0.0) {  // column already reduced: no reflector, S unchanged
      if (g == 0 && tid == 0) {
        dg[k] = Aw[(size_t)k * m + k];
        eg[k] = 0.0;
      }
      continue;
    }
    const double alpha = (x0 >= 0.0) ? -sig : sig;
    const double vn = sqrt(2.0 * (sig2 - alpha * x0));
    if (tid == 0) vs[0] = x0 - alpha;
    __syncthreads();
    for (int i = tid; i < R; i += nt) {
      const double v = vs[i] / vn;
      vs[i] = v;
      if (g == 0) Hv[(size_t)k * m + r0 + i] = v;
    }
    if (g == 0 && tid == 0) {
      dg[k] = Aw[(size_t)k * m + k];
      eg[k] = alpha;
    }
    __syncthreads();
    // p = S v for this workgroup's rows: thread (row, column group), groups summed in order
    const int rper = (R + G - 1) / G, rlo = min(R, g * rper), nr = min(R, rlo + rper) - rlo;
    double vp = 0.0;
    if (nr > 0) {
      const int ngrp = max(1, nt / nr), ri = tid % nr, cg = tid / nr;
      double acc = 0.0;
      if (cg < ngrp)
        for (int j = cg; j < R; j += ngrp) acc += Aw[(size_t)(r0 + j) * m + r0 + rlo + ri] * vs[j];
      psum[tid] = (cg < ngrp) ? acc : 0.0;
      __syncthreads();
      if (tid < nr) {
        double sacc = 0.0;
        for (int c = 0; c < ngrp; ++c) sacc += psum[c * nr + tid];
        pg[r0 + rlo + tid] = sacc;
        vp = sacc * vs[rlo + tid];
      }
    }
    const double vps = wsum(vp, red);
    if (tid == 0) partg[g] = vps;
    if (!grid_barrier(ctr, abort_w, ++nbar * G, &ok)) break;
    // w = p - (v^T p) v, and the rank-2 update of the owned columns within the trailing block
    double Kv = 0.0;
    for (int q = 0; q < G; ++q) Kv += partg[q];
    const int jlo = max(clo, r0);
    for (int j = jlo; j < chi; ++j) {
      const double vj = vs[j - r0];
      const double wj = pg[j] - Kv * vj;
      for (int i = tid; i < R; i += nt) {
        const double vi = vs[i];
        const double wi = pg[r0 + i] - Kv * vi;
        Aw[(size_t)j * m + r0 + i] -= 2.0 * (vi * wj + wi * vj);
      }
    }
    if (!grid_barrier(ctr, abort_w, ++nbar * G, &ok)) break;
  }
  if (__hip_atomic_load(abort_w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
    if (tid == 0) flag[0] = 1;
    return;
  }
  if (g == 0 && tid == 0) {
    if (m >= 2) {
      dg[m - 2] = Aw[(size_t)(m - 2) * m + m - 2];
      dg[m - 1] = Aw[(size_t)(m - 1) * m + m - 1];
      eg[m - 2] = Aw[(size_t)(m - 2) * m + m - 1];
    } else {
      dg[0] = Aw[0];
    }
    eg[m - 1] = 0.0;
  }
}

// Register-tile variant. The lower triangle of K is cut into 9 x 9 tiles (R, C), R >= C, one
// tile per lane (81 FP64 registers); diagonal tiles hold the full symmetric block. Lanes are
// ordered by tile column, then tile row, so whole waves fall idle as the reduction moves
// right. Every sum is taken in a fixed order (no atomics), so the result
// is the same bit for bit on every run. Step k of the reduction is three phases and three
// barriers:
//   phase 1  apply the pending rank-2 update of step k-1, with w = p - (v^T p) v formed per lane
//            from v and p of step k-1, and gather column k and the partial |x|^2; the block
//            stores reflector k-1 to global memory;
//   phase 2  every lane forms the Householder scalars from |x|^2 (the column-block tiles' parts,
//            one slot per tile row, summed in order) and x_{k+1} and its own slices of v (rows
//            and columns of its tile), and writes its tile's share of p = A v (row sums and, off
//            the diagonal, column sums) into the slot of its partner block; each wave reduces
//            its lanes' shares of v^T A v by a fixed shuffle tree; the diagonal lanes store v;
//   phase 3  p[i] = the sum of its slots over the active partner blocks, in a fixed order.
// v, p and v^T p are double-buffered by step parity.
// Sum over the wave, returned to every lane (the same value, bit for bit, in every wave for the
// same inputs): DPP adds within each row of 16 lanes (quad_perm [1,0,3,2] and [2,3,0,1],
// half-row mirror, row mirror), then row_bcast:15 and row_bcast:31 carry the row sums up to
// lane 63, read back by v_readlane. No LDS traffic, unlike a ds_bpermute tree.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_add_src(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_add_src<0xB1, 0xf>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_add_src<0x4E, 0xf>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_add_src<0x141, 0xf>(v);  // row_half_mirror
  v += dpp_add_src<0x140, 0xf>(v);  // row_mirror
  v += dpp_add_src<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_add_src<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(b & 0xffffffffLL), 63);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));

constexpr int kTB = 9;
constexpr int kTileMaxNb = 31;  // m <= 279
constexpr int kTileMaxThreads = 512;

__host__ __device__ inline int tile_nb(int m) { return (m + kTB - 1) / kTB; }
__host__ inline int tile_threads(int m) {
  const int nb = tile_nb(m);
  return (nb * (nb + 1) / 2 + 63) / 64 * 64;
}
__host__ inline bool tile_fits(int m) { return m >= 3 && tile_nb(m) <= kTileMaxNb; }

template <int S>
__device__ __forceinline__ double tile_gather(const double (&a)[kTB][kTB], int r0, int k,
                                              double *xs) {
  const int kr = k - r0;
  double s2 = 0.0;
#pragma unroll
  for (int t = 0; t < kTB; ++t) {
    if (t >= kr) xs[r0 + t] = a[t][S];
    s2 = fma((t > kr) ? a[t][S] : 0.0, a[t][S], s2);
  }
  return s2;
}

// a -= v_r (2 w_c)^T + (2 w_r) v_c^T with w = p - kp v on indices >= k (v is already zero
// below; p is masked here). Offsets within the tile are compared with k - r0 and k - c0, so
// no per-row index stays live, and the loads are unconditional.
__device__ __forceinline__ void tile_update(double (&a)[kTB][kTB], const double *vv,
                                            const double *pp, double kp, int r0, int c0, int k) {
  const int kr = k - r0, kc = k - c0;
  double vc[kTB], wc[kTB];
#pragma unroll
  for (int s = 0; s < kTB; ++s) {
    vc[s] = vv[c0 + s];
    const double w = 2.0 * (pp[c0 + s] - kp * vc[s]);
    wc[s] = (s >= kc) ? w : 0.0;
  }
  double v = vv[r0], p = pp[r0];
#pragma unroll
  for (int t = 0; t < kTB; ++t) {
    // the next row's v and p are in flight while this row updates; one row ahead only, since
    // hoisting all of them would spill the tile
    const int tn = t + 1 < kTB ? t + 1 : t;
    const double vn = vv[r0 + tn], pn = pp[r0 + tn];
    const double w = 2.0 * (p - kp * v);
    const double wr = (t >= kr) ? w : 0.0;
#pragma unroll
    for (int s = 0; s < kTB; ++s) a[t][s] = fma(-v, wc[s], fma(-wr, vc[s], a[t][s]));
    __builtin_amdgcn_sched_barrier(0);
    v = vn;
    p = pn;
  }
}

// column k - c0 of the tile into xs (rows >= k); returns the tile's part of |x|^2 below row k
__device__ __forceinline__ double tile_gather_col(const double (&a)[kTB][kTB], int r0, int c0,
                                                  int k, double *xs) {
  switch (k - c0) {
    case 0: return tile_gather<0>(a, r0, k, xs);
    case 1: return tile_gather<1>(a, r0, k, xs);
    case 2: return tile_gather<2>(a, r0, k, xs);
    case 3: return tile_gather<3>(a, r0, k, xs);
    case 4: return tile_gather<4>(a, r0, k, xs);
    case 5: return tile_gather<5>(a, r0, k, xs);
    case 6: return tile_gather<6>(a, r0, k, xs);
    case 7: return tile_gather<7>(a, r0, k, xs);
    default: return tile_gather<8>(a, r0, k, xs);
  }
}

// v^T A v: one partial per wave, summed in wave order where it is used
constexpr int kKpWaves = kTileMaxThreads / 64;
__device__ __forceinline__ double kp_sum(const double *kw) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kKpWaves; ++i) s += kw[i];
  return s;
}
// p's partial sums: slot [partner block][entry], rows of 281 doubles (odd, so the lanes of a
// wave, one tile column and consecutive tile rows, write their column sums to distinct banks)
constexpr int kPslotLd = kTB * kTileMaxNb + 2;

__global__ void __launch_bounds__(kTileMaxThreads)
    tridiag_tile_kernel(int m, const double *__restrict__ K, double *__restrict__ work,
                        const EigJob *__restrict__ jobs) {
  if (jobs) m = jobs[blockIdx.y].m, K = jobs[blockIdx.y].K, work = jobs[blockIdx.y].work;
  __shared__ double vb[2][kTB * kTileMaxNb], pb[2][kTB * kTileMaxNb];
  __shared__ double xs[kTB * kTileMaxNb];
  __shared__ double s2s[kTileMaxNb];             // |x|^2 parts of the column block's tiles
  __shared__ double kpw[2][kKpWaves];            // v^T A v parts, one per wave
  __shared__ double pslot[kTileMaxNb * kPslotLd];  // p's parts, one per (partner block, entry)
  EigLayout Lw(m);
  gmem<double> *Hv = gptr(work + Lw.Hv), *dg = gptr(work + Lw.d), *eg = gptr(work + Lw.e);
  const int tid = threadIdx.x, nt = blockDim.x;
  const int nb = tile_nb(m), mp = nb * kTB;
  // lane -> tile by tile column, then row: the tiles of the left columns, which the
  // reduction leaves first, fill the first waves, so whole waves fall idle as it proceeds
  // and the waves still working get their SIMDs to themselves
  int C = 0, R = tid;
  while (C < nb && R >= nb - C) R -= nb - (C++);
  const bool own = C < nb;
  if (!own) C = 0, R = 0;
  R += C;
  const int d = R - C;
  const int r0 = R * kTB, c0 = C * kTB;
  const bool diag = d == 0;
  double a[kTB][kTB];
#pragma unroll
  for (int t = 0; t < kTB; ++t)
#pragma unroll
    for (int s = 0; s < kTB; ++s) {
      const int i = r0 + t, j = c0 + s;
      a[t][s] = (own && i < m && j < m) ? gptr(K)[(size_t)min(i, j) * m + max(i, j)] : 0.0;
    }
  for (int i = tid; i < mp; i += nt) {
    vb[0][i] = vb[1][i] = 0.0;
    pb[0][i] = pb[1][i] = 0.0;
    xs[i] = 0.0;
  }
  if (tid < 2 * kKpWaves) kpw[tid / kKpWaves][tid % kKpWaves] = 0.0;
  for (int i = tid; i < kTileMaxNb * kPslotLd; i += nt) pslot[i] = 0.0;
  for (size_t idx = tid; idx < (size_t)m * m; idx += nt) Hv[idx] = 0.0;
  __syncthreads();
  for (int k = 0; k + 2 < m; ++k) {
    const int cur = k & 1, prv = cur ^ 1;
    const int cb = k / kTB;
    // phase 1
    if (own && c0 + kTB > k) {
      if (k > 0) tile_update(a, vb[prv], pb[prv], kp_sum(kpw[prv]), r0, c0, k);
      if (C == cb) s2s[C + d] = tile_gather_col(a, r0, c0, k, xs);
    }
    for (int i = tid; i < mp; i += nt) {
      if (k > 0 && i >= k && i < m) Hv[(size_t)(k - 1) * m + i] = vb[prv][i];
      vb[cur][i] = 0.0;
    }
    __syncthreads();
    // phase 2
    // |x|^2: the column block's slots summed by each wave's fixed DPP tree (the same value,
    // bit for bit, in every wave)
    const double s2 = wave_sum_dpp((cb + (tid & 63) < nb) ? s2s[cb + (tid & 63)] : 0.0);
    const double x0 = xs[k + 1];
    // |x| = s2 / sqrt(s2) and 1 / |v| by reciprocal square roots: a short dependent chain
    const double sig = (s2 > 0.0) ? s2 * rsqrt(s2) : 0.0;
    const double alpha = (x0 >= 0.0) ? -sig : sig;
    const double rvn = (sig != 0.0) ? rsqrt(2.0 * (s2 - alpha * x0)) : 0.0;
    if (tid == 0) {
      dg[k] = xs[k];
      eg[k] = (sig != 0.0) ? alpha : 0.0;
    }
    double kpart = 0.0;
    if (own && c0 + kTB - 1 > k) {
      // v on the tile's rows and columns, then the row sums, then the column sums; the fences
      // keep one stage's work from being hoisted into the previous one
      const int kr = k - r0, kc = k - c0;
      const double h = x0 - alpha;
      double vr[kTB], vc[kTB];
#pragma unroll
      for (int s = 0; s < kTB; ++s) {
        const double xv = (s == kc + 1) ? h : xs[c0 + s];
        vc[s] = (s > kc) ? xv * rvn : 0.0;
      }
#pragma unroll
      for (int t = 0; t < kTB; ++t) {
        const double xv = (t == kr + 1) ? h : xs[r0 + t];
        vr[t] = (t > kr) ? xv * rvn : 0.0;
      }
      __builtin_amdgcn_sched_barrier(0);
      // row sums two rows at a time (two independent FMA chains)
#pragma unroll
      for (int t = 0; t < kTB; t += 2) {
        double rp0 = 0.0, rp1 = 0.0;
#pragma unroll
        for (int s = 0; s < kTB; ++s) {
          rp0 = fma(a[t][s], vc[s], rp0);
          if (t + 1 < kTB) rp1 = fma(a[t + 1][s], vc[s], rp1);
        }
        if (t > kr) pslot[C * kPslotLd + r0 + t] = rp0;
        kpart = fma(vr[t], rp0, kpart);
        if (t + 1 < kTB) {
          if (t + 1 > kr) pslot[C * kPslotLd + r0 + t + 1] = rp1;
          kpart = fma(vr[t + 1], rp1, kpart);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      if (diag) {
#pragma unroll
        for (int t = 0; t < kTB; ++t) {
          if (t > kr) vb[cur][r0 + t] = vr[t];
        }
      } else {
        kpart *= 2.0;
#pragma unroll
        for (int s = 0; s < kTB; s += 2) {
          double cp0 = 0.0, cp1 = 0.0;
#pragma unroll
          for (int t = 0; t < kTB; ++t) {
            cp0 = fma(a[t][s], vr[t], cp0);
            if (s + 1 < kTB) cp1 = fma(a[t][s + 1], vr[t], cp1);
          }
          if (s > kc) pslot[(C + d) * kPslotLd + c0 + s] = cp0;
          if (s + 1 < kTB && s + 1 > kc) pslot[(C + d) * kPslotLd + c0 + s + 1] = cp1;
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    // the wave's share of v^T A v by the fixed DPP tree
    kpart = wave_sum_dpp(kpart);
    if ((tid & 63) == 0) kpw[cur][tid >> 6] = kpart;
    __syncthreads();
    // phase 3: p on the rows below k from the slots of the active partner blocks (tiles whose
    // columns all lie at or left of k took no part); batches of eight loads in flight, four
    // running sums combined in a fixed order
    {
      const int cba = (k + 1) / kTB;
      for (int i = tid; i < mp; i += nt) {
        double pv = 0.0;
        if (i > k && i < m) {
          const double *ps = pslot + i;
          double acc[4] = {0.0, 0.0, 0.0, 0.0};
          for (int j0 = cba; j0 < nb; j0 += 8) {
            double v8[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v8[u] = ps[min(j0 + u, kTileMaxNb - 1) * kPslotLd];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[u & 3] += (j0 + u < nb) ? v8[u] : 0.0;
          }
          pv = (acc[0] + acc[1]) + (acc[2] + acc[3]);
        }
        pb[cur][i] = pv;
      }
    }
    __syncthreads();
  }
  // pending update of step m - 3, then the trailing 2 x 2 block, one column at a time
  const int k = m - 2;
  if (own && c0 + kTB > k) {
    tile_update(a, vb[(k - 1) & 1], pb[(k - 1) & 1], kp_sum(kpw[(k - 1) & 1]), r0, c0, k);
    if (C == k / kTB) tile_gather_col(a, r0, c0, k, xs);
  }
  for (int i = tid; i < m; i += nt)
    if (i >= k) Hv[(size_t)(k - 1) * m + i] = vb[(k - 1) & 1][i];
  __syncthreads();
  if (tid == 0) {
    dg[k] = xs[k];
    eg[k] = xs[k + 1];
  }
  __syncthreads();
  if (own && C == (k + 1) / kTB) tile_gather_col(a, r0, c0, k + 1, xs);
  __syncthreads();
  if (tid == 0) {
    dg[k + 1] = xs[k + 1];
    eg[k + 1] = 0.0;
  }
}

// Quotient a / b through the hardware reciprocal and two Newton steps (about one ulp): a shorter
// dependent chain than the correctly rounded division. Used only where the sign pattern of a
// recurrence matters (Sturm and negative counts), not its last bit.
__device__ __forceinline__ double quot_nr(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(r, fma(-b, r, 1.0), r);
  r = fma(r, fma(-b, r, 1.0), r);
  return a * r;
}

// Sturm count of T - x I (number of eigenvalues below x).
__device__ int sturm_count(int m, const double *d, const double *e, double x, double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0) ++c;
  for (int i = 1; i < m; ++i) {
    q = d[i] - x - quot_nr(e[i - 1] * e[i - 1], q);
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++c;
  }
  return c;
}

// Negative count of L D L^T - tau I (stationary qd transform).
__device__ int negcount(int m, const double *D, const double *LLD, double tau, double pivmin) {
  int c = 0;
  double s = -tau;
  for (int i = 0; i < m - 1; ++i) {
    double dp = D[i] + s;
    if (fabs(dp) < pivmin) dp = -pivmin;
    if (dp < 0) ++c;
    s = LLD[i] * quot_nr(s, dp) - tau;
  }
  double dp = D[m - 1] + s;
  if (fabs(dp) < pivmin) dp = -pivmin;
  if (dp < 0) ++c;
  return c;
}

// ---------------------------------------------------------------------------
// 2. Root representation (one workgroup of 64 threads).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) root_kernel(int m, double *__restrict__ work,
                                                  int *__restrict__ flag,
                                                  const EigJob *__restrict__ jobs) {
  if (jobs) m = jobs[blockIdx.y].m, work = jobs[blockIdx.y].work, flag = jobs[blockIdx.y].flag;
  EigLayout Lw(m);
  extern __shared__ double rsh[];
  double *dg = rsh, *eg = rsh + m, *Dl = rsh + 2 * m, *Ll = rsh + 3 * m;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    dg[i] = work[Lw.d + i];
    eg[i] = work[Lw.e + i];
  }
  __syncthreads();
  gmem<double> *D = gptr(work + Lw.D);
  gmem<double> *Ls = gptr(work + Lw.Ls);
  gmem<double> *LLD = gptr(work + Lw.LLD);
  gmem<double> *misc = gptr(work + Lw.misc);
  __shared__ double sh_lo, sh_hi, sh_sigma;
  __shared__ int sh_ok;
  __shared__ int sh_first[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // Gershgorin bounds and the norm
  if (tid == 0) {
    double gl = dg[0], gu = dg[0], tn = 0.0;
    for (int i = 0; i < m; ++i) {
      const double r = (i > 0 ? fabs(eg[i - 1]) : 0.0) + (i < m - 1 ? fabs(eg[i]) : 0.0);
      gl = fmin(gl, dg[i] - r);
      gu = fmax(gu, dg[i] + r);
    }
    tn = fmax(fabs(gl), fabs(gu));
    sh_lo = gl - 2.0 * 0x1.0p-52 * tn - 1e-300;
    sh_hi = gu + 2.0 * 0x1.0p-52 * tn + 1e-300;
    misc[0] = tn;
    misc[1] = gl;
    misc[2] = gu;
  }
  __syncthreads();
  const double tn = misc[0];
  const double pivmin = 1e-290 * fmax(1.0, tn * tn);
  // smallest eigenvalue by 256-way multisection on Sturm counts (8 bits per round) until the
  // bracket is below eps * |T| or 2^-14 of its lower end: the shift below takes a margin of at
  // least 1e-3 of that end (or 64 eps |T|), which a bracket 16 times narrower leaves intact
  for (int round = 0; round < 8; ++round) {
    const double lo = sh_lo, hi = sh_hi;
    // the same shared values in every thread
    if (hi - lo <= fmax(0x1.0p-52 * tn, 0x1.0p-14 * fabs(lo))) break;
    const double x = lo + (hi - lo) * (tid + 1) / 257.0;
    const int c = sturm_count(m, dg, eg, x, pivmin);
    // smallest point with at least one eigenvalue below it: first lane per wave, then the
    // first wave that has one
    const unsigned long long bal = __ballot(c >= 1);
    if (lane == 0) sh_first[wave] = bal ? __ffsll((long long)bal) - 1 : 64;
    __syncthreads();
    if (tid == 0) {
      int first = 256;
      for (int w = 0; w < 4; ++w)
        if (sh_first[w] < 64) {
          first = 64 * w + sh_first[w];
          break;
        }
      if (first == 256) {
        sh_lo = lo + (hi - lo) * 256.0 / 257.0;
      } else {
        sh_hi = lo + (hi - lo) * (first + 1) / 257.0;
        if (first > 0) sh_lo = lo + (hi - lo) * first / 257.0;
      }
    }
    __syncthreads();
  }
  // sigma below the spectrum; retry lower until L D L^T is positive definite
  if (tid == 0) {
    const double lmin = sh_lo;
    double margin = fmax(1e-3 * fabs(lmin), 64.0 * 0x1.0p-52 * tn) + 1e-300;
    bool ok = false;
    double sigma = lmin;
    for (int tries = 0; tries < 60 && !ok; ++tries) {
      sigma = lmin - margin;
      ok = true;
      double dprev = dg[0] - sigma;
      if (!(dprev > 0.0)) ok = false;
      Dl[0] = dprev;
      for (int i = 0; i < m - 1 && ok; ++i) {
        const double l = eg[i] / Dl[i];
        Ll[i] = l;
        const double dn = dg[i + 1] - sigma - l * eg[i];
        Dl[i + 1] = dn;
        if (!(dn > 0.0) || !isfinite(dn)) ok = false;
      }
      margin *= 2.0;
    }
    Ll[m - 1] = 0.0;
    misc[3] = sigma;
    sh_ok = ok ? 1 : 0;
    // upper bound of the shifted spectrum
    misc[4] = (sh_hi > sigma ? misc[2] - sigma : 1.0) * (1.0 + 1e-12) + 1e-300;
  }
  __syncthreads();
  for (int i = tid; i < m; i += blockDim.x) {
    D[i] = Dl[i];
    Ls[i] = Ll[i];
    LLD[i] = Ll[i] * Ll[i] * Dl[i];
  }
  if (tid == 0 && !sh_ok) flag[0] = 1;
}

// ---------------------------------------------------------------------------
// 3. Eigenvalues of L D L^T: one wave per eigenvalue index (ascending).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) bisect_kernel(int m, double *__restrict__ work,
                                                     const EigJob *__restrict__ jobs) {
  if (jobs) m = jobs[blockIdx.y].m, work = jobs[blockIdx.y].work;
  if ((int)blockIdx.x * (int)(blockDim.x >> 6) >= m) return;
  EigLayout Lw(m);
  extern __shared__ double bsh[];
  double *D = bsh, *LLD = bsh + m;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    D[i] = work[Lw.D + i];
    LLD[i] = work[Lw.LLD + i];
  }
  __syncthreads();
  const gmem<double> *misc = gptr(work + Lw.misc);
  gmem<double> *mu = gptr(work + Lw.mu);
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= m) return;
  const double tn = misc[0];
  const double pivmin = 1e-290 * fmax(1.0, tn * tn);
  double lo = 0.0, hi = misc[4];
  // geometric brackets: points hi * 2^-(lane+1); the eigenvalue index j is the (j+1)-th smallest
  for (int g = 0; g < 4; ++g) {
    const double x = hi * exp2(-(double)(lane + 1));
    const int c = negcount(m, D, LLD, x, pivmin);
    // largest lane k with count(x_k) >= j+1 gives hi = x_k; next lane gives lo
    const unsigned long long bal = __ballot(c >= j + 1);
    if (bal == 0ull) {  // eigenvalue above hi/2
      lo = hi * 0.5;
      break;
    }
    const int last = 63 - __clzll((long long)bal);
    const double xh = hi * exp2(-(double)(last + 1));
    if (last < 63) {
      lo = hi * exp2(-(double)(last + 2));
      hi = xh;
      break;
    }
    hi = xh;  // still below every geometric point: continue further down
  }
  // uniform 64-way multisection
  for (int round = 0; round < 10; ++round) {
    const double x = lo + (hi - lo) * (lane + 1) / 65.0;
    const int c = negcount(m, D, LLD, x, pivmin);
    const unsigned long long bal = __ballot(c >= j + 1);
    double nlo = lo, nhi = hi;
    if (bal == 0ull) {
      nlo = lo + (hi - lo) * 64.0 / 65.0;
    } else {
      const int first = __ffsll((long long)bal) - 1;
      nhi = lo + (hi - lo) * (first + 1) / 65.0;
      if (first > 0) nlo = lo + (hi - lo) * first / 65.0;
    }
    lo = nlo;
    hi = nhi;
    if (hi - lo <= 2.0 * 0x1.0p-53 * hi) break;
  }
  if (lane == 0) mu[j] = 0.5 * (lo + hi);
}

// ---------------------------------------------------------------------------
// 4. Eigenvectors by twisted factorisation, two waves per 64 eigenvalues: lane l of both
//    waves of a workgroup takes eigenvalue j = 64 blockIdx.x + l. Wave 0 runs the
//    stationary transform (top down) while wave 1 runs the progressive one (bottom up);
//    each wave scans half of the twist range and the two halves are combined through LDS
//    (the smaller |gamma|, the smaller index on ties); wave 0 builds the vector above the
//    twist and wave 1 below it. The per-eigenvalue arrays live in scratch laid out [i][j]
//    (coalesced in j); workgroup barriers order the exchanges. Every thread runs the three
//    Rayleigh-quotient passes' barriers; an eigenvalue that has converged skips the work.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(128) vector_kernel(int m, double *__restrict__ work,
                                                     const EigJob *__restrict__ jobs) {
  if (jobs) m = jobs[blockIdx.y].m, work = jobs[blockIdx.y].work;
  if ((int)(blockIdx.x * 64) >= m) return;
  EigLayout Lw(m);
  extern __shared__ double vsh[];
  double *D = vsh, *Ls = vsh + m, *LLD = vsh + 2 * m;
  __shared__ double xg[2][64], xn[2][64];
  __shared__ int xr[2][64];
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    D[i] = work[Lw.D + i];
    Ls[i] = work[Lw.Ls + i];
    LLD[i] = work[Lw.LLD + i];
  }
  __syncthreads();
  gmem<double> *mu = gptr(work + Lw.mu);
  gmem<double> *Z = gptr(work + Lw.Z);
  gmem<double> *Lp = gptr(work + Lw.scr);
  gmem<double> *Um = gptr(work + Lw.scr + (size_t)m * m);
  gmem<double> *sv = gptr(work + Lw.scr + 2 * (size_t)m * m);
  gmem<double> *pv = gptr(work + Lw.scr + 3 * (size_t)m * m);
  const int l = threadIdx.x & 63, role = threadIdx.x >> 6;  // role: wave-uniform
  const int j = blockIdx.x * 64 + l;
  const bool act = j < m;
  const double tiny = 1e-300;
  double lam = act ? mu[j] : 0.0;
  int r = 0;
  double nrm2 = 1.0;
  bool done = !act;
  for (int it = 0; it < 3; ++it) {
    if (!done) {
      if (role == 0) {
        // stationary: L D L^T - lam I = L+ D+ L+^T
        double s = -lam;
        for (int i = 0; i < m - 1; ++i) {
          sv[(size_t)i * m + j] = s;
          double dp = D[i] + s;
          if (fabs(dp) < tiny) dp = -tiny;
          const double lp = D[i] * Ls[i] / dp;
          Lp[(size_t)i * m + j] = lp;
          s = lp * Ls[i] * s - lam;
        }
        sv[(size_t)(m - 1) * m + j] = s;
      } else {
        // progressive: L D L^T - lam I = U- D- U-^T
        double p = D[m - 1] - lam;
        pv[(size_t)(m - 1) * m + j] = p;
        for (int i = m - 2; i >= 0; --i) {
          double dm = LLD[i] + p;
          if (fabs(dm) < tiny) dm = -tiny;
          const double t = D[i] / dm;
          Um[(size_t)i * m + j] = Ls[i] * t;
          p = p * t - lam;
          pv[(size_t)i * m + j] = p;
        }
      }
    }
    __syncthreads();
    // twist index: r minimises |gamma_k| = |s_k + p_k + lam| (the smallest k on ties); wave 0
    // scans the lower half of the range
    if (!done) {
      const int h = m / 2, k0 = role ? h : 0, k1 = role ? m : h;
      double gmin = 0.0;
      int rl = -1;
      // chunks of kTw rows, the next chunk's loads in flight while one is scanned (rows
      // past the range read its last row and are skipped)
      constexpr int kTw = 8;
      double sa[kTw], pa[kTw], sb[kTw], pb[kTw];
      auto ld = [&](int kb, double (&s_)[kTw], double (&p_)[kTw]) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < kTw; ++u) {
          const int k = min(kb + u, k1 - 1);
          s_[u] = sv[(size_t)k * m + j];
          p_[u] = pv[(size_t)k * m + j];
        }
      };
      auto scan = [&](int kb, const double (&s_)[kTw], const double (&p_)[kTw])
          __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < kTw; ++u) {
          const double gk = s_[u] + p_[u] + lam;
          const bool take = kb + u < k1 && (rl < 0 || fabs(gk) < fabs(gmin));
          gmin = take ? gk : gmin;
          rl = take ? kb + u : rl;
        }
      };
      ld(k0, sa, pa);
      for (int kb = k0; kb < k1; kb += 2 * kTw) {
        ld(kb + kTw, sb, pb);
        scan(kb, sa, pa);
        ld(kb + 2 * kTw, sa, pa);
        scan(kb + kTw, sb, pb);
      }
      xg[role][l] = gmin;
      xr[role][l] = rl;
    }
    __syncthreads();
    double gmin = 0.0;
    if (!done) {
      const bool take_low = xr[0][l] >= 0 && (xr[1][l] < 0 || fabs(xg[0][l]) <= fabs(xg[1][l]));
      gmin = take_low ? xg[0][l] : xg[1][l];
      r = take_low ? xr[0][l] : xr[1][l];
      // vector with z_r = 1: wave 0 builds z_i for i < r, wave 1 for i > r
      // chunks of kBd rows with the next chunk's factors in flight; the stores go through a
      // buffer resource over Z, rows outside the vector's part at an offset past its end
      // (dropped), so no branch separates a chunk's loads from the previous chunk's stores
      constexpr int kBd = 8;
      const __amdgpu_buffer_rsrc_t zres = __builtin_amdgcn_make_buffer_rsrc(
          (void *)Z, (short)0, (int)((size_t)m * m * sizeof(double)), 0x00020000);
      const int zcol = j * m;
      auto zstore = [&](bool valid, int row, double v) __attribute__((always_inline)) {
        u32x2_t bits;
        __builtin_memcpy(&bits, &v, sizeof(bits));
        __builtin_amdgcn_raw_buffer_store_b64(
            bits, zres, valid ? (zcol + row) * (int)sizeof(double) : 0x7ffffff8, 0, 0);
      };
      double part, cur[kBd], nxt[kBd];
      if (role == 0) {
        Z[(size_t)j * m + r] = 1.0;
        part = 1.0;
        double z = 1.0;
        // rows r - 1 down to 0: L+ factors Lp[i]
#pragma unroll
        for (int u = 0; u < kBd; ++u) cur[u] = Lp[(size_t)max(r - 1 - u, 0) * m + j];
        for (int base = r - 1; base >= 0; base -= kBd) {
#pragma unroll
          for (int u = 0; u < kBd; ++u) nxt[u] = Lp[(size_t)max(base - kBd - u, 0) * m + j];
#pragma unroll
          for (int u = 0; u < kBd; ++u) {
            const int i = base - u;
            const bool valid = i >= 0;
            const double zn = -cur[u] * z;
            z = valid ? zn : z;
            part = valid ? part + zn * zn : part;
            zstore(valid, i, zn);
          }
#pragma unroll
          for (int u = 0; u < kBd; ++u) cur[u] = nxt[u];
        }
      } else {
        part = 0.0;
        double z = 1.0;
        // rows r + 1 up to m - 1: U- factors Um[i], i = r .. m - 2
#pragma unroll
        for (int u = 0; u < kBd; ++u) cur[u] = Um[(size_t)min(r + u, m - 2) * m + j];
        for (int base = r; base < m - 1; base += kBd) {
#pragma unroll
          for (int u = 0; u < kBd; ++u) nxt[u] = Um[(size_t)min(base + kBd + u, m - 2) * m + j];
#pragma unroll
          for (int u = 0; u < kBd; ++u) {
            const int i = base + u;
            const bool valid = i < m - 1;
            const double zn = -cur[u] * z;
            z = valid ? zn : z;
            part = valid ? part + zn * zn : part;
            zstore(valid, i + 1, zn);
          }
#pragma unroll
          for (int u = 0; u < kBd; ++u) cur[u] = nxt[u];
        }
      }
      xn[role][l] = part;
    }
    __syncthreads();
    if (!done) {
      nrm2 = xn[0][l] + xn[1][l];
      // Rayleigh-quotient correction of lam (gamma_r / ||z||^2), the same in both waves; a
      // correction within a few units of rounding of lam (the bisection's own tolerance) is
      // rounding noise, and another pass would not change the vector
      const double corr = gmin / nrm2;
      if (!(fabs(corr) > 8.0 * 0x1.0p-53 * fabs(lam)))
        done = true;
      else
        lam += corr;
    }
    __syncthreads();  // the exchange buffers are reused by the next pass
  }
  if (!act) return;
  const double inv = 1.0 / sqrt(nrm2);
  if (role == 0) {
#pragma unroll 8
    for (int i = 0; i <= r; ++i) Z[(size_t)j * m + i] *= inv;
    mu[j] = lam;
  } else {
#pragma unroll 8
    for (int i = r + 1; i < m; ++i) Z[(size_t)j * m + i] *= inv;
  }
}

// ---------------------------------------------------------------------------
// 5. Clusters (relative gap < 1e-3): Gram-Schmidt and Rayleigh-Ritz (one workgroup per cluster).
// ---------------------------------------------------------------------------
constexpr int kMaxCluster = 48;

// Cluster list: where the relative gap between neighbouring mu is below 1e-3, at most
// kMaxCluster per cluster; the neighbour gaps of the vector step's mu are tested in
// parallel, then scanned in order by one thread. A longer run is cut into a chain of
// clusters, each after the first marked as continuing the one before (it may then be a
// single index). list[0] = number of clusters;
// list[1 + 3 g .. 3 + 3 g] = first index, last index, continuation flag of cluster g. The
// list sits after the m x m part of the scratch that the cluster kernel uses for T Z_c.
__global__ void __launch_bounds__(64) cluster_scan_kernel(int m, double *__restrict__ work,
                                                          const EigJob *__restrict__ jobs) {
  if (jobs) m = jobs[blockIdx.y].m, work = jobs[blockIdx.y].work;
  EigLayout Lw(m);
  // the gap tests in parallel (one flag per neighbour pair), then the scan by one thread
  __shared__ unsigned char cl[kEigMaxM];
  const gmem<double> *mu = gptr(work + Lw.mu);
  for (int i = threadIdx.x; i + 1 < m; i += blockDim.x) {
    const double a = mu[i], b = mu[i + 1];
    cl[i] = fabs(b - a) < 1e-3 * fmax(fabs(b), fabs(a)) ? 1 : 0;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  gmem<int> *list = gptr(reinterpret_cast<int *>(work + Lw.scr + (size_t)m * m));
  auto close = [&](int i) { return cl[i] != 0; };
  int cnt = 0, a = 0;
  bool cont = false;
  while (a < m) {
    int s0 = a;
    if (!cont)
      while (s0 + 1 < m && !close(s0)) ++s0;
    int e = s0;
    while (e + 1 < m && e + 1 - s0 < kMaxCluster && close(e)) ++e;
    if (e > s0 || cont) {
      list[1 + 3 * cnt] = s0;
      list[2 + 3 * cnt] = e;
      list[3 + 3 * cnt] = cont ? 1 : 0;
      ++cnt;
    }
    cont = e + 1 < m && close(e);  // the cap cut a run: the next cluster continues it
    a = e + 1;
  }
  list[0] = cnt;
}

// Sum over the wave (all lanes get it).
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One workgroup per chain of clusters (chains are disjoint column sets), its clusters
// Z_c = Z[:, a..b] in order: the vectors are re-orthonormalised against every earlier vector
// of the chain and of the cluster (classical Gram-Schmidt twice, the dot products of one
// vector with all earlier ones spread over the waves; a vector that collapses is replaced by
// a probe), then rotated by the eigenvectors of H = Z_c^T T Z_c, found by Jacobi with the
// round-robin parallel ordering (the rotations of one round act on disjoint index pairs).
__global__ void __launch_bounds__(256) cluster_kernel(int m, double *__restrict__ work,
                                                      int *__restrict__ flag,
                                                      const EigJob *__restrict__ jobs) {
  if (jobs) m = jobs[blockIdx.y].m, work = jobs[blockIdx.y].work, flag = jobs[blockIdx.y].flag;
  EigLayout Lw(m);
  const int *list = reinterpret_cast<const int *>(work + Lw.scr + (size_t)m * m);
  const int g = blockIdx.x;
  const int ncl = list[0];
  if (g >= ncl || list[3 + 3 * g]) return;  // not a cluster, or inside a chain
  const int c0 = list[1 + 3 * g];           // the chain's first index
  const gmem<double> *dg = gptr(work + Lw.d);
  const gmem<double> *eg = gptr(work + Lw.e);
  const gmem<double> *misc = gptr(work + Lw.misc);
  gmem<double> *mu = gptr(work + Lw.mu);
  gmem<double> *Z = gptr(work + Lw.Z);
  __shared__ double H[kMaxCluster][kMaxCluster + 1];
  __shared__ double Vc[kMaxCluster][kMaxCluster + 1];
  __shared__ double dots[kEigMaxM];
  __shared__ double Cb[kMaxCluster * 65];  // P^T Z_c for a chunk of 64 earlier vectors
  __shared__ double rot[kMaxCluster / 2][2];
  __shared__ int pr[kMaxCluster / 2][2];
  __shared__ double red[16];
  __shared__ int done;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6;
  const int nw = nt >> 6;
  const double sigma = misc[3];
  for (int cl = g; cl < ncl && (cl == g || list[3 + 3 * cl]); ++cl) {
  const int a = list[1 + 3 * cl], c = list[2 + 3 * cl] - a + 1;
  gmem<double> *W = gptr(work + Lw.scr + (size_t)a * m);  // m x c, this cluster's columns of the scratch
  // 1a. against the chain's earlier clusters (columns c0 .. a - 1, orthonormal already), as
  //     blocks: twice Z_c <- Z_c - P (P^T Z_c) for chunks P of 64 columns, on the matrix cores
  for (int pass = 0; pass < 2 && a > c0; ++pass) {
    for (int p0 = c0; p0 < a; p0 += 64) {
      const int pc = min(64, a - p0);
      {  // Cb = P^T Z_c (pc x c, column-major, leading dimension 65), a 32 x 32 tile per wave
        const int rt = wave >> 1, ct = wave & 1, li = lane & 15, lg = lane >> 4;
        if (32 * rt < pc && 32 * ct < c) {
          d4 acc[2][2];
          zero_acc(acc);
          wave_mma32<true, false>(Z + (size_t)(p0 + 32 * rt) * m, m, Z + (size_t)(a + 32 * ct) * m,
                                  m, m, pc - 32 * rt, c - 32 * ct, acc);
#pragma unroll
          for (int r2 = 0; r2 < 2; ++r2)
#pragma unroll
            for (int c2 = 0; c2 < 2; ++c2)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int row = 32 * rt + 16 * r2 + lg + 4 * r, col = 32 * ct + 16 * c2 + li;
                if (row < pc && col < c) Cb[col * 65 + row] = acc[r2][c2][r];
              }
        }
      }
      __syncthreads();
      // Z_c -= P Cb, one 32 x 32 tile of Z_c per wave at a time
      const int nrt = (m + 31) / 32, nct = (c + 31) / 32;
      for (int t = wave; t < nrt * nct; t += nw) {
        const int i0 = 32 * (t % nrt), j0 = 32 * (t / nrt), li = lane & 15, lg = lane >> 4;
        double old[2][2][4];
#pragma unroll
        for (int r2 = 0; r2 < 2; ++r2)
#pragma unroll
          for (int c2 = 0; c2 < 2; ++c2)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = i0 + 16 * r2 + lg + 4 * r, col = j0 + 16 * c2 + li;
              old[r2][c2][r] = (row < m && col < c) ? Z[(size_t)(a + col) * m + row] : 0.0;
            }
        d4 acc[2][2];
        zero_acc(acc);
        wave_mma32<false, false>(Z + (size_t)p0 * m + i0, m, Cb + j0 * 65, 65, pc, m - i0, c - j0,
                                 acc);
#pragma unroll
        for (int r2 = 0; r2 < 2; ++r2)
#pragma unroll
          for (int c2 = 0; c2 < 2; ++c2)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = i0 + 16 * r2 + lg + 4 * r, col = j0 + 16 * c2 + li;
              if (row < m && col < c) Z[(size_t)(a + col) * m + row] = old[r2][c2][r] - acc[r2][c2][r];
            }
      }
      __syncthreads();
    }
  }
  // 1b. the cluster's own vectors in order (a vector replaced by a probe is taken against
  //     the whole chain again)
  for (int q = 0; q < c; ++q) {
    gmem<double> *zq = Z + (size_t)(a + q) * m;
    int replaced = 0;
    for (int pass = 0; pass < 2; ++pass) {
      const int pbase = replaced ? c0 : a;
      const int np = a + q - pbase;  // earlier vectors: columns pbase .. a + q - 1
      if (np > 0) {
        for (int p = wave; p < np; p += nw) {
          const gmem<double> *zp = Z + (size_t)(pbase + p) * m;
          double part = 0.0;
          for (int i = lane; i < m; i += 64) part += zp[i] * zq[i];
          part = wave_sum(part);
          if (lane == 0) dots[p] = part;
        }
        __syncthreads();
        for (int i = tid; i < m; i += nt) {
          double v = zq[i];
          for (int p = 0; p < np; ++p) v -= dots[p] * Z[(size_t)(pbase + p) * m + i];
          zq[i] = v;
        }
        __syncthreads();
      }
      double part = 0.0;
      for (int i = tid; i < m; i += nt) part += zq[i] * zq[i];
      const double nn = sqrt(wsum(part, red));
      if (nn < 1e-6 && pass == 0 && replaced < 2) {
        ++replaced;
        for (int i = tid; i < m; i += nt) {
          unsigned h = (unsigned)(i * 2654435761u) ^ (unsigned)((a + q) * 40503u + 1u);
          h ^= h >> 13;
          h *= 0x5bd1e995u;
          h ^= h >> 15;
          zq[i] = ((double)(h & 0xffffu) / 65536.0) - 0.5;
        }
        __syncthreads();
        pass = -1;  // orthogonalise the probe again from scratch
        continue;
      }
      for (int i = tid; i < m; i += nt) zq[i] /= nn;
      __syncthreads();
    }
  }
  // 2. W = T Z_c and H = Z_c^T W, one dot product per wave at a time
  for (int q = 0; q < c; ++q) {
    const gmem<double> *zq = Z + (size_t)(a + q) * m;
    for (int i = tid; i < m; i += nt) {
      double v = dg[i] * zq[i];
      if (i > 0) v += eg[i - 1] * zq[i - 1];
      if (i < m - 1) v += eg[i] * zq[i + 1];
      W[(size_t)q * m + i] = v;
    }
  }
  __syncthreads();
  for (int pq = wave; pq < c * c; pq += nw) {
    const int p = pq % c, q = pq / c;
    if (p > q) continue;
    const gmem<double> *zp = Z + (size_t)(a + p) * m;
    double part = 0.0;
    for (int i = lane; i < m; i += 64) part += zp[i] * W[(size_t)q * m + i];
    part = wave_sum(part);
    if (lane == 0) H[p][q] = H[q][p] = part;
  }
  for (int idx = tid; idx < kMaxCluster * kMaxCluster; idx += nt) {
    const int p = idx % kMaxCluster, q = idx / kMaxCluster;
    Vc[p][q] = (p == q) ? 1.0 : 0.0;
  }
  __syncthreads();
  // 3. Jacobi, round-robin ordering over ce = c rounded up to even (index c is a dummy)
  const int ce = c + (c & 1), npair = ce / 2;
  for (int sweep = 0; sweep < 30; ++sweep) {
    if (tid == 0) {
      double off = 0.0, dn = 0.0;
      for (int p = 0; p < c; ++p)
        for (int q = 0; q < c; ++q) (p == q ? dn : off) += H[p][q] * H[p][q];
      done = off <= 1e-32 * dn;
    }
    __syncthreads();
    if (done) break;
    for (int r = 0; r < ce - 1; ++r) {
      // pair i: positions i and ce - 1 - i of the rotated ring (position 0 fixed)
      if (tid < npair) {
        auto at = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + r) % (ce - 1); };
        int p = at(tid), q = at(ce - 1 - tid);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        double cs = 1.0, sn = 0.0;
        if (q < c && H[p][q] != 0.0) {
          const double th = (H[q][q] - H[p][p]) / (2.0 * H[p][q]);
          const double t = copysign(1.0, th) / (fabs(th) + sqrt(th * th + 1.0));
          cs = 1.0 / sqrt(t * t + 1.0);
          sn = t * cs;
        }
        pr[tid][0] = p, pr[tid][1] = q;
        rot[tid][0] = cs, rot[tid][1] = sn;
      }
      __syncthreads();
      // rows p, q of H (J^T from the left)
      for (int w = tid; w < npair * c; w += nt) {
        const int i = w / c, k = w % c, p = pr[i][0], q = pr[i][1];
        if (q >= c) continue;
        const double cs = rot[i][0], sn = rot[i][1];
        const double hp = H[p][k], hq = H[q][k];
        H[p][k] = cs * hp - sn * hq;
        H[q][k] = sn * hp + cs * hq;
      }
      __syncthreads();
      // columns p, q of H and of Vc (J from the right)
      for (int w = tid; w < npair * c; w += nt) {
        const int i = w / c, k = w % c, p = pr[i][0], q = pr[i][1];
        if (q >= c) continue;
        const double cs = rot[i][0], sn = rot[i][1];
        const double hp = H[k][p], hq = H[k][q];
        H[k][p] = cs * hp - sn * hq;
        H[k][q] = sn * hp + cs * hq;
        const double vp = Vc[k][p], vq = Vc[k][q];
        Vc[k][p] = cs * vp - sn * vq;
        Vc[k][q] = sn * vp + cs * vq;
      }
      __syncthreads();
    }
  }
  // ascending order inside the cluster (selection sort of the diagonal)
  if (tid == 0) {
    for (int p = 0; p < c; ++p) {
      int best = p;
      for (int q = p + 1; q < c; ++q)
        if (H[q][q] < H[best][best]) best = q;
      if (best != p) {
        const double t = H[p][p];
        H[p][p] = H[best][best];
        H[best][best] = t;
        for (int k = 0; k < c; ++k) {
          const double v = Vc[k][p];
          Vc[k][p] = Vc[k][best];
          Vc[k][best] = v;
        }
      }
    }
  }
  __syncthreads();
  // 4. Z_c <- Z_c Vc (through W), eigenvalues of the cluster
  for (int q = 0; q < c; ++q)
    for (int i = tid; i < m; i += nt) {
      double v = 0.0;
      for (int p = 0; p < c; ++p) v += Z[(size_t)(a + p) * m + i] * Vc[p][q];
      W[(size_t)q * m + i] = v;
    }
  __syncthreads();
  for (int q = 0; q < c; ++q)
    for (int i = tid; i < m; i += nt) Z[(size_t)(a + q) * m + i] = W[(size_t)q * m + i];
  if (tid < c) mu[a + tid] = H[tid][tid] - sigma;
  __syncthreads();
  }
  (void)flag;
}

// ---------------------------------------------------------------------------
// 6. Back-transformation Z <- H_0 ... H_{m-3} Z, eigenvalues lam = mu + sigma in
//    descending order. One wave per column.
// ---------------------------------------------------------------------------
// PER entries of the column per lane (64 PER >= m): 5, 9 or 17, chosen from m at launch, so
// a small m carries no dead entries.
template <int PER>
__global__ void __launch_bounds__(256)
    backtransform_kernel(int m, const double *__restrict__ work, double *__restrict__ lam,
                         double *__restrict__ Vout, const EigJob *__restrict__ jobs) {
  if (jobs) {
    const EigJob &J = jobs[blockIdx.y];
    m = J.m, work = J.work, lam = J.lam, Vout = J.Z;
  }
  EigLayout Lw(m);
  const gmem<double> *Hv = gptr(work + Lw.Hv);
  const gmem<double> *Z = gptr(work + Lw.Z);
  const gmem<double> *mu = gptr(work + Lw.mu);
  const gmem<double> *misc = gptr(work + Lw.misc);
  const int lane = threadIdx.x & 63;
  const int col = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (col >= m) return;
  double z[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int i = lane + 64 * q;
    z[q] = (i < m) ? Z[(size_t)col * m + i] : 0.0;
  }
  // Reflectors applied four at a time, k0, k0 - 1, k0 - 2, k0 - 3 (rows of Hv are zero on
  // and above the diagonal, and rows k < 0 count as zero): one reduction of the four dots
  // d_b = v_b^T z and the six products g_bc = v_b^T v_c gives the coefficients
  // t_b = d_b - 2 sum_{c<b} t_c g_bc of z <- z - 2 sum_b t_b v_b, so a wave waits for one
  // reduction per four reflectors. The next block's rows load during this one's.
  constexpr int B = 4, NR = B + B * (B - 1) / 2;
  auto load_block = [&](int k0, double (&v)[B][PER]) {
#pragma unroll
    for (int b = 0; b < B; ++b)
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int i = lane + 64 * q, k = k0 - b;
        v[b][q] = (k >= 0 && i < m) ? Hv[(size_t)k * m + i] : 0.0;
      }
  };
  double vb[B][PER], vn[B][PER];
  load_block(m - 3, vb);
  for (int k0 = m - 3; k0 >= 0; k0 -= B) {
    load_block(k0 - B, vn);
    double r[NR];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      double d = 0.0;
#pragma unroll
      for (int q = 0; q < PER; ++q) d += vb[b][q] * z[q];
      r[b] = d;
    }
    int g = B;
#pragma unroll
    for (int b = 1; b < B; ++b)
#pragma unroll
      for (int c = 0; c < b; ++c) {
        double d = 0.0;
#pragma unroll
        for (int q = 0; q < PER; ++q) d += vb[b][q] * vb[c][q];
        r[g++] = d;
      }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
      for (int t = 0; t < NR; ++t) r[t] += __shfl_xor(r[t], o, 64);
    double tc[B];
    g = B;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      double t = r[b];
#pragma unroll
      for (int c = 0; c < b; ++c) t -= 2.0 * tc[c] * r[g + c];
      if (b > 0) g += b;
      tc[b] = t;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      double u = 0.0;
#pragma unroll
      for (int b = 0; b < B; ++b) u += tc[b] * vb[b][q];
      z[q] -= 2.0 * u;
    }
#pragma unroll
    for (int b = 0; b < B; ++b)
#pragma unroll
      for (int q = 0; q < PER; ++q) vb[b][q] = vn[b][q];
  }
  // ascending index col -> descending position m-1-col (ties keep a stable order)
  const double lj = mu[col] + misc[3];
  int rank = 0;
  for (int i = lane; i < m; i += 64) {
    const double li = mu[i] + misc[3];
    rank += (li > lj || (li == lj && i > col)) ? 1 : 0;
  }
  for (int o = 32; o > 0; o >>= 1) rank += __shfl_xor(rank, o, 64);
  if (lane == 0) lam[rank] = lj;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int i = lane + 64 * q;
    if (i < m) Vout[(size_t)rank * m + i] = z[q];
  }
}

// 6'. Blocked back-transformation (compact WY, m <= kWyMaxM). The reflectors are taken in
// blocks of 32: Q_b = H_{32b} ... H_{32b+31} = I - V_b T_b V_b^T, with V_b's column j the
// reflector 32b + j and T_b upper triangular (T_jj = 2 for the unit reflectors, T[0:j, j] =
// -2 T[0:j, 0:j] V_b[:, 0:j]^T v_j). Z <- Q_0 Q_1 ... Z is applied last block first to strips
// of 16 columns held in LDS, S <- S - V_b (T_b (V_b^T S)): three MFMA products per block, with
// V_b staged in LDS once per block.
constexpr int kWyB = 32;
constexpr int kWyS = 16;  // strip width
constexpr int kWyMaxM = 288;

// T_b of block blockIdx.x into the scratch area (column-major 32 x 32 per block).
// Four waves: the Gram's rows split in four ranges of whole 16-row chunks, the partial sums
// added in a fixed order; wave 0 then runs the recurrence.
constexpr int kWyTWaves = 4;
__global__ void __launch_bounds__(64 * kWyTWaves)
    wy_t_kernel(int m, double *__restrict__ work, const EigJob *__restrict__ jobs) {
  if (jobs) m = jobs[blockIdx.y].m, work = jobs[blockIdx.y].work;
  const int k0 = blockIdx.x * kWyB;
  if (k0 >= m) return;
  EigLayout Lw(m);
  const gmem<double> *V = gptr(work + Lw.Hv + (size_t)k0 * m);  // V[i + j m] = v_{k0+j}[i]
  gmem<double> *Tb = gptr(work + Lw.scr + (size_t)blockIdx.x * kWyB * kWyB);
  const int nr = min(kWyB, m - k0);
  __shared__ double G[kWyB][kWyB + 1];
  __shared__ double Gp[kWyTWaves][kWyB * kWyB];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, lg = lane >> 4;
  // G = V^T V over rows k0.. (the reflectors vanish above); wave w takes rows
  // [k0 + r0, k0 + r1) of the range, whole chunks of 16
  {
    const int rows = m - k0, chunks = (rows + 15) / 16;
    const int c0 = chunks * wave / kWyTWaves, c1 = chunks * (wave + 1) / kWyTWaves;
    const int r0 = 16 * c0, r1 = min(rows, 16 * c1);
    d4 acc[2][2];
    zero_acc(acc);
    if (r1 > r0)
      wave_mma32<true, false>(V + k0 + r0, m, V + k0 + r0, m, r1 - r0, nr, nr, acc);
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          Gp[wave][(16 * rt + lg + 4 * r) * kWyB + 16 * ct + li] = acc[rt][ct][r];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < kWyB * kWyB; idx += 64 * kWyTWaves) {
    double g = Gp[0][idx];
#pragma unroll
    for (int w = 1; w < kWyTWaves; ++w) g += Gp[w][idx];
    G[idx / kWyB][idx % kWyB] = g;
  }
  __syncthreads();
  if (wave != 0) return;
  // lane i builds row i of T in registers: T[i][j] = -2 sum_{i<=l<j} T[i][l] G[l][j] needs only
  // its own row and broadcast reads of G, so the recurrence has no barrier
  double x[kWyB];
#pragma unroll
  for (int j = 0; j < kWyB; ++j) {
    double t = 0.0;
#pragma unroll
    for (int l = 0; l < j; ++l) t += x[l] * G[l][j];  // x[l] = 0 for l < i
    x[j] = (j == lane) ? ((j < nr) ? 2.0 : 0.0) : ((j > lane) ? -2.0 * t : 0.0);
  }
  if (lane < kWyB) {
#pragma unroll
    for (int j = 0; j < kWyB; ++j) Tb[lane + kWyB * j] = x[j];
  }
}

// One workgroup (four waves) per strip of 16 columns of Z; eigenvalues and vectors leave in
// descending order, as from backtransform_kernel.
__global__ void __launch_bounds__(256)
    backtransform_wy_kernel(int m, const double *__restrict__ work, double *__restrict__ lam,
                            double *__restrict__ Vout, const EigJob *__restrict__ jobs) {
  if (jobs) {
    const EigJob &J = jobs[blockIdx.y];
    m = J.m, work = J.work, lam = J.lam, Vout = J.Z;
  }
  const int c0 = blockIdx.x * kWyS;
  if (c0 >= m) return;
  EigLayout Lw(m);
  const gmem<double> *Hv = gptr(work + Lw.Hv);
  const gmem<double> *Z = gptr(work + Lw.Z);
  const gmem<double> *mu = gptr(work + Lw.mu);
  const gmem<double> *misc = gptr(work + Lw.misc);
  const gmem<double> *Tall = gptr(work + Lw.scr);
  constexpr int LW = kWyB + 1;
  // strip and reflector block, column-major with ld = m + 1 (odd: no bank clash)
  __shared__ double S[kWyS * (kWyMaxM + 1)], Vs[kWyB * (kWyMaxM + 1)];
  __shared__ double Wp[4][kWyS * LW], Ws[kWyS * LW], W2[kWyS * LW], Ts[kWyB * kWyB];
  const int ldS = m + 1, ldV = m + 1, nc = min(kWyS, m - c0);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lg = lane >> 4;
  __shared__ double muS[kWyMaxM];  // the shifted eigenvalues, for the final ordering
  {
    // every load of the strip (and of the eigenvalues) issued before the first wait, at a
    // clamped address past the strip's end (values dropped)
    constexpr int kPer = (kWyS * kWyMaxM + 255) / 256;
    double v[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const int idx = min(tid + 256 * t, kWyS * m - 1);
      const int i = idx % m, j = min(idx / m, nc - 1);
      v[t] = Z[(size_t)(c0 + j) * m + i];
    }
    const double shift = misc[3];
    const double mv0 = mu[min(tid, m - 1)], mv1 = mu[min(tid + 256, m - 1)];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const int idx = tid + 256 * t;
      if (idx < kWyS * m) {
        const int i = idx % m, j = idx / m;
        S[i + j * ldS] = (j < nc) ? v[t] : 0.0;
      }
    }
    if (tid < m) muS[tid] = mv0 + shift;
    if (tid + 256 < m) muS[tid + 256] = mv1 + shift;
  }
  __syncthreads();
  const int nblk = (m + kWyB - 1) / kWyB;
  // The next block's reflectors and T are fetched into registers while this block computes.
  constexpr int kPf = (kWyB * kWyMaxM + 255) / 256;
  double pf[kPf], tf[kWyB * kWyB / 256];
  auto fetch = [&](int bb) {
    const int k0 = kWyB * bb, nr = min(kWyB, m - k0), mk = m - k0;
    const int q256 = 256 / mk, r256 = 256 % mk;
    int i = tid % mk, j = tid / mk;
#pragma unroll
    for (int q = 0; q < kPf; ++q) {
      pf[q] = (j < nr) ? Hv[(size_t)(k0 + j) * m + k0 + i] : 0.0;
      i += r256;
      j += q256;
      if (i >= mk) i -= mk, ++j;
    }
#pragma unroll
    for (int q = 0; q < kWyB * kWyB / 256; ++q) tf[q] = Tall[(size_t)bb * kWyB * kWyB + tid + 256 * q];
  };
  fetch(nblk - 1);
  for (int b = nblk - 1; b >= 0; --b) {
    const int k0 = kWyB * b, nr = min(kWyB, m - k0), mk = m - k0;
    // Vs[(i - k0) + j ldV] = v_{k0+j}[i] for i >= k0 (the reflectors vanish above)
    {
      const int q256 = 256 / mk, r256 = 256 % mk;
      int i = tid % mk, j = tid / mk;
#pragma unroll
      for (int q = 0; q < kPf; ++q) {
        if (j < nr) Vs[i + j * ldV] = pf[q];
        i += r256;
        j += q256;
        if (i >= mk) i -= mk, ++j;
      }
#pragma unroll
      for (int q = 0; q < kWyB * kWyB / 256; ++q) Ts[tid + 256 * q] = tf[q];
    }
    __syncthreads();
    if (b > 0) fetch(b - 1);
    // a) W = V^T S over rows k0..m-1, the rows split four ways over the waves
    {
      const int kq = ((m - k0 + 3) / 4 + 3) & ~3;
      const int ks = k0 + wave * kq, ke = min(m, ks + kq);
      d4 acc[2][1];
      zero_acc(acc);
      if (ke > ks) wave_mma32<true, false, 1>(Vs + (ks - k0), ldV, S + ks, ldS, ke - ks, nr, nc, acc);
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 1; ++ct)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (16 * ct + li < kWyS) Wp[wave][(16 * rt + lg + 4 * r) + (16 * ct + li) * LW] = acc[rt][ct][r];
    }
    __syncthreads();
    for (int idx = tid; idx < kWyB * kWyS; idx += 256) {
      const int o = (idx % kWyB) + (idx / kWyB) * LW;
      Ws[o] = (Wp[0][o] + Wp[1][o]) + (Wp[2][o] + Wp[3][o]);
    }
    __syncthreads();
    // b) W2 = T_b W
    if (wave == 0) {
      d4 acc[2][1];
      zero_acc(acc);
      wave_mma32<false, false, 1>(Ts, kWyB, Ws, LW, kWyB, kWyB, nc, acc);
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 1; ++ct)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (16 * ct + li < kWyS) W2[(16 * rt + lg + 4 * r) + (16 * ct + li) * LW] = acc[rt][ct][r];
    }
    __syncthreads();
    // c) S -= V W2 on the row tiles from k0 down (each wave its own rows)
    for (int I = b + wave; I < nblk; I += 4) {
      const int r0 = kWyB * I;
      d4 acc[2][1];
      zero_acc(acc);
      wave_mma32<false, false, 1>(Vs + (r0 - k0), ldV, W2, LW, nr, m - r0, nc, acc);
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 1; ++ct)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = r0 + 16 * rt + lg + 4 * r, col = 16 * ct + li;
            if (row < m && col < nc) S[row + col * ldS] -= acc[rt][ct][r];
          }
    }
    __syncthreads();
  }
  // ascending index col -> descending position (ties keep a stable order)
  for (int j = wave; j < nc; j += 4) {
    const int col = c0 + j;
    const double lj = muS[col];
    int rank = 0;
    for (int i = lane; i < m; i += 64) {
      const double lv = muS[i];
      rank += (lv > lj || (lv == lj && i > col)) ? 1 : 0;
    }
    for (int o = 32; o > 0; o >>= 1) rank += __shfl_xor(rank, o, 64);
    if (lane == 0) lam[rank] = lj;
    for (int i = lane; i < m; i += 64) Vout[(size_t)rank * m + i] = S[i + j * ldS];
  }
}

// back-transform launch with the per-lane count for m (mmax: the largest m of the launch)
void launch_backtransform(dim3 grid, int mmax, int m, const double *work, double *lam, double *Z,
                          const EigJob *jobs, hipStream_t st) {
  if (mmax <= kWyMaxM) {
    const unsigned nblk = (unsigned)((mmax + kWyB - 1) / kWyB);
    const unsigned nstrip = (unsigned)((mmax + kWyS - 1) / kWyS);
    hipLaunchKernelGGL(wy_t_kernel, dim3(nblk, grid.y), dim3(64 * kWyTWaves), 0, st, m,
                       const_cast<double *>(work), jobs);
    hipLaunchKernelGGL(backtransform_wy_kernel, dim3(nstrip, grid.y), dim3(256), 0, st, m, work, lam,
                       Z, jobs);
    return;
  }
  if (mmax <= 5 * 64)
    hipLaunchKernelGGL(backtransform_kernel<5>, grid, dim3(256), 0, st, m, work, lam, Z, jobs);
  else if (mmax <= 9 * 64)
    hipLaunchKernelGGL(backtransform_kernel<9>, grid, dim3(256), 0, st, m, work, lam, Z, jobs);
  else
    hipLaunchKernelGGL(backtransform_kernel<17>, grid, dim3(256), 0, st, m, work, lam, Z, jobs);
}

}  // namespace

size_t eig_work_doubles(int m) { return EigLayout(m).total; }

hipError_t launch_eig(int m, const double *K, double *lam, double *Z, double *work, int *flag,
                      hipStream_t st) {
  if (m < 1 || m > kEigMaxM) return hipErrorInvalidValue;
  if (tile_fits(m))
    hipLaunchKernelGGL(tridiag_tile_kernel, dim3(1), dim3(tile_threads(m)), 0, st, m, K, work,
                       nullptr);
  else {
    // barrier counter and abort word after p and the workgroups' shares, cleared first
    int *gsync = reinterpret_cast<int *>(work + EigLayout(m).scr + m + kTriGridWG);
    hipError_t e0 = launch_zero_ints(gsync, 2, st);
    if (e0 != hipSuccess) return e0;
    hipLaunchKernelGGL(tridiag_grid_kernel, dim3(kTriGridWG), dim3(kTriGridThreads), 0, st, m, K,
                       work, gsync, flag);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(root_kernel, dim3(1), dim3(256), (size_t)4 * m * sizeof(double), st, m, work,
                     flag, nullptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(bisect_kernel, dim3((m + 3) / 4), dim3(256), (size_t)2 * m * sizeof(double), st,
                     m, work, nullptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(vector_kernel, dim3((m + 63) / 64), dim3(128), (size_t)3 * m * sizeof(double), st,
                     m, work, nullptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(cluster_scan_kernel, dim3(1), dim3(64), 0, st, m, work, nullptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(cluster_kernel, dim3(m), dim3(256), 0, st, m, work, flag, nullptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  launch_backtransform(dim3((m + 3) / 4), m, m, work, lam, Z, nullptr, st);
  return hipGetLastError();
}

// Batched: every problem's m must satisfy the register-tile tridiagonalisation bound.
hipError_t launch_eig_batched(int nprob, int maxm, const EigJob *jobs, hipStream_t st) {
  if (nprob <= 0) return hipSuccess;
  if (maxm < 1 || !tile_fits(maxm)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(tridiag_tile_kernel, dim3(1, nprob), dim3(tile_threads(maxm)), 0, st, 0,
                     nullptr, nullptr, jobs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(root_kernel, dim3(1, nprob), dim3(256), (size_t)4 * maxm * sizeof(double), st,
                     0, nullptr, nullptr, jobs);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(bisect_kernel, dim3((maxm + 3) / 4, nprob), dim3(256),
                     (size_t)2 * maxm * sizeof(double), st, 0, nullptr, jobs);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(vector_kernel, dim3((maxm + 63) / 64, nprob), dim3(128),
                     (size_t)3 * maxm * sizeof(double), st, 0, nullptr, jobs);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(cluster_scan_kernel, dim3(1, nprob), dim3(64), 0, st, 0, nullptr, jobs);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(cluster_kernel, dim3(maxm, nprob), dim3(256), 0, st, 0, nullptr, nullptr,
                     jobs);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  launch_backtransform(dim3((maxm + 3) / 4, nprob), maxm, 0, nullptr, nullptr, nullptr, jobs, st);
  return hipGetLastError();
}


}  // namespace riot
