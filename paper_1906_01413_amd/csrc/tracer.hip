// Tracer source inversion on a periodic 2-D grid: forward model, tangent-linear and adjoint
// sweeps over a batch of members, the square root of B, and the prior-preconditioned
// Hessian product of Alg. 3 for this model.
//
// Model (a synthetic stand-in for the transport model of the paper's black-carbon
// inversion, Sec. 3.2): explicit upwind advection by a positive wind (u(y) along x, v
// along y) and 5-point diffusion on an N x N periodic grid, emissions E * exp(s) on
// coarse space-time blocks of controls s (the lognormal transform of Sec. 3.2), point
// observations. The transport is linear in the concentration, so the tangent and the
// adjoint need the base emissions only, never a stored trajectory.
//
// Layout: fields [member][y][x] (x fastest); controls [member][time block][by][bx].
// The sweeps run two steps per launch over (tile, member): a 64 x 16 tile of cells plus a
// two-cell halo is staged in LDS (every row segment one coalesced run), the intermediate
// field stays in LDS, and each thread computes four rows of the tile. An odd last step
// uses the single-step kernels, which stage a one-cell halo.

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "riot_internal.h"

namespace riot {
namespace {

// cell tile kTX x kTY, threads kTX x kWY; thread (lx, ly) owns rows ly + kWY r, r < kRY
// (kRY ly + r in the adjoint pair kernel, for its control-block sums)
constexpr int kTX = 64, kWY = 4, kRY = 4, kTY = kWY * kRY;
constexpr int kThreads = kTX * kWY;
constexpr int kHX = kTX + 2, kHY = kTY + 2;

struct TracerView {
  int N, T, block, bshift, ntb, Nb, spb;  // block = 1 << bshift; spb: steps per time block
  double dt, aS, aE, aN;
  const double *a0, *aW;          // [N] row coefficients
};

__device__ __forceinline__ int wrap(int i, int N) { return i < 0 ? i + N : (i >= N ? i - N : i); }

// Tile of this workgroup. Workgroups are dealt round-robin to the 8 XCDs, each with its own
// L2; in dispatch order an XCD would get the tiles of one x column only, so its tiles'
// x-halo lines would never be in its L2. With the remap (when the tile rows split into 8
// bands) XCD j takes band j of tile rows for every member, x fastest: x neighbours share
// their halo lines in one L2, and its band of the emission fields stays resident there.
struct TileId {
  int x0, y0, mem;
};
__device__ __forceinline__ TileId tile_id() {
  const int gx = gridDim.x, gy = gridDim.y;
  int id = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  int bx, by, mem;
  if ((gy & 7) == 0) {
    const int band = gy >> 3, xcd = id & 7;
    int q = id >> 3;  // rank of this workgroup among its XCD's
    bx = q % gx;
    q /= gx;
    by = xcd * band + q % band;
    mem = q / band;
  } else {
    bx = id % gx;
    id /= gx;
    by = id % gy;
    mem = id / gy;
  }
  return {bx * kTX, by * kTY, mem};
}

// Stage the tile of `f` with its halo in LDS (row-major, kHY x kHX).
__device__ __forceinline__ void stage_tile(const double *__restrict__ f, int N, int x0, int y0,
                                           double *t) {
  for (int k = threadIdx.x; k < kHX * kHY; k += kThreads) {
    const int ty = k / kHX, tx = k - ty * kHX;
    t[k] = f[(size_t)wrap(y0 + ty - 1, N) * N + wrap(x0 + tx - 1, N)];
  }
}

// out = A in + dt W * up(bv): one step of the forward model (W = E, bv = exp(s_tau)) or of
// the tangent-linear model (W = E exp(up(s_b,tau)), bv = ds_tau). in may be nullptr (zero).
__global__ void __launch_bounds__(kThreads)
    tracer_step_kernel(TracerView tv, const double *__restrict__ in, double *__restrict__ out,
                       const double *__restrict__ W, const double *__restrict__ bv,
                       long long bv_stride) {
  __shared__ double t[kHX * kHY];
  const int N = tv.N;
  const size_t NN = (size_t)N * N;
  const TileId ti = tile_id();
  const int x0 = ti.x0, y0 = ti.y0, mem = ti.mem;
  const int lx = threadIdx.x % kTX, ly = threadIdx.x / kTX;
  const int x = x0 + lx;
  if (in) {
    stage_tile(in + mem * NN, N, x0, y0, t);
    __syncthreads();
  }
  const double *bvm = bv + mem * bv_stride;
#pragma unroll
  for (int r = 0; r < kRY; ++r) {
    const int yl = ly + kWY * r, y = y0 + yl;
    double acc = 0.0;
    if (in) {
      const int c = (yl + 1) * kHX + lx + 1;
      acc = tv.a0[y] * t[c] + tv.aW[y] * t[c - 1] + tv.aS * t[c - kHX] + tv.aE * t[c + 1] +
            tv.aN * t[c + kHX];
    }
    const double e = bvm[(size_t)(y >> tv.bshift) * tv.Nb + (x >> tv.bshift)];
    out[mem * NN + (size_t)y * N + x] = acc + tv.dt * W[(size_t)y * N + x] * e;
  }
}

// lam_out = A^T lam_in, and gS_tau += down(dt W * lam_in) per block x block cells
// (each control block of the tile summed row by row by one thread: fixed order).
__global__ void __launch_bounds__(kThreads)
    tracer_adjoint_kernel(TracerView tv, const double *__restrict__ lam_in,
                          double *__restrict__ lam_out, const double *__restrict__ W,
                          double *__restrict__ gS, long long gS_stride) {
  __shared__ double t[kHX * kHY];
  __shared__ double w[kTY][kTX];
  const int N = tv.N;
  const size_t NN = (size_t)N * N;
  const TileId ti = tile_id();
  const int x0 = ti.x0, y0 = ti.y0, mem = ti.mem;
  const int lx = threadIdx.x % kTX, ly = threadIdx.x / kTX;
  const int x = x0 + lx;
  stage_tile(lam_in + mem * NN, N, x0, y0, t);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRY; ++r) {
    const int yl = ly + kWY * r, y = y0 + yl;
    const int c = (yl + 1) * kHX + lx + 1;
    if (lam_out)
      lam_out[mem * NN + (size_t)y * N + x] = tv.a0[y] * t[c] + tv.aW[y] * t[c + 1] +
                                              tv.aS * t[c + kHX] + tv.aE * t[c - 1] +
                                              tv.aN * t[c - kHX];
    w[yl][lx] = tv.dt * W[(size_t)y * N + x] * t[c];
  }
  __syncthreads();
  const int b = tv.block;
  const int nbx = kTX / b, nby = kTY / b;
  for (int cb = threadIdx.x; cb < nbx * nby; cb += kThreads) {
    const int bxl = cb % nbx, byl = cb / nbx;
    double s = 0.0;
    for (int r = 0; r < b; ++r)
      for (int q = 0; q < b; ++q) s += w[byl * b + r][bxl * b + q];
    double *g = gS + mem * gS_stride + (size_t)((y0 / b) + byl) * tv.Nb + (x0 / b) + bxl;
    *g += s;
  }
}

// ---------------------------------------------------------------------------
// Two steps per launch (temporal blocking): the input tile is staged with a two-cell halo,
// the intermediate field is computed on the tile plus a one-cell ring and kept in LDS,
// and only the second step's field goes back to memory, so each field is read and
// written once per two steps. Observations of the intermediate state are taken (forward)
// or injected (adjoint) inside the launch.
// ---------------------------------------------------------------------------
constexpr int kGX = kTX + 4, kGY = kTY + 4;  // input tile with a two-cell halo

// out = A (A in + dt W0 up(bv0)) + dt W1 up(bv1) (steps t and t + 1; in may be nullptr);
// obs[mem nobs + orig[o]] = intermediate field at cell[o] for o in [beg, end).
// Every global load (the input tile, both steps' emission terms, the observation list) is
// issued before the first barrier, so a workgroup waits for memory once; the ring rows'
// coefficients a0, aW go to LDS.
constexpr int kStage2 = (kGX * kGY + kThreads - 1) / kThreads;
constexpr int kRing = (kHX * kHY + kThreads - 1) / kThreads;

template <bool IN>
__global__ void __launch_bounds__(kThreads)
    tracer_step2_kernel(TracerView tv, const double *__restrict__ in, double *__restrict__ out,
                        const double *__restrict__ W0, const double *__restrict__ bv0,
                        const double *__restrict__ W1, const double *__restrict__ bv1,
                        long long bv_stride, int beg, int end, const int *__restrict__ cell,
                        const int *__restrict__ orig, int nobs, double *__restrict__ obs) {
  __shared__ double t0[kGX * kGY];
  __shared__ double t1[kHX * kHY];
  __shared__ double ca0[kHY], caW[kHY];
  const int N = tv.N, sh = tv.bshift, tid = threadIdx.x;
  const size_t NN = (size_t)N * N;
  const TileId ti = tile_id();
  const int x0 = ti.x0, y0 = ti.y0, mem = ti.mem;
  const int lx = tid % kTX, ly = tid / kTX;
  const int x = x0 + lx;
  const double *b0m = bv0 + mem * bv_stride, *b1m = bv1 + mem * bv_stride;
  // Loads past the end of a strip are clamped to its last element and their values
  // dropped, so that every load is unconditional straight-line code and all of them are
  // in flight together.
  double sv[kStage2];
  if constexpr (IN) {
    const double *src = in + mem * NN;
#pragma unroll
    for (int i = 0; i < kStage2; ++i) {
      const int k = min(tid + i * kThreads, kGX * kGY - 1);
      const int ty = k / kGX, tx = k - ty * kGX;
      sv[i] = src[(size_t)wrap(y0 + ty - 2, N) * N + wrap(x0 + tx - 2, N)];
    }
  }
  double e0[kRing];  // emission term of the first step on the ring cells
#pragma unroll
  for (int i = 0; i < kRing; ++i) {
    const int k = min(tid + i * kThreads, kHX * kHY - 1);
    const int ry = k / kHX, rx = k - ry * kHX;
    const int y = wrap(y0 + ry - 1, N), xr = wrap(x0 + rx - 1, N);
    e0[i] = tv.dt * W0[(size_t)y * N + xr] * b0m[(size_t)(y >> sh) * tv.Nb + (xr >> sh)];
  }
  double e1[kRY];  // emission term of the second step on this thread's cells
#pragma unroll
  for (int r = 0; r < kRY; ++r) {
    const int y = y0 + ly + kWY * r;
    e1[r] = tv.dt * W1[(size_t)y * N + x] * b1m[(size_t)(y >> sh) * tv.Nb + (x >> sh)];
  }
  // observations of the intermediate state: one per thread prefetched (more loop below);
  // index 0 stands in where there is none (the tables hold at least one entry)
  const int o = beg + tid;
  const bool has_o = obs != nullptr && o < end;
  const int oc = cell[has_o ? o : 0], oo = orig[has_o ? o : 0];
  const int yr = wrap(y0 + min(tid, kHY - 1) - 1, N);
  const double a0r = tv.a0[yr], aWr = tv.aW[yr];
  if (tid < kHY) {
    ca0[tid] = a0r;
    caW[tid] = aWr;
  }
  if constexpr (IN) {
#pragma unroll
    for (int i = 0; i < kStage2; ++i) {
      const int k = tid + i * kThreads;
      if (k < kGX * kGY) t0[k] = sv[i];
    }
  }
  __syncthreads();
  // intermediate field on the tile and a one-cell ring (kHY x kHX, wrapped coordinates)
#pragma unroll
  for (int i = 0; i < kRing; ++i) {
    const int k = tid + i * kThreads;
    if (k < kHX * kHY) {
      const int ry = k / kHX, rx = k - ry * kHX;
      double acc = 0.0;
      if constexpr (IN) {
        const int c = (ry + 1) * kGX + rx + 1;
        acc = ca0[ry] * t0[c] + caW[ry] * t0[c - 1] + tv.aS * t0[c - kGX] + tv.aE * t0[c + 1] +
              tv.aN * t0[c + kGX];
      }
      t1[k] = acc + e0[i];
    }
  }
  __syncthreads();
  if (has_o) {
    const int cy = oc / N, cx = oc - cy * N;
    if (cy >= y0 && cy < y0 + kTY && cx >= x0 && cx < x0 + kTX)
      obs[(size_t)mem * nobs + oo] = t1[(cy - y0 + 1) * kHX + cx - x0 + 1];
  }
  if (obs) {
    for (int o2 = o + kThreads; o2 < end; o2 += kThreads) {
      const int cy = cell[o2] / N, cx = cell[o2] - cy * N;
      if (cy >= y0 && cy < y0 + kTY && cx >= x0 && cx < x0 + kTX)
        obs[(size_t)mem * nobs + orig[o2]] = t1[(cy - y0 + 1) * kHX + cx - x0 + 1];
    }
  }
#pragma unroll
  for (int r = 0; r < kRY; ++r) {
    const int yl = ly + kWY * r, y = y0 + yl;
    const int c = (yl + 1) * kHX + lx + 1;
    const double acc = ca0[yl + 1] * t1[c] + caW[yl + 1] * t1[c - 1] + tv.aS * t1[c - kHX] +
                       tv.aE * t1[c + 1] + tv.aN * t1[c + kHX];
    out[mem * NN + (size_t)y * N + x] = acc + e1[r];
  }
}

// Adjoint of two steps (states t -> t-1 -> t-2): lam1 = A^T lam_in on the tile and a ring,
// gS1 += down(dt W1 lam_in) (step t-1's emissions), the observation forcing of state t-1
// added to lam1 (unique cells u in [ubeg, uend)), lam_out = A^T lam1 (may be nullptr),
// gS0 += down(dt W0 lam1) (step t-2's emissions). gS1 and gS0 are the same block when both
// steps use one control time block, so they may alias.
//
// Here thread (lx, ly) owns the kRY consecutive rows kRY ly + r, so a control block
// (side 1, 2 or 4) has all its rows in one thread: its rows are summed in registers and its
// columns across b adjacent lanes of the wave by shuffles (a fixed tree, so the sums are
// deterministic), with no LDS for the block sums.
__device__ __forceinline__ void block_sums_add(double v[kRY], int b, int lx, double *g,
                                               int Nb) {
  // g points at the control of this thread's first row and column, (y / b, x / b)
  if (b == 1) {
#pragma unroll
    for (int r = 0; r < kRY; ++r) g[(size_t)r * Nb] += v[r];
  } else if (b == 2) {
    double s0 = v[0] + v[1], s1 = v[2] + v[3];
    s0 += __shfl_xor(s0, 1);
    s1 += __shfl_xor(s1, 1);
    if ((lx & 1) == 0) {
      g[0] += s0;
      g[Nb] += s1;
    }
  } else {
    double s = (v[0] + v[1]) + (v[2] + v[3]);
    s += __shfl_xor(s, 1);
    s += __shfl_xor(s, 2);
    if ((lx & 3) == 0) g[0] += s;
  }
}

__global__ void __launch_bounds__(kThreads)
    tracer_adjoint2_kernel(TracerView tv, const double *__restrict__ lam_in,
                           double *__restrict__ lam_out, const double *__restrict__ W1,
                           const double *__restrict__ W0, double *gS1, double *gS0,
                           long long gS_stride, int ubeg, int uend,
                           const int *__restrict__ ucell, const double *__restrict__ fu,
                           int nuniq) {
  __shared__ double t0[kGX * kGY];
  __shared__ double t1[kHX * kHY];
  __shared__ double ca0[kHY], caW[kHY];
  const int N = tv.N, tid = threadIdx.x;
  const size_t NN = (size_t)N * N;
  const TileId ti = tile_id();
  const int x0 = ti.x0, y0 = ti.y0, mem = ti.mem;
  const int lx = tid % kTX, ly = tid / kTX;
  const int x = x0 + lx, yb = y0 + kRY * ly;  // this thread's first row
  // every global load first: the input tile, both steps' emission fields on this thread's
  // cells, one forcing entry of state t-1 (more in the loop below)
  // (loads clamped to valid elements and unconditional, as in the forward pair)
  double sv[kStage2];
  {
    const double *src = lam_in + mem * NN;
#pragma unroll
    for (int i = 0; i < kStage2; ++i) {
      const int k = min(tid + i * kThreads, kGX * kGY - 1);
      const int ty = k / kGX, tx = k - ty * kGX;
      sv[i] = src[(size_t)wrap(y0 + ty - 2, N) * N + wrap(x0 + tx - 2, N)];
    }
  }
  double w1[kRY], w0[kRY];
#pragma unroll
  for (int r = 0; r < kRY; ++r) {
    w1[r] = W1[(size_t)(yb + r) * N + x];
    w0[r] = W0[(size_t)(yb + r) * N + x];
  }
  const int u = ubeg + tid;
  const bool has_u = u < uend;
  const int uc = ucell[has_u ? u : 0];
  const double uf = fu[(size_t)mem * nuniq + (has_u ? u : 0)];
  const int yr = wrap(y0 + min(tid, kHY - 1) - 1, N);
  const double a0r = tv.a0[yr], aWr = tv.aW[yr];
  if (tid < kHY) {
    ca0[tid] = a0r;
    caW[tid] = aWr;
  }
#pragma unroll
  for (int i = 0; i < kStage2; ++i) {
    const int k = tid + i * kThreads;
    if (k < kGX * kGY) t0[k] = sv[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kRing; ++i) {
    const int k = tid + i * kThreads;
    if (k < kHX * kHY) {
      const int ry = k / kHX, rx = k - ry * kHX;
      const int c = (ry + 1) * kGX + rx + 1;
      t1[k] = ca0[ry] * t0[c] + caW[ry] * t0[c + 1] + tv.aS * t0[c + kGX] + tv.aE * t0[c - 1] +
              tv.aN * t0[c - kGX];
    }
  }
  double v[kRY];
#pragma unroll
  for (int r = 0; r < kRY; ++r)
    v[r] = tv.dt * w1[r] * t0[(kRY * ly + r + 2) * kGX + lx + 2];
  __syncthreads();
  // forcing of state t-1 on the ring; a cell may sit at two ring positions when the ring
  // spans the whole period (N = kTX): the forcing goes to every copy
  auto add_forcing = [&](int cellu, double val) {
    const int cy = cellu / N, cx = cellu - cy * N;
    const int ry0 = wrap(cy - (y0 - 1), N), rx0 = wrap(cx - (x0 - 1), N);
    for (int ry = ry0; ry < kHY; ry += N)
      for (int rx = rx0; rx < kHX; rx += N) t1[ry * kHX + rx] += val;
  };
  if (has_u) add_forcing(uc, uf);
  for (int u2 = u + kThreads; u2 < uend; u2 += kThreads)
    add_forcing(ucell[u2], fu[(size_t)mem * nuniq + u2]);
  const int sh = tv.bshift;
  const size_t goff = (size_t)mem * gS_stride + (size_t)(yb >> sh) * tv.Nb + (x >> sh);
  block_sums_add(v, tv.block, lx, gS1 + goff, tv.Nb);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRY; ++r) {
    const int y = yb + r, rr = kRY * ly + r + 1;  // ring row of this cell
    const int c = rr * kHX + lx + 1;
    if (lam_out)
      lam_out[mem * NN + (size_t)y * N + x] = ca0[rr] * t1[c] + caW[rr] * t1[c + 1] +
                                              tv.aS * t1[c + kHX] + tv.aE * t1[c - 1] +
                                              tv.aN * t1[c - kHX];
    v[r] = tv.dt * w0[r] * t1[c];
  }
  block_sums_add(v, tv.block, lx, gS0 + goff, tv.Nb);
}

// Observation samples after a step: out[orig[o] + mem nobs] = f[y_o, x_o] for the step's o.
__global__ void tracer_sample_kernel(int N, int beg, int end, const int *__restrict__ cell,
                                     const int *__restrict__ orig, const double *__restrict__ f,
                                     int nobs, double *__restrict__ out) {
  const int o = beg + blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= end) return;
  const int mem = blockIdx.y;
  out[(size_t)mem * nobs + orig[o]] = f[(size_t)mem * N * N + cell[o]];
}

// Observation forcing gathered per unique cell: fu[mem nuniq + u] = sum of f over the
// observations of u (all steps at once, before an adjoint sweep).
__global__ void tracer_gather_kernel(int nuniq, const int *__restrict__ uptr,
                                     const int *__restrict__ orig, const double *__restrict__ f,
                                     int nobs, double *__restrict__ fu) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= nuniq) return;
  const int mem = blockIdx.y;
  double s = 0.0;
  for (int k = uptr[u]; k < uptr[u + 1]; ++k) s += f[(size_t)mem * nobs + orig[k]];
  fu[(size_t)mem * nuniq + u] = s;
}

// Observation forcing of one step: lam[cell_u] += fu[u] for the step's unique cells.
__global__ void tracer_inject_kernel(int N, int beg, int end, const int *__restrict__ ucell,
                                     const double *__restrict__ fu, int nuniq,
                                     double *__restrict__ lam) {
  const int u = beg + blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= end) return;
  const int mem = blockIdx.y;
  lam[(size_t)mem * N * N + ucell[u]] += fu[(size_t)mem * nuniq + u];
}

// Elementwise helpers.
__global__ void exp_kernel(long long n, const double *__restrict__ a, double *__restrict__ b) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = exp(a[i]);
}

// W_tau[y, x] = E[y, x] exp(s_b[tau, y / block, x / block]) for every time block.
__global__ void base_emission_kernel(TracerView tv, const double *__restrict__ E,
                                     const double *__restrict__ sb, double *__restrict__ W) {
  const size_t NN = (size_t)tv.N * tv.N;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NN * tv.ntb) return;
  const int tau = (int)(i / NN);
  const size_t c = i - (size_t)tau * NN;
  const int y = (int)(c / tv.N), x = (int)(c - (size_t)y * tv.N);
  W[i] = E[c] * exp(sb[(size_t)tau * tv.Nb * tv.Nb + (size_t)(y >> tv.bshift) * tv.Nb + (x >> tv.bshift)]);
}

__global__ void zero_kernel(long long n, double *__restrict__ a) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0;
}

// d = y - hx; f = rinv d (observation space, one column)
__global__ void innov_kernel(int nobs, const double *__restrict__ y, const double *__restrict__ hx,
                             const double *__restrict__ rinv, double *__restrict__ d,
                             double *__restrict__ f) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nobs) return;
  const double dv = y[o] - hx[o];
  d[o] = dv;
  f[o] = rinv[o] * dv;
}

// out = v - a (v nullable); out = rinv * in row by row (scale_rows) for m columns
__global__ void axpy_rows_kernel(long long n, const double *__restrict__ v,
                                 const double *__restrict__ a, double *__restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (v ? v[i] : 0.0) - a[i];
}

__global__ void scale_rows_kernel(int nobs, int m, const double *__restrict__ rinv,
                                  const double *in, double *out) {  // in may alias out
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)nobs * m) return;
  out[i] = rinv[i % nobs] * in[i];
}

__global__ void cost_terms_kernel(int n, const double *__restrict__ v, int nobs,
                                  const double *__restrict__ d, const double *__restrict__ rinv,
                                  double *__restrict__ out) {
  __shared__ double red[1024];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    if (v) a += v[i] * v[i];
  for (int o = threadIdx.x; o < nobs; o += blockDim.x) a += rinv[o] * d[o] * d[o];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = 0.5 * red[0];
}

unsigned blocks_for(long long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace
}  // namespace riot

using riot::TracerView;

struct riot_tracer {
  riot_tracer_desc d{};
  hipStream_t st = nullptr;
  int Nb = 0, ncontrol = 0, nuniq = 0;
  TracerView tv{};
  // device regions
  double *a0 = nullptr, *aW = nullptr, *E = nullptr, *Wb = nullptr, *sb = nullptr,
         *expS = nullptr;
  double *y = nullptr, *rinv = nullptr, *L1 = nullptr;
  int *cell = nullptr, *orig = nullptr, *ucell = nullptr, *uptr = nullptr;
  double *F0 = nullptr, *F1 = nullptr;           // m_max fields each (ping-pong)
  double *CA = nullptr, *CB = nullptr, *CC = nullptr;  // m_max control blocks each
  double *OA = nullptr;                          // m_max observation columns
  double *FU = nullptr;                          // m_max forcing columns per unique cell
  double *hx = nullptr, *dvec = nullptr, *fvec = nullptr, *scal = nullptr;
  // host tables: observations sorted by step (offsets per step), unique cells per step
  std::vector<int> obs_off, u_off;
  bool has_base = false;
};

namespace {

size_t a256(size_t b) { return (b + 255) / 256 * 256; }

struct TCarve {
  char *base;
  size_t off = 0;
  explicit TCarve(void *b) : base(static_cast<char *>(b)) {}
  template <typename T>
  T *take(size_t n) {
    off = a256(off);
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += std::max<size_t>(n, 1) * sizeof(T);
    return p;
  }
};

bool tracer_desc_ok(const riot_tracer_desc *d) {
  if (!d || d->N < 4 || d->N % 64 || d->nsteps < 1 || d->nobs < 0 || d->m_max < 1) return false;
  if (!(d->block == 1 || d->block == 2 || d->block == 4) || d->N % d->block) return false;
  if (d->ntb < 1 || d->nsteps % d->ntb) return false;
  if (!(d->dt > 0) || d->u0 - std::fabs(d->u1) < 0 || d->v < 0 || d->K < 0) return false;
  const double cmax = d->dt * (d->u0 + std::fabs(d->u1) + d->v) + 4.0 * d->dt * d->K;
  if (cmax > 1.0) return false;  // the explicit upwind step needs a Courant number <= 1
  if (!d->E || !d->L1 || !(d->sigma > 0)) return false;
  if (d->nobs > 0 && (!d->obs_t || !d->obs_y || !d->obs_x || !d->y || !d->rinv)) return false;
  for (int o = 0; o < d->nobs; ++o)
    if (d->obs_t[o] < 1 || d->obs_t[o] > d->nsteps || d->obs_y[o] < 0 || d->obs_y[o] >= d->N ||
        d->obs_x[o] < 0 || d->obs_x[o] >= d->N)
      return false;
  return true;
}

size_t tracer_carve(riot_tracer &h, void *base) {
  TCarve c(base);
  const riot_tracer_desc &d = h.d;
  const size_t NN = (size_t)d.N * d.N, m = d.m_max;
  const int Nb = d.N / d.block;
  const size_t nc = (size_t)d.ntb * Nb * Nb;
  h.a0 = c.take<double>(d.N);
  h.aW = c.take<double>(d.N);
  h.E = c.take<double>(NN);
  h.Wb = c.take<double>(NN * d.ntb);
  h.sb = c.take<double>(nc);
  h.expS = c.take<double>(nc);
  h.y = c.take<double>(d.nobs);
  h.rinv = c.take<double>(d.nobs);
  h.L1 = c.take<double>((size_t)Nb * Nb);
  h.cell = c.take<int>(d.nobs);
  h.orig = c.take<int>(d.nobs);
  h.ucell = c.take<int>(d.nobs);
  h.uptr = c.take<int>(d.nobs + 1);
  h.F0 = c.take<double>(NN * m);
  h.F1 = c.take<double>(NN * m);
  h.CA = c.take<double>(nc * m);
  h.CB = c.take<double>(nc * m);
  h.CC = c.take<double>(nc * m);
  h.OA = c.take<double>((size_t)std::max(d.nobs, 1) * m);
  h.FU = c.take<double>((size_t)std::max(d.nobs, 1) * m);
  h.hx = c.take<double>(d.nobs);
  h.dvec = c.take<double>(d.nobs);
  h.fvec = c.take<double>(d.nobs);
  h.scal = c.take<double>(16);
  return a256(c.off) + 256;
}

#define TR_HIP(call)                            \
  do {                                          \
    if ((call) != hipSuccess) return RIOT_E_HIP; \
  } while (0)

// One sweep of the forward or tangent model over all members: fields start at zero,
// step t uses control block tau(t); observation samples into obs [nobs x m].
riot_status tracer_forward_sweep(riot_tracer *h, int m, const double *Wfield, long long Wstride,
                                 const double *bv, long long bv_stride, double *obs) {
  const riot_tracer_desc &d = h->d;
  const TracerView &tv = h->tv;
  const dim3 grid(d.N / riot::kTX, d.N / riot::kTY, m);
  double *cur = nullptr, *bufs[2] = {h->F0, h->F1};
  const int Nbb = h->Nb * h->Nb;
  int nb = 0;  // buffers written so far
  // observations of state s (the field after step s - 1) are [obs_off[s + 1], obs_off[s + 2])
  auto sample = [&](int s, const double *f) -> riot_status {
    const int beg = h->obs_off[s + 1], end = h->obs_off[s + 2];
    if (end > beg && obs) {
      hipLaunchKernelGGL(riot::tracer_sample_kernel, dim3(riot::blocks_for(end - beg), m),
                         dim3(256), 0, h->st, d.N, beg, end, h->cell, h->orig, f, d.nobs, obs);
      TR_HIP(hipGetLastError());
    }
    return RIOT_OK;
  };
  int t = 0;
  for (; t + 1 < d.nsteps; t += 2) {  // steps t and t + 1 in one launch
    const int tau0 = t / tv.spb, tau1 = (t + 1) / tv.spb;
    double *next = bufs[(nb++) & 1];
    hipLaunchKernelGGL(cur ? riot::tracer_step2_kernel<true> : riot::tracer_step2_kernel<false>,
                       grid, dim3(riot::kThreads), 0, h->st, tv, cur,
                       next, Wfield + Wstride * tau0, bv + (size_t)tau0 * Nbb,
                       Wfield + Wstride * tau1, bv + (size_t)tau1 * Nbb, bv_stride,
                       h->obs_off[t + 2], h->obs_off[t + 3], h->cell, h->orig, d.nobs, obs);
    TR_HIP(hipGetLastError());
    riot_status rs = sample(t + 2, next);
    if (rs != RIOT_OK) return rs;
    cur = next;
  }
  if (t < d.nsteps) {  // odd number of steps: the last one alone
    const int tau = t / tv.spb;
    double *next = bufs[(nb++) & 1];
    hipLaunchKernelGGL(riot::tracer_step_kernel, grid, dim3(riot::kThreads), 0, h->st, tv, cur,
                       next, Wfield + Wstride * tau, bv + (size_t)tau * Nbb, bv_stride);
    TR_HIP(hipGetLastError());
    riot_status rs = sample(t + 1, next);
    if (rs != RIOT_OK) return rs;
  }
  return RIOT_OK;
}

// Adjoint sweep: gS [ncontrol x m] = G^T f for observation-space f [nobs x m].
riot_status tracer_adjoint_sweep(riot_tracer *h, int m, const double *f, double *gS) {
  const riot_tracer_desc &d = h->d;
  const TracerView &tv = h->tv;
  const size_t NN = (size_t)d.N * d.N;
  const dim3 grid(d.N / riot::kTX, d.N / riot::kTY, m);
  hipLaunchKernelGGL(riot::zero_kernel, dim3(riot::blocks_for((long long)NN * m)), dim3(256), 0,
                     h->st, (long long)NN * m, h->F0);
  TR_HIP(hipGetLastError());
  hipLaunchKernelGGL(riot::zero_kernel, dim3(riot::blocks_for((long long)h->ncontrol * m)),
                     dim3(256), 0, h->st, (long long)h->ncontrol * m, gS);
  TR_HIP(hipGetLastError());
  if (h->nuniq > 0) {
    hipLaunchKernelGGL(riot::tracer_gather_kernel, dim3(riot::blocks_for(h->nuniq), m), dim3(256),
                       0, h->st, h->nuniq, h->uptr, h->orig, f, d.nobs, h->FU);
    TR_HIP(hipGetLastError());
  }
  double *lam = h->F0, *other = h->F1;
  const int Nbb = h->Nb * h->Nb;
  // forcing of state t: unique cells [u_off[t], u_off[t + 1])
  auto inject = [&](int t) -> riot_status {
    const int beg = h->u_off[t], end = h->u_off[t + 1];
    if (end > beg) {
      hipLaunchKernelGGL(riot::tracer_inject_kernel, dim3(riot::blocks_for(end - beg), m),
                         dim3(256), 0, h->st, d.N, beg, end, h->ucell, h->FU, h->nuniq, lam);
      TR_HIP(hipGetLastError());
    }
    return RIOT_OK;
  };
  int t = d.nsteps;
  for (; t >= 2; t -= 2) {  // states t -> t-1 -> t-2 in one launch
    riot_status rs = inject(t);
    if (rs != RIOT_OK) return rs;
    const int tau1 = (t - 1) / tv.spb, tau0 = (t - 2) / tv.spb;
    hipLaunchKernelGGL(riot::tracer_adjoint2_kernel, grid, dim3(riot::kThreads), 0, h->st, tv,
                       lam, t > 2 ? other : nullptr, h->Wb + NN * tau1, h->Wb + NN * tau0,
                       gS + (size_t)tau1 * Nbb, gS + (size_t)tau0 * Nbb, (long long)h->ncontrol,
                       h->u_off[t - 1], h->u_off[t], h->ucell, h->FU, h->nuniq);
    TR_HIP(hipGetLastError());
    std::swap(lam, other);
  }
  if (t == 1) {  // odd number of steps: the first one alone
    riot_status rs = inject(1);
    if (rs != RIOT_OK) return rs;
    hipLaunchKernelGGL(riot::tracer_adjoint_kernel, grid, dim3(riot::kThreads), 0, h->st, tv, lam,
                       nullptr, h->Wb, gS, (long long)h->ncontrol);
    TR_HIP(hipGetLastError());
  }
  return RIOT_OK;
}

// S = L Z = sigma (L1 kron L1) Z per time-block image: with an image Z stored [by][bx]
// read as the column-major matrix M = Z^T, L1 Z L1 corresponds to L1 M L1 (L1 symmetric).
riot_status tracer_apply_L(riot_tracer *h, int m, const double *Z, double *S, double *tmp) {
  const int Nb = h->Nb;
  const long long img = (long long)Nb * Nb;
  const int nimg = m * h->d.ntb;
  TR_HIP(riot::gemm_f64_strided(0, 0, Nb, Nb, Nb, 1.0, Z, Nb, img, h->L1, Nb, 0, 0.0, tmp, Nb, img,
                                nimg, h->st));
  TR_HIP(riot::gemm_f64_strided(0, 0, Nb, Nb, Nb, h->d.sigma, h->L1, Nb, 0, tmp, Nb, img, 0.0, S,
                                Nb, img, nimg, h->st));
  return RIOT_OK;
}

}  // namespace

extern "C" {

size_t riot_tracer_workspace_bytes(const riot_tracer_desc *desc) {
  if (!tracer_desc_ok(desc)) return 0;
  riot_tracer h;
  h.d = *desc;
  return tracer_carve(h, nullptr);
}

riot_status riot_tracer_init(const riot_tracer_desc *desc, void *workspace, size_t bytes,
                             void *hip_stream, riot_tracer **out) {
  if (!out) return RIOT_E_ARG;
  *out = nullptr;
  if (!tracer_desc_ok(desc) || !workspace) return RIOT_E_ARG;
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return RIOT_E_WORKSPACE;
  if (bytes < riot_tracer_workspace_bytes(desc)) return RIOT_E_WORKSPACE;
  riot_tracer *h = new (std::nothrow) riot_tracer();
  if (!h) return RIOT_E_ARG;
  h->d = *desc;
  h->st = static_cast<hipStream_t>(hip_stream);
  tracer_carve(*h, workspace);
  const riot_tracer_desc &d = h->d;
  h->Nb = d.N / d.block;
  h->ncontrol = d.ntb * h->Nb * h->Nb;
  // stencil coefficients of the upwind / diffusion step
  std::vector<double> a0(d.N), aW(d.N);
  for (int yy = 0; yy < d.N; ++yy) {
    const double u = d.u0 + d.u1 * std::sin(2.0 * 3.14159265358979323846 * yy / d.N);
    a0[yy] = 1.0 - d.dt * (u + d.v) - 4.0 * d.dt * d.K;
    aW[yy] = d.dt * (u + d.K);
  }
  TracerView &tv = h->tv;
  tv.N = d.N, tv.T = d.nsteps, tv.block = d.block, tv.ntb = d.ntb, tv.Nb = h->Nb;
  tv.bshift = d.block == 4 ? 2 : (d.block == 2 ? 1 : 0);
  tv.spb = d.nsteps / d.ntb;
  tv.dt = d.dt, tv.aS = d.dt * (d.v + d.K), tv.aE = d.dt * d.K, tv.aN = d.dt * d.K;
  tv.a0 = h->a0, tv.aW = h->aW;
  // observations sorted by step; per step, unique cells with lists of observations.
  // obs_off[t + 1] .. obs_off[t + 2]: sorted observations of step t; u_off[t] .. u_off[t + 1]:
  // unique cells of step t
  std::vector<int> ord(d.nobs);
  for (int o = 0; o < d.nobs; ++o) ord[o] = o;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    if (d.obs_t[a] != d.obs_t[b]) return d.obs_t[a] < d.obs_t[b];
    return (long long)d.obs_y[a] * d.N + d.obs_x[a] < (long long)d.obs_y[b] * d.N + d.obs_x[b];
  });
  std::vector<int> cell(d.nobs), ucell, uptr{0};
  h->obs_off.assign(d.nsteps + 3, 0);
  h->u_off.assign(d.nsteps + 2, 0);
  for (int k = 0; k < d.nobs; ++k) {
    const int o = ord[k];
    cell[k] = d.obs_y[o] * d.N + d.obs_x[o];
    h->obs_off[d.obs_t[o] + 2]++;
    if (k == 0 || d.obs_t[ord[k - 1]] != d.obs_t[o] || cell[k - 1] != cell[k]) {
      ucell.push_back(cell[k]);
      uptr.push_back(uptr.back());
      h->u_off[d.obs_t[o] + 1]++;
    }
    uptr.back()++;
  }
  for (int t = 1; t < (int)h->obs_off.size(); ++t) h->obs_off[t] += h->obs_off[t - 1];
  for (int t = 1; t < (int)h->u_off.size(); ++t) h->u_off[t] += h->u_off[t - 1];
  h->nuniq = (int)ucell.size();
  riot_status rs = RIOT_OK;
  auto cp = [&](void *dst, const void *src, size_t b) {
    if (b && hipMemcpyAsync(dst, src, b, hipMemcpyHostToDevice, h->st) != hipSuccess)
      rs = RIOT_E_HIP;
  };
  const size_t NN = (size_t)d.N * d.N;
  cp(h->a0, a0.data(), d.N * sizeof(double));
  cp(h->aW, aW.data(), d.N * sizeof(double));
  cp(h->E, d.E, NN * sizeof(double));
  cp(h->L1, d.L1, (size_t)h->Nb * h->Nb * sizeof(double));
  cp(h->cell, cell.data(), cell.size() * sizeof(int));
  cp(h->orig, ord.data(), ord.size() * sizeof(int));
  cp(h->ucell, ucell.data(), ucell.size() * sizeof(int));
  cp(h->uptr, uptr.data(), uptr.size() * sizeof(int));
  cp(h->y, d.y, (size_t)d.nobs * sizeof(double));
  cp(h->rinv, d.rinv, (size_t)d.nobs * sizeof(double));
  if (hipStreamSynchronize(h->st) != hipSuccess) rs = RIOT_E_HIP;
  h->d.E = nullptr, h->d.L1 = nullptr, h->d.obs_t = nullptr, h->d.obs_y = nullptr;
  h->d.obs_x = nullptr, h->d.y = nullptr, h->d.rinv = nullptr;
  if (rs != RIOT_OK) {
    delete h;
    return rs;
  }
  *out = h;
  return RIOT_OK;
}

void riot_tracer_free(riot_tracer *h) { delete h; }

riot_status riot_tracer_forward(riot_tracer *h, const double *s, double *obs) {
  if (!h || !s || (h->d.nobs > 0 && !obs)) return RIOT_E_ARG;
  const riot_tracer_desc &d = h->d;
  hipStream_t st = h->st;
  // base state for the derivatives: s_b = s, W_tau = E exp(up(s_tau))
  TR_HIP(hipMemcpyAsync(h->sb, s, (size_t)h->ncontrol * sizeof(double), hipMemcpyDeviceToDevice,
                        st));
  const size_t NN = (size_t)d.N * d.N;
  hipLaunchKernelGGL(riot::base_emission_kernel, dim3(riot::blocks_for((long long)NN * d.ntb)),
                     dim3(256), 0, st, h->tv, h->E, h->sb, h->Wb);
  TR_HIP(hipGetLastError());
  hipLaunchKernelGGL(riot::exp_kernel, dim3(riot::blocks_for(h->ncontrol)), dim3(256), 0, st,
                     (long long)h->ncontrol, s, h->expS);
  TR_HIP(hipGetLastError());
  h->has_base = true;
  return tracer_forward_sweep(h, 1, h->E, 0, h->expS, h->ncontrol, obs);
}

riot_status riot_tracer_tangent(riot_tracer *h, int32_t m, const double *dS, double *dObs) {
  if (!h || !dS || m < 1 || m > h->d.m_max || (h->d.nobs > 0 && !dObs)) return RIOT_E_ARG;
  if (!h->has_base) return RIOT_E_STATE;
  return tracer_forward_sweep(h, m, h->Wb, (long long)h->d.N * h->d.N, dS, h->ncontrol, dObs);
}

riot_status riot_tracer_adjoint(riot_tracer *h, int32_t m, const double *gObs, double *gS) {
  if (!h || !gS || m < 1 || m > h->d.m_max || (h->d.nobs > 0 && !gObs)) return RIOT_E_ARG;
  if (!h->has_base) return RIOT_E_STATE;
  return tracer_adjoint_sweep(h, m, gObs, gS);
}

riot_status riot_tracer_apply_L(riot_tracer *h, int32_t m, const double *Z, double *S) {
  if (!h || !Z || !S || Z == S || m < 1 || m > h->d.m_max) return RIOT_E_ARG;
  return tracer_apply_L(h, m, Z, S, h->CC);
}

riot_status riot_tracer_hess_apply(riot_tracer *h, int32_t m, const double *W, double *Y) {
  if (!h || !W || !Y || W == Y || m < 1 || m > h->d.m_max) return RIOT_E_ARG;
  if (!h->has_base) return RIOT_E_STATE;
  const riot_tracer_desc &d = h->d;
  riot_status rs;
  if ((rs = tracer_apply_L(h, m, W, h->CA, h->CC)) != RIOT_OK) return rs;
  if ((rs = tracer_forward_sweep(h, m, h->Wb, (long long)d.N * d.N, h->CA, h->ncontrol, h->OA)) !=
      RIOT_OK)
    return rs;
  if (d.nobs > 0) {
    hipLaunchKernelGGL(riot::scale_rows_kernel, dim3(riot::blocks_for((long long)d.nobs * m)),
                       dim3(256), 0, h->st, d.nobs, m, h->rinv, h->OA, h->OA);
    TR_HIP(hipGetLastError());
  }
  if ((rs = tracer_adjoint_sweep(h, m, h->OA, h->CB)) != RIOT_OK) return rs;
  return tracer_apply_L(h, m, h->CB, Y, h->CC);
}

riot_status riot_tracer_gradient(riot_tracer *h, const double *v, double *grad, double *d_out,
                                 double *J_host) {
  if (!h || !grad) return RIOT_E_ARG;
  if (!h->has_base) return RIOT_E_STATE;
  const riot_tracer_desc &d = h->d;
  hipStream_t st = h->st;
  riot_status rs;
  // d = y - H(M(s_b)) from a fresh forward sweep at the base, f = R^{-1} d
  if ((rs = tracer_forward_sweep(h, 1, h->E, 0, h->expS, h->ncontrol, h->hx)) != RIOT_OK) return rs;
  if (d.nobs > 0) {
    hipLaunchKernelGGL(riot::innov_kernel, dim3(riot::blocks_for(d.nobs)), dim3(256), 0, st,
                       d.nobs, h->y, h->hx, h->rinv, h->dvec, h->fvec);
    TR_HIP(hipGetLastError());
    if (d_out)
      TR_HIP(hipMemcpyAsync(d_out, h->dvec, (size_t)d.nobs * sizeof(double),
                            hipMemcpyDeviceToDevice, st));
  }
  if ((rs = tracer_adjoint_sweep(h, 1, h->fvec, h->CB)) != RIOT_OK) return rs;
  if ((rs = tracer_apply_L(h, 1, h->CB, h->CA, h->CC)) != RIOT_OK) return rs;
  hipLaunchKernelGGL(riot::axpy_rows_kernel, dim3(riot::blocks_for(h->ncontrol)), dim3(256), 0, st,
                     (long long)h->ncontrol, v, h->CA, grad);
  TR_HIP(hipGetLastError());
  if (J_host) {
    hipLaunchKernelGGL(riot::cost_terms_kernel, dim3(1), dim3(1024), 0, st, h->ncontrol, v, d.nobs,
                       h->dvec, h->rinv, h->scal);
    TR_HIP(hipGetLastError());
    TR_HIP(hipMemcpyAsync(J_host, h->scal, sizeof(double), hipMemcpyDeviceToHost, st));
    TR_HIP(hipStreamSynchronize(st));
  }
  return RIOT_OK;
}

}  // extern "C"
