// Lorenz-96 nonlinear, tangent-linear and adjoint integrations for gfx950.
//
// Model: Section 3.1.1 (Lorenz-96, periodic), integrated with classical RK4.
// Hessian-probe product (Alg. 3, y_i = A w_i with A = L^T G^T R^{-1} G L):
// one TL sweep over the window collecting R^{-1}-weighted observation values,
// one AD sweep injecting them at the observed steps. Each member (probe) runs
// in one workgroup with its state in registers; the periodic halo is exchanged
// through LDS once per RK4 stage.

#include <cstdlib>

#include "riot_internal.h"

namespace riot {
namespace {

constexpr int kLdsSlots = 4;

__device__ __forceinline__ int slot_of(int jj, int E) {
  if (jj == 0) return 0;
  if (jj == 1) return 1;
  if (jj == E - 2) return 2;
  return 3;
}

// LDS offsets of the four neighbours a-2, a-1, a+E, a+E+1 of thread l.
template <int E>
struct HaloMap {
  int off[4];
  __device__ void init(int l, int n, int NT) {
    const int a = l * E;
    const int g[4] = {a - 2, a - 1, a + E, a + E + 1};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int gg = g[k] % n;
      if (gg < 0) gg += n;
      off[k] = slot_of(gg % E, E) * NT + gg / E;
    }
  }
};

// Barrier for a halo exchange: the workgroup, or (WAVE) only the calling wave, whose LDS
// operations complete in issue order, so waiting for its own writes is enough.
template <bool WAVE>
__device__ __forceinline__ void member_sync() {
  if constexpr (WAVE) {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

// Write this thread's boundary values, barrier, read the neighbours'.
// All threads of the block (of the wave, WAVE) must call it (inactive ones pass active=false).
template <typename Real, int E, bool WAVE = false>
__device__ __forceinline__ void exchange(Real *lds, int &parity, int NT, int l, bool active,
                                         const HaloMap<E> &hm, const Real (&v)[E], Real &hl2,
                                         Real &hl1, Real &hr1, Real &hr2) {
  Real *b = lds + parity * kLdsSlots * NT;
  if (active) {
    b[0 * NT + l] = v[0];
    b[1 * NT + l] = v[E > 1 ? 1 : 0];
    b[2 * NT + l] = v[E > 1 ? E - 2 : 0];
    b[3 * NT + l] = v[E - 1];
  }
  member_sync<WAVE>();
  if (active) {
    hl2 = b[hm.off[0]];
    hl1 = b[hm.off[1]];
    hr1 = b[hm.off[2]];
    hr2 = b[hm.off[3]];
  }
  parity ^= 1;
}

// Load the (E + 4)-value extended base state xe[k] = x[a - 2 + k] of one stage block.
template <typename Real, int E>
__device__ __forceinline__ void load_base(const Real *__restrict__ blk, int NT, int l,
                                          Real (&xe)[E + 4]) {
#pragma unroll
  for (int j = 0; j < E; ++j) xe[2 + j] = blk[j * NT + l];
  xe[0] = blk[(E + 0) * NT + l];
  xe[1] = blk[(E + 1) * NT + l];
  xe[E + 2] = blk[(E + 2) * NT + l];
  xe[E + 3] = blk[(E + 3) * NT + l];
}

// The same load through a buffer resource over the whole trajectory: the row offset is a
// scalar (SGPR) and the lane offset one VGPR, so no per-row 64-bit vector address is
// formed or kept live across the window loop. Reads past the resource return 0.
struct TrajRsrc {
  __amdgpu_buffer_rsrc_t r;
  int row_bytes;  // NT * sizeof(Real)
};

template <typename Real>
__device__ __forceinline__ TrajRsrc traj_rsrc(const ModelView &mv) {
  const long long bytes = (long long)(mv.T + 1) * 4 * (mv.E + 4) * mv.NT * (long long)sizeof(Real);
  const int nrec = bytes > 0x7fffffffLL ? 0x7fffffff : (int)bytes;
  // dword 3 = 0x00020000: raw 32-bit data format of the gfx9 family
  return {__builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(mv.xs), (short)0, nrec, 0x00020000),
          mv.NT * (int)sizeof(Real)};
}

template <typename Real>
__device__ __forceinline__ Real buf_load(const TrajRsrc &tr, int voff, int soff);
template <>
__device__ __forceinline__ double buf_load<double>(const TrajRsrc &tr, int voff, int soff) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(tr.r, voff, soff, 0);
  double d;
  __builtin_memcpy(&d, &v, sizeof(d));
  return d;
}
template <>
__device__ __forceinline__ float buf_load<float>(const TrajRsrc &tr, int voff, int soff) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b32(tr.r, voff, soff, 0);
  float f;
  __builtin_memcpy(&f, &v, sizeof(f));
  return f;
}

// Stage block (t, s) into xe, as load_base.
template <typename Real, int E>
__device__ __forceinline__ void load_base_buf(const TrajRsrc &tr, int t, int s, int l,
                                              Real (&xe)[E + 4]) {
  const int blk = (t * 4 + s) * (E + 4) * tr.row_bytes;
  const int voff = l * (int)sizeof(Real);
#pragma unroll
  for (int j = 0; j < E; ++j) xe[2 + j] = buf_load<Real>(tr, voff, blk + j * tr.row_bytes);
  xe[0] = buf_load<Real>(tr, voff, blk + (E + 0) * tr.row_bytes);
  xe[1] = buf_load<Real>(tr, voff, blk + (E + 1) * tr.row_bytes);
  xe[E + 2] = buf_load<Real>(tr, voff, blk + (E + 2) * tr.row_bytes);
  xe[E + 3] = buf_load<Real>(tr, voff, blk + (E + 3) * tr.row_bytes);
}

// d = J(x) e : (J e)_i = (e_{i+1} - e_{i-2}) x_{i-1} + (x_{i+1} - x_{i-2}) e_{i-1} - e_i
template <typename Real, int E>
__device__ __forceinline__ void tl_jac(const Real (&xe)[E + 4], const Real (&e)[E], Real hl2,
                                       Real hl1, Real hr1, Real (&d)[E]) {
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const Real em2 = (j >= 2) ? e[j - 2] : (j == 0 ? hl2 : hl1);
    const Real em1 = (j >= 1) ? e[j - 1] : hl1;
    const Real ep1 = (j + 1 < E) ? e[j + 1] : hr1;
    d[j] = (ep1 - em2) * xe[j + 1] + (xe[j + 3] - xe[j]) * em1 - e[j];
  }
}

// s = J(x)^T w : (J^T w)_i = x_{i-2} w_{i-1} - x_{i+1} w_{i+2} + (x_{i+2} - x_{i-1}) w_{i+1} - w_i
template <typename Real, int E>
__device__ __forceinline__ void ad_jac(const Real (&xe)[E + 4], const Real (&w)[E], Real hl1,
                                       Real hr1, Real hr2, Real (&s)[E]) {
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const Real wm1 = (j >= 1) ? w[j - 1] : hl1;
    const Real wp1 = (j + 1 < E) ? w[j + 1] : hr1;
    const Real wp2 = (j + 2 < E) ? w[j + 2] : (j + 2 == E ? hr1 : hr2);
    s[j] = xe[j] * wm1 - xe[j + 3] * wp2 + (xe[j + 4] - xe[j + 1]) * wp1 - w[j];
  }
}

// Nonlinear tendency on the extended state: f_i = (x_{i+1} - x_{i-2}) x_{i-1} - x_i + F
template <int E>
__device__ __forceinline__ void tendency(const double (&xe)[E + 4], double F, double (&f)[E]) {
#pragma unroll
  for (int j = 0; j < E; ++j) f[j] = (xe[j + 3] - xe[j]) * xe[j + 1] - xe[j + 2] + F;
}

template <typename Real>
__device__ __forceinline__ const Real *stage_block(const ModelView &mv, int t, int s) {
  return reinterpret_cast<const Real *>(mv.xs) +
         (size_t)(t * 4 + s) * (size_t)(mv.E + 4) * (size_t)mv.NT;
}

// ---------------------------------------------------------------------------
// Nonlinear trajectory (one workgroup).
// ---------------------------------------------------------------------------

template <int E>
__device__ void store_block(double *xs64, float *xs32, int t, int s, int E_, int NT, int l,
                            const double (&v)[E], double hl2, double hl1, double hr1, double hr2) {
  const size_t base = (size_t)(t * 4 + s) * (size_t)(E_ + 4) * NT;
  gmem<double> *b = gptr(xs64 + base);
#pragma unroll
  for (int j = 0; j < E; ++j) b[j * NT + l] = v[j];
  b[(E + 0) * NT + l] = hl2;
  b[(E + 1) * NT + l] = hl1;
  b[(E + 2) * NT + l] = hr1;
  b[(E + 3) * NT + l] = hr2;
  if (xs32) {
    gmem<float> *c = gptr(xs32 + base);
#pragma unroll
    for (int j = 0; j < E; ++j) c[j * NT + l] = (float)v[j];
    c[(E + 0) * NT + l] = (float)hl2;
    c[(E + 1) * NT + l] = (float)hl1;
    c[(E + 2) * NT + l] = (float)hr1;
    c[(E + 3) * NT + l] = (float)hr2;
  }
}

// The same stores through buffer resources over the whole trajectory: the block and row
// offsets are scalars (SGPR soffset) and the lane offset one VGPR, so no 64-bit address is
// formed per store. Used when the trajectory is below 2^31 bytes.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
struct TrajStore {
  __amdgpu_buffer_rsrc_t r64, r32;
  bool has32;
};
template <int E>
__device__ __forceinline__ void store_block_buf(const TrajStore &ts, int t, int s, int NT, int l,
                                                const double (&v)[E], double hl2, double hl1,
                                                double hr1, double hr2) {
  const int row0 = (t * 4 + s) * (E + 4);
  auto st64 = [&](int row, double x) {
    u32x2 d;
    __builtin_memcpy(&d, &x, sizeof(d));
    __builtin_amdgcn_raw_buffer_store_b64(d, ts.r64, l * 8, (row0 + row) * NT * 8, 0);
  };
  auto st32 = [&](int row, double x) {
    const float f = (float)x;
    unsigned u;
    __builtin_memcpy(&u, &f, sizeof(u));
    __builtin_amdgcn_raw_buffer_store_b32(u, ts.r32, l * 4, (row0 + row) * NT * 4, 0);
  };
#pragma unroll
  for (int j = 0; j < E; ++j) st64(j, v[j]);
  st64(E + 0, hl2);
  st64(E + 1, hl1);
  st64(E + 2, hr1);
  st64(E + 3, hr2);
  if (ts.has32) {
#pragma unroll
    for (int j = 0; j < E; ++j) st32(j, v[j]);
    st32(E + 0, hl2);
    st32(E + 1, hl1);
    st32(E + 2, hr1);
    st32(E + 3, hr2);
  }
}

// xu != nullptr: one workgroup per initial state (x0 + blockIdx.x n), no stage blocks; the
// state at every observed (step, variable) pair u is written to xu[blockIdx.x U + u].
template <int E>
__device__ __forceinline__ void sample_obs(const ModelView &mv, int t, int l,
                                           const double (&x)[E], double *__restrict__ xu) {
  const int k = gptr(mv.stepk)[t];
  if (k < 0) return;
  const int us = gptr(mv.ustart)[k * mv.NT + l];
  const unsigned mask = (unsigned)gptr(mv.umask)[k * mv.NT + l];
#pragma unroll
  for (int j = 0; j < E; ++j)
    if ((mask >> j) & 1u) gptr(xu)[us + __popc(mask & ((1u << j) - 1u))] = x[j];
}

template <int E>
__global__ void __launch_bounds__(E >= 8 ? 512 : 1024)
    trajectory_kernel(ModelView mv, int nsteps, const double *__restrict__ x0,
                      double *__restrict__ xout, double *__restrict__ xs64,
                      float *__restrict__ xs32, const TrajJob *__restrict__ jobs,
                      double *__restrict__ xu) {
  if (jobs) {  // batched: one workgroup per problem (blockDim may exceed the problem's NT)
    const TrajJob &J = jobs[blockIdx.x];
    mv = J.mv, nsteps = J.mv.T, x0 = J.x0, xout = nullptr, xs64 = J.xs64, xs32 = J.xs32;
  }
  if (xu) {
    x0 += (size_t)blockIdx.x * mv.n;
    xu += (size_t)blockIdx.x * mv.U;
  }
  extern __shared__ double lds_d[];
  const int l = threadIdx.x;
  const int NT = mv.NT;
  const bool active = l < mv.A;
  const int a = l * E;
  HaloMap<E> hm;
  if (active) hm.init(l, mv.n, NT);
  int parity = 0;
  const double h = mv.h, F = mv.F;
  double x[E], xs[E], acc[E], k[E], xe[E + 4];
  double hl2 = 0, hl1 = 0, hr1 = 0, hr2 = 0;
  // the stage blocks through buffer stores when the whole trajectory fits a 2^31-byte resource
  const long long traj_bytes = (long long)(nsteps + 1) * 4 * (E + 4) * NT * (long long)sizeof(double);
  const bool bufst = xs64 != nullptr && !jobs && traj_bytes <= 0x7fffffffLL;
  TrajStore tst;
  tst.has32 = xs32 != nullptr;
  if (bufst) {
    tst.r64 = __builtin_amdgcn_make_buffer_rsrc(xs64, (short)0, (int)traj_bytes, 0x00020000);
    tst.r32 = __builtin_amdgcn_make_buffer_rsrc(tst.has32 ? (void *)xs32 : (void *)xs64, (short)0,
                                                (int)(traj_bytes / 2), 0x00020000);
  }
  auto store_blk = [&](int t, int sidx, const double (&v)[E]) __attribute__((always_inline)) {
    if (bufst)
      store_block_buf<E>(tst, t, sidx, NT, l, v, hl2, hl1, hr1, hr2);
    else
      store_block<E>(xs64, xs32, t, sidx, E, NT, l, v, hl2, hl1, hr1, hr2);
  };
#pragma unroll
  for (int j = 0; j < E; ++j) x[j] = active ? gptr(x0)[a + j] : 0.0;

  auto build = [&](const double (&v)[E]) {
    xe[0] = hl2;
    xe[1] = hl1;
#pragma unroll
    for (int j = 0; j < E; ++j) xe[2 + j] = v[j];
    xe[E + 2] = hr1;
    xe[E + 3] = hr2;
  };

  if constexpr (E >= 8) {
    if (!jobs && !xu && mv.A == NT) {
      // One full problem: each stage computes its four boundary elements first and publishes
      // the next stage's boundary values before the interior elements and the block's
      // stores, so the halo exchange's LDS round trip overlaps that work. The same
      // expressions as the general loop below, so the same results bit for bit.
      auto publish = [&](const double (&v)[E]) __attribute__((always_inline)) {
        double *bb = lds_d + parity * kLdsSlots * NT;
        bb[0 * NT + l] = v[0];
        bb[1 * NT + l] = v[1];
        bb[2 * NT + l] = v[E - 2];
        bb[3 * NT + l] = v[E - 1];
      };
      auto receive = [&]() __attribute__((always_inline)) {
        __syncthreads();
        const double *bb = lds_d + parity * kLdsSlots * NT;
        hl2 = bb[hm.off[0]];
        hl1 = bb[hm.off[1]];
        hr1 = bb[hm.off[2]];
        hr2 = bb[hm.off[3]];
        parity ^= 1;
      };
      auto store_xe = [&](int t, int sidx) __attribute__((always_inline)) {
        double cur[E];
#pragma unroll
        for (int j = 0; j < E; ++j) cur[j] = xe[2 + j];
        store_blk(t, sidx, cur);
      };
      // stage update of element j: c1 = first stage (acc = k), cw = weight of k in acc,
      // cn = coefficient of k in the next state, to4 = the final stage (the next state is x)
#define RIOT_TRAJ_ELEM(J, FIRST, CW, CN, LAST)                                   \
  {                                                                              \
    const int j_ = (J);                                                          \
    k[j_] = (xe[j_ + 3] - xe[j_]) * xe[j_ + 1] - xe[j_ + 2] + F;                 \
    if (FIRST)                                                                   \
      acc[j_] = k[j_];                                                           \
    else if (LAST)                                                               \
      acc[j_] += k[j_];                                                          \
    else                                                                         \
      acc[j_] += 2.0 * k[j_];                                                    \
    if (LAST)                                                                    \
      x[j_] = x[j_] + (h / 6.0) * acc[j_];                                       \
    else                                                                         \
      xs[j_] = x[j_] + (CN) * k[j_];                                             \
  }
#define RIOT_TRAJ_STAGE(T_, SIDX, FIRST, CN, LAST)                               \
  {                                                                              \
    receive();                                                                   \
    if (SIDX == 0) build(x); else build(xs);                                     \
    _Pragma("unroll") for (int b_ = 0; b_ < 4; ++b_)                             \
        RIOT_TRAJ_ELEM(b_ < 2 ? b_ : E - 4 + b_, FIRST, 0, CN, LAST)             \
    if (LAST) publish(x); else publish(xs);                                      \
    if (xs64) store_xe(T_, SIDX);                                                \
    _Pragma("unroll") for (int j2 = 2; j2 < E - 2; ++j2)                         \
        RIOT_TRAJ_ELEM(j2, FIRST, 0, CN, LAST)                                   \
  }
      publish(x);
      for (int t = 0; t < nsteps; ++t) {
        RIOT_TRAJ_STAGE(t, 0, true, 0.5 * h, false)
        RIOT_TRAJ_STAGE(t, 1, false, 0.5 * h, false)
        RIOT_TRAJ_STAGE(t, 2, false, h, false)
        RIOT_TRAJ_STAGE(t, 3, false, 0.0, true)
      }
#undef RIOT_TRAJ_STAGE
#undef RIOT_TRAJ_ELEM
      if (xs64) {
        receive();
        store_blk(nsteps, 0, x);
      }
      if (xout) {
#pragma unroll
        for (int j = 0; j < E; ++j) gptr(xout)[a + j] = x[j];
      }
      return;
    }
  }
  for (int t = 0; t < nsteps; ++t) {
    if (xu && active) sample_obs<E>(mv, t, l, x, xu);
    // stage 1
    exchange<double, E>(lds_d, parity, NT, l, active, hm, x, hl2, hl1, hr1, hr2);
    if (active) {
      build(x);
      if (xs64) store_blk(t, 0, x);
      tendency<E>(xe, F, k);
#pragma unroll
      for (int j = 0; j < E; ++j) {
        acc[j] = k[j];
        xs[j] = x[j] + (0.5 * h) * k[j];
      }
    }
    // stage 2
    exchange<double, E>(lds_d, parity, NT, l, active, hm, xs, hl2, hl1, hr1, hr2);
    if (active) {
      build(xs);
      if (xs64) store_blk(t, 1, xs);
      tendency<E>(xe, F, k);
#pragma unroll
      for (int j = 0; j < E; ++j) {
        acc[j] += 2.0 * k[j];
        xs[j] = x[j] + (0.5 * h) * k[j];
      }
    }
    // stage 3
    exchange<double, E>(lds_d, parity, NT, l, active, hm, xs, hl2, hl1, hr1, hr2);
    if (active) {
      build(xs);
      if (xs64) store_blk(t, 2, xs);
      tendency<E>(xe, F, k);
#pragma unroll
      for (int j = 0; j < E; ++j) {
        acc[j] += 2.0 * k[j];
        xs[j] = x[j] + h * k[j];
      }
    }
    // stage 4
    exchange<double, E>(lds_d, parity, NT, l, active, hm, xs, hl2, hl1, hr1, hr2);
    if (active) {
      build(xs);
      if (xs64) store_blk(t, 3, xs);
      tendency<E>(xe, F, k);
#pragma unroll
      for (int j = 0; j < E; ++j) {
        acc[j] += k[j];
        x[j] = x[j] + (h / 6.0) * acc[j];
      }
    }
  }
  if (xu && active) sample_obs<E>(mv, nsteps, l, x, xu);
  if (xs64) {
    exchange<double, E>(lds_d, parity, NT, l, active, hm, x, hl2, hl1, hr1, hr2);
    if (active) store_blk(nsteps, 0, x);
  }
  if (xout && active) {
#pragma unroll
    for (int j = 0; j < E; ++j) gptr(xout)[a + j] = x[j];
  }
}

// ---------------------------------------------------------------------------
// Member TL/AD sweep (device function shared by the batched kernel and CG).
// ---------------------------------------------------------------------------

// FULL: every thread of the member owns state (n = E * NT), so the activity tests compile
// away and each RK4 stage is one straight-line block.
template <typename Real, int E, bool WAVE = false, bool FULL = false>
struct Member {
  const ModelView &mv;
  Real *lds;
  int l, NT;
  bool active;
  HaloMap<E> hm;
  int parity;

  __device__ Member(const ModelView &m, Real *lds_, int l_)
      : mv(m), lds(lds_), l(l_), NT(m.NT), active(FULL || l_ < m.A), parity(0) {
    if (active) hm.init(l, mv.n, NT);
  }

  // TL of one observed step: f[u] = wgt[u] * dx_i (weighted) or dx_i for observed elements.
  __device__ __forceinline__ void tl_store(int k, const Real (&dl)[E], Real *__restrict__ f,
                                           bool weighted) {
    const int us = mv.ustart[k * NT + l];
    const unsigned mask = (unsigned)mv.umask[k * NT + l];
    const Real *wgt = reinterpret_cast<const Real *>(mv.wgt);
#pragma unroll
    for (int j = 0; j < E; ++j) {
      if ((mask >> j) & 1u) {
        const int u = us + __popc(mask & ((1u << j) - 1u));
        f[u] = weighted ? wgt[u] * dl[j] : dl[j];
      }
    }
  }

  __device__ __forceinline__ void ad_inject(int k, Real (&lam)[E], const Real *__restrict__ f) {
    const int us = mv.ustart[k * NT + l];
    const unsigned mask = (unsigned)mv.umask[k * NT + l];
#pragma unroll
    for (int j = 0; j < E; ++j) {
      if ((mask >> j) & 1u) {
        const int u = us + __popc(mask & ((1u << j) - 1u));
        lam[j] += f[u];
      }
    }
  }

  // Tangent-linear sweep from dl (in registers) over the whole window, storing forcing.
  __device__ void tl_sweep(Real (&dl)[E], Real *__restrict__ f, bool weighted, bool skip0) {
    const Real h = (Real)mv.h;
    const Real h2 = (Real)(0.5 * mv.h);
    const Real h6 = (Real)(mv.h / 6.0);
    Real xe[E + 4], e[E], d[E], acc[E];
    Real hl2 = 0, hl1 = 0, hr1 = 0, hr2 = 0;
    const TrajRsrc tr = traj_rsrc<Real>(mv);
    for (int t = 0; t <= mv.T; ++t) {
      const int k = mv.stepk[t];
      if (k >= 0 && active && !(skip0 && t == 0)) tl_store(k, dl, f, weighted);
      if (t == mv.T) break;
      // stage 1
      load_base_buf<Real, E>(tr, t, 0, l, xe);
      exchange<Real, E, WAVE>(lds, parity, NT, l, active, hm, dl, hl2, hl1, hr1, hr2);
      if (active) {
        tl_jac<Real, E>(xe, dl, hl2, hl1, hr1, d);
#pragma unroll
        for (int j = 0; j < E; ++j) {
          acc[j] = d[j];
          e[j] = dl[j] + h2 * d[j];
        }
      }
      // stage 2
      load_base_buf<Real, E>(tr, t, 1, l, xe);
      exchange<Real, E, WAVE>(lds, parity, NT, l, active, hm, e, hl2, hl1, hr1, hr2);
      if (active) {
        tl_jac<Real, E>(xe, e, hl2, hl1, hr1, d);
#pragma unroll
        for (int j = 0; j < E; ++j) {
          acc[j] += (Real)2 * d[j];
          e[j] = dl[j] + h2 * d[j];
        }
      }
      // stage 3
      load_base_buf<Real, E>(tr, t, 2, l, xe);
      exchange<Real, E, WAVE>(lds, parity, NT, l, active, hm, e, hl2, hl1, hr1, hr2);
      if (active) {
        tl_jac<Real, E>(xe, e, hl2, hl1, hr1, d);
#pragma unroll
        for (int j = 0; j < E; ++j) {
          acc[j] += (Real)2 * d[j];
          e[j] = dl[j] + h * d[j];
        }
      }
      // stage 4
      load_base_buf<Real, E>(tr, t, 3, l, xe);
      exchange<Real, E, WAVE>(lds, parity, NT, l, active, hm, e, hl2, hl1, hr1, hr2);
      if (active) {
        tl_jac<Real, E>(xe, e, hl2, hl1, hr1, d);
#pragma unroll
        for (int j = 0; j < E; ++j) {
          acc[j] += d[j];
          dl[j] = dl[j] + h6 * acc[j];
        }
      }
    }
  }

  // Adjoint sweep over the whole window with forcing f injected at observed steps.
  __device__ void ad_sweep(Real (&lam)[E], const Real *__restrict__ f, bool skip0, bool init) {
    const Real h = (Real)mv.h;
    const Real h2 = (Real)(0.5 * mv.h);
    const Real h3 = (Real)(mv.h / 3.0);
    const Real h6 = (Real)(mv.h / 6.0);
    Real xe[E + 4], lp[E], a[E], s[E];
    Real hl2 = 0, hl1 = 0, hr1 = 0, hr2 = 0;
    const TrajRsrc tr = traj_rsrc<Real>(mv);
    if (!init) {
#pragma unroll
      for (int j = 0; j < E; ++j) lam[j] = 0;
    }
    for (int t = mv.T; t >= 0; --t) {
      const int k = mv.stepk[t];
      if (k >= 0 && active && !(skip0 && t == 0)) ad_inject(k, lam, f);
      if (t == 0) break;
      const int ts = t - 1;
      // adjoint of stage 4 input
      if (active) {
#pragma unroll
        for (int j = 0; j < E; ++j) {
          lp[j] = lam[j];
          a[j] = h6 * lp[j];
        }
      }
      load_base_buf<Real, E>(tr, ts, 3, l, xe);
      exchange<Real, E, WAVE>(lds, parity, NT, l, active, hm, a, hl2, hl1, hr1, hr2);
      if (active) {
        ad_jac<Real, E>(xe, a, hl1, hr1, hr2, s);
#pragma unroll
        for (int j = 0; j < E; ++j) {
          lam[j] = lp[j] + s[j];
          a[j] = h3 * lp[j] + h * s[j];
        }
      }
      // stage 3
      load_base_buf<Real, E>(tr, ts, 2, l, xe);
      exchange<Real, E, WAVE>(lds, parity, NT, l, active, hm, a, hl2, hl1, hr1, hr2);
      if (active) {
        ad_jac<Real, E>(xe, a, hl1, hr1, hr2, s);
#pragma unroll
        for (int j = 0; j < E; ++j) {
          lam[j] += s[j];
          a[j] = h3 * lp[j] + h2 * s[j];
        }
      }
      // stage 2
      load_base_buf<Real, E>(tr, ts, 1, l, xe);
      exchange<Real, E, WAVE>(lds, parity, NT, l, active, hm, a, hl2, hl1, hr1, hr2);
      if (active) {
        ad_jac<Real, E>(xe, a, hl1, hr1, hr2, s);
#pragma unroll
        for (int j = 0; j < E; ++j) {
          lam[j] += s[j];
          a[j] = h6 * lp[j] + h2 * s[j];
        }
      }
      // stage 1
      load_base_buf<Real, E>(tr, ts, 0, l, xe);
      exchange<Real, E, WAVE>(lds, parity, NT, l, active, hm, a, hl2, hl1, hr1, hr2);
      if (active) {
        ad_jac<Real, E>(xe, a, hl1, hr1, hr2, s);
#pragma unroll
        for (int j = 0; j < E; ++j) lam[j] += s[j];
      }
    }
  }

  // One member. Base mode (mode & 7): 0 = TL (R^{-1}-weighted store) then AD -> lam0;
  // 1 = AD forced by the shared fsrc -> lam0; 2 = TL only, raw observed values into f;
  // 3 = AD forced by this member's own f -> lam0. Flags: kTladSkip0 = no store or injection
  // at the window's step 0 (a checkpoint segment after the first, whose step 0 is the
  // previous segment's last step); kTladInitLam = the AD starts from dx0 instead of zero;
  // kTladOutState = mode 2 writes the final tangent state into lam0. dx0 and lam0 use the
  // natural layout (double).
  // FLAGS = false compiles the flag tests out (the single-window hot path, whose register
  // budget is full at 16 elements per lane).
  template <bool FLAGS = true>
  __device__ void run(int mode, const double *__restrict__ dx0, double *__restrict__ lam0,
                      Real *__restrict__ f, const Real *__restrict__ fsrc) {
    const int base = FLAGS ? (mode & 7) : mode;
    const bool skip0 = FLAGS && (mode & kTladSkip0) != 0;
    const int a = l * E;
    Real v[E];
    if (base == 0 || base == 2) {
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = active ? (Real)dx0[a + j] : (Real)0;
      tl_sweep(v, f, base == 0, skip0);
      if (base == 2) {
        if (FLAGS && (mode & kTladOutState) && active) {
#pragma unroll
          for (int j = 0; j < E; ++j) lam0[a + j] = (double)v[j];
        }
        return;
      }
      // each forcing value is re-read by the thread that stored it; the barrier only
      // separates the two sweeps' LDS traffic
      member_sync<WAVE>();
      ad_sweep(v, f, skip0, false);
    } else {
      const bool init = FLAGS && (mode & kTladInitLam) != 0;
      if (init) {
#pragma unroll
        for (int j = 0; j < E; ++j) v[j] = active ? (Real)dx0[a + j] : (Real)0;
      }
      ad_sweep(v, base == 1 ? fsrc : f, skip0, init);
    }
    if (active) {
#pragma unroll
      for (int j = 0; j < E; ++j) lam0[a + j] = (double)v[j];
    }
  }
};

template <typename Real, int E, bool FLAGS, bool FULL>
__global__ void __launch_bounds__(E >= 8 ? 512 : 1024)
    tlad_kernel(ModelView mv, int mode, const double *__restrict__ dx0, double *__restrict__ lam0,
                Real *__restrict__ f, const Real *__restrict__ fsrc) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  Real *lds = reinterpret_cast<Real *>(lds_raw);
  const int mem = blockIdx.x;
  Member<Real, E, false, FULL> M(mv, lds, threadIdx.x);
  M.template run<FLAGS>(mode, dx0 + (size_t)mem * mv.n, lam0 + (size_t)mem * mv.n,
                        f + (size_t)mem * (size_t)mv.U, fsrc);
}

// ---------------------------------------------------------------------------
// TL/AD sweep with the base states staged through LDS (full members, E = 16, 256 threads per
// member, two members per workgroup).
//
// Every RK4 stage reads one stage block of the stored trajectory. Loading it into registers
// when the stage starts leaves the L2 latency on each stage's critical path (one member per
// compute unit is a single wave per SIMD, with nothing else to switch to). Here the first E
// rows of each block (the lane-interleaved own values; the four halo rows are the
// neighbours' rows) are copied straight into a ring of four LDS slots with direct-to-LDS
// loads (buffer_load_dwordx4 ... lds, no VGPRs), three stages before they are read: the TL
// walks the blocks forward and refills, after each stage's barrier, the slot the previous
// stage read with the block three ahead; the AD walks them backward the same way. Each wave
// waits with s_waitcnt vmcnt for its own copies of the block it is about to read, and the
// stage's halo barrier then covers the other waves' copies. The barriers are plain
// s_barrier (a __syncthreads fence would wait for every copy in flight), and the LDS
// pointers of one stage are restrict-qualified so the compiler does not add such a wait
// either. Two members share the ring and each barrier (their base states are the same), one
// wave of each per SIMD, so that each SIMD has a second wave to issue while one waits. The
// arithmetic is that of Member (same order, same results), except that R^{-1} is applied
// when the AD injects an observed value instead of when the TL stores it (the same product).
// ---------------------------------------------------------------------------

constexpr int kRingSlots = 4;
constexpr int kRingNT = 256;   // threads per member (n = 16 * 256 = 4096)
constexpr int kRingMembers = 2;  // members per workgroup, one group of waves each

#define RIOT_LDSP(p) ((__attribute__((address_space(3))) void *)(p))

// Wait until at most `later` fill groups (of K copies each) issued after the wanted one are
// still in flight (later >= 2 is treated as 2, which only waits longer).
template <int K>
__device__ __forceinline__ void ring_wait(int later) {
  static_assert(K == 2 || K == 4, "fill group size");
  if (later >= 2) {
    if constexpr (K == 4) asm volatile("s_waitcnt vmcnt(8)" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(4)" ::: "memory");
  } else if (later == 1) {
    if constexpr (K == 4) asm volatile("s_waitcnt vmcnt(4)" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(2)" ::: "memory");
  } else {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
}

__device__ __forceinline__ void raw_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <typename Real, int E>
struct MemberRing {
  static constexpr int NT = kRingNT;
  static constexpr int WGT = kRingMembers * NT;           // threads per workgroup
  static constexpr int per = 16 / (int)sizeof(Real);     // Reals per lane per copy
  static constexpr int K = E * NT / (WGT * per);           // copies per stage block and thread
  static constexpr int SLOT = E * NT;                      // Reals per slot
  const ModelView &mv;
  Real *xch;      // this member's halo exchange, 2 parities x kLdsSlots x NT
  Real *ring;     // kRingSlots slots of E x NT, shared by the workgroup's members
  int l, parity;  // l: lane within the member
  int lm, lp;     // neighbour lanes (periodic)
  int wv;         // wave index within the workgroup, read into a scalar register
  unsigned voff;  // this thread's byte offset inside one copy of 16 bytes per thread
  HaloMap<E> hm;
  TrajRsrc tr;
  int blk_bytes;  // bytes per stored stage block, (E + 4) NT sizeof(Real)
  int nblk;       // 4 T stage blocks per sweep
  // the observation tables, read-only for the whole launch (kernel arguments declared
  // __restrict__, so that the uniform step table is read by scalar loads and no read of
  // them waits on the ring copies in flight)
  const int *__restrict__ stepk;
  const int *__restrict__ ustart;
  const int *__restrict__ umask;
  const Real *__restrict__ wgt;

  __device__ MemberRing(const ModelView &m, Real *xch_, Real *ring_, int tid,
                        const int *__restrict__ stepk_, const int *__restrict__ ustart_,
                        const int *__restrict__ umask_, const Real *__restrict__ wgt_)
      : mv(m), xch(xch_), ring(ring_), l(tid % NT), parity(0), stepk(stepk_), ustart(ustart_),
        umask(umask_), wgt(wgt_) {
    hm.init(l, mv.n, NT);
    lm = (l + NT - 1) % NT;
    lp = (l + 1) % NT;
    wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    voff = (unsigned)tid * 16u;
    tr = traj_rsrc<Real>(mv);
    blk_bytes = (E + 4) * NT * (int)sizeof(Real);
    nblk = 4 * mv.T;
  }

  // Copy the first E rows (the own values, E x NT) of stage block b into slot F: K copies of
  // 16 bytes per thread over the whole workgroup, straight into LDS (buffer_load_dwordx4 ...
  // lds, no VGPR destination).
  template <int F>
  __device__ __forceinline__ void fill(int b) {
    Real *dst = ring + F * SLOT + wv * 64 * per;
#pragma unroll
    for (int i = 0; i < K; ++i)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(tr.r, RIOT_LDSP(dst + i * WGT * per), 16, voff,
                                               (unsigned)(b * blk_bytes + i * WGT * 16), 0, 0);
  }

  // One stage: wait for this stage's block in slot S (`later` = fills issued after it that
  // may still be in flight), publish the boundary values, barrier, refill slot F with block
  // `next` (when 0 <= next < nblk; slot F was read one stage earlier), then read the
  // neighbours' values and the base state from LDS.
  template <int S, int F>
  __device__ __forceinline__ void stage_in(int later, int next, const Real (&v)[E], Real &hl2,
                                           Real &hl1, Real &hr1, Real &hr2, Real (&xe)[E + 4]) {
    ring_wait<K>(later);
    stage_io<F>(ring + S * SLOT, xch + parity * kLdsSlots * NT, next, v, hl2, hl1, hr1, hr2, xe);
    parity ^= 1;
  }

  template <int F>
  __device__ __forceinline__ void stage_io(const Real *__restrict__ slot, Real *__restrict__ x,
                                           int next, const Real (&v)[E], Real &hl2, Real &hl1,
                                           Real &hr1, Real &hr2, Real (&xe)[E + 4]) {
    x[0 * NT + l] = v[0];
    x[1 * NT + l] = v[1];
    x[2 * NT + l] = v[E - 2];
    x[3 * NT + l] = v[E - 1];
    raw_barrier();
    if (next >= 0 && next < nblk) fill<F>(next);
    hl2 = x[hm.off[0]];
    hl1 = x[hm.off[1]];
    hr1 = x[hm.off[2]];
    hr2 = x[hm.off[3]];
#pragma unroll
    for (int j = 0; j < E; ++j) xe[2 + j] = slot[j * NT + l];
    xe[0] = slot[(E - 2) * NT + lm];
    xe[1] = slot[(E - 1) * NT + lm];
    xe[E + 2] = slot[0 * NT + lp];
    xe[E + 3] = slot[1 * NT + lp];
  }

  // The TL stores the raw observed values and the AD applies R^{-1} as it injects them (the
  // same single product as weighting at the store): the TL then only stores, and never
  // waits on a load, which would also wait for the ring copies in flight.
  __device__ __forceinline__ void tl_store(int k, const Real (&dl)[E], Real *__restrict__ f) {
    const int us = ustart[k * NT + l];
    const unsigned mask = (unsigned)umask[k * NT + l];
#pragma unroll
    for (int j = 0; j < E; ++j) {
      if ((mask >> j) & 1u) {
        const int u = us + __popc(mask & ((1u << j) - 1u));
        f[u] = dl[j];
      }
    }
  }

  __device__ __forceinline__ void ad_inject(int k, Real (&lam)[E], const Real *__restrict__ f) {
    const int us = ustart[k * NT + l];
    const unsigned mask = (unsigned)umask[k * NT + l];
#pragma unroll
    for (int j = 0; j < E; ++j) {
      if ((mask >> j) & 1u) {
        const int u = us + __popc(mask & ((1u << j) - 1u));
        lam[j] += wgt[u] * f[u];
      }
    }
  }

  // Fill-order bookkeeping. TL: blocks 0, 1, 2 before the sweep, then block b + 3 at stage b,
  // so fills after block b's: min(2, nblk - 1 - b). AD (blocks nblk-1 .. 0): block b - 3 at
  // stage b; the first block's fill is the TL's last (nothing after it), every other block
  // has at least min(2, b) fills after its own.
  __device__ __forceinline__ int later_tl(int b) const { return min(2, nblk - 1 - b); }
  __device__ __forceinline__ int later_ad(int b) const { return b == nblk - 1 ? 0 : min(2, b); }

  // TL over the window (R^{-1}-weighted observed values into f), then the AD forced by them.
  __device__ void run(const double *__restrict__ dx0, double *__restrict__ lam0,
                      Real *__restrict__ f) {
    const int a = l * E;
    const Real h = (Real)mv.h;
    const Real h2 = (Real)(0.5 * mv.h);
    const Real h3 = (Real)(mv.h / 3.0);
    const Real h6 = (Real)(mv.h / 6.0);
    Real dl[E], e[E], d[E], acc[E], xe[E + 4];
    Real hl2, hl1, hr1, hr2;
#pragma unroll
    for (int j = 0; j < E; ++j) dl[j] = (Real)dx0[a + j];
    fill<0>(0);
    if (nblk > 1) fill<1>(1);
    if (nblk > 2) fill<2>(2);
    // tangent-linear sweep, blocks 0 .. 4T-1 (block 4t + s in slot s)
    for (int t = 0; t <= mv.T; ++t) {
      const int k = stepk[t];
      if (k >= 0) tl_store(k, dl, f);
      if (t == mv.T) break;
      const int b0 = 4 * t;
      stage_in<0, 3>(later_tl(b0), b0 + 3, dl, hl2, hl1, hr1, hr2, xe);
      tl_jac<Real, E>(xe, dl, hl2, hl1, hr1, d);
#pragma unroll
      for (int j = 0; j < E; ++j) {
        acc[j] = d[j];
        e[j] = dl[j] + h2 * d[j];
      }
      stage_in<1, 0>(later_tl(b0 + 1), b0 + 4, e, hl2, hl1, hr1, hr2, xe);
      tl_jac<Real, E>(xe, e, hl2, hl1, hr1, d);
#pragma unroll
      for (int j = 0; j < E; ++j) {
        acc[j] += (Real)2 * d[j];
        e[j] = dl[j] + h2 * d[j];
      }
      stage_in<2, 1>(later_tl(b0 + 2), b0 + 5, e, hl2, hl1, hr1, hr2, xe);
      tl_jac<Real, E>(xe, e, hl2, hl1, hr1, d);
#pragma unroll
      for (int j = 0; j < E; ++j) {
        acc[j] += (Real)2 * d[j];
        e[j] = dl[j] + h * d[j];
      }
      stage_in<3, 2>(later_tl(b0 + 3), b0 + 6, e, hl2, hl1, hr1, hr2, xe);
      tl_jac<Real, E>(xe, e, hl2, hl1, hr1, d);
#pragma unroll
      for (int j = 0; j < E; ++j) {
        acc[j] += d[j];
        dl[j] = dl[j] + h6 * acc[j];
      }
    }
    // adjoint sweep, blocks 4T-1 .. 0 (the last three are still in their slots; the first
    // stages refill them with the same data, which no stage reads in between)
    Real (&lam)[E] = dl;
    Real (&lp_)[E] = e;
    Real (&aa)[E] = acc;
    Real (&sv)[E] = d;
#pragma unroll
    for (int j = 0; j < E; ++j) lam[j] = 0;
    for (int t = mv.T; t >= 0; --t) {
      const int k = stepk[t];
      if (k >= 0) ad_inject(k, lam, f);
      if (t == 0) break;
      const int b3 = 4 * (t - 1) + 3;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        lp_[j] = lam[j];
        aa[j] = h6 * lp_[j];
      }
      stage_in<3, 0>(later_ad(b3), b3 - 3, aa, hl2, hl1, hr1, hr2, xe);
      ad_jac<Real, E>(xe, aa, hl1, hr1, hr2, sv);
#pragma unroll
      for (int j = 0; j < E; ++j) {
        lam[j] = lp_[j] + sv[j];
        aa[j] = h3 * lp_[j] + h * sv[j];
      }
      stage_in<2, 3>(later_ad(b3 - 1), b3 - 4, aa, hl2, hl1, hr1, hr2, xe);
      ad_jac<Real, E>(xe, aa, hl1, hr1, hr2, sv);
#pragma unroll
      for (int j = 0; j < E; ++j) {
        lam[j] += sv[j];
        aa[j] = h3 * lp_[j] + h2 * sv[j];
      }
      stage_in<1, 2>(later_ad(b3 - 2), b3 - 5, aa, hl2, hl1, hr1, hr2, xe);
      ad_jac<Real, E>(xe, aa, hl1, hr1, hr2, sv);
#pragma unroll
      for (int j = 0; j < E; ++j) {
        lam[j] += sv[j];
        aa[j] = h6 * lp_[j] + h2 * sv[j];
      }
      stage_in<0, 1>(later_ad(b3 - 3), b3 - 6, aa, hl2, hl1, hr1, hr2, xe);
      ad_jac<Real, E>(xe, aa, hl1, hr1, hr2, sv);
#pragma unroll
      for (int j = 0; j < E; ++j) lam[j] += sv[j];
    }
    // no copy may still be writing LDS when the workgroup ends
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    if (lam0) {
#pragma unroll
      for (int j = 0; j < E; ++j) lam0[a + j] = (double)lam[j];
    }
  }
};

// Two members per workgroup (waves 0-3 and 4-7), one wave of each per SIMD: while one waits
// on LDS or its dependences the SIMD issues the other's. They share the LDS ring (the base
// state is the same for every member) and each barrier. An odd last member is shadowed by a
// copy of the one before it, which computes but writes no result.
template <typename Real, int E>
__global__ void __launch_bounds__(kRingMembers * kRingNT)
    tlad_ring_kernel(ModelView mv, int m, const double *__restrict__ dx0,
                     double *__restrict__ lam0, Real *__restrict__ f,
                     const int *__restrict__ stepk, const int *__restrict__ ustart,
                     const int *__restrict__ umask, const Real *__restrict__ wgt) {
  __shared__ __align__(16) Real ring[kRingSlots * E * kRingNT];
  __shared__ __align__(16) Real xch[kRingMembers * 2 * kLdsSlots * kRingNT];
  const int q = threadIdx.x / kRingNT;
  const int mem = blockIdx.x * kRingMembers + q;
  const int src = mem < m ? mem : m - 1;
  MemberRing<Real, E> M(mv, xch + q * 2 * kLdsSlots * kRingNT, ring, threadIdx.x, stepk, ustart,
                        umask, wgt);
  M.run(dx0 + (size_t)src * mv.n, mem < m ? lam0 + (size_t)mem * mv.n : nullptr,
        f + (size_t)mem * (size_t)mv.U);
}

// ---------------------------------------------------------------------------
// Persistent TL/AD over a batch of independent problems (8 elements per lane). Phase 1:
// each workgroup takes whole-workgroup tiles (one member of a problem with NT > 64) from
// an atomic counter; phase 2: each wave takes member-per-wave tiles (NT <= 64, the halo
// exchanged inside the wave without workgroup barriers) from a second counter. The tile
// lists are in decreasing cost order, so the longest integrations start first and the
// short ones fill the tail. Every wave leaves once both lists are exhausted.
// ---------------------------------------------------------------------------

template <typename Real>
__device__ __forceinline__ void run_tile(int mode, const TladProb &P, int mem, Real *lds, int l,
                                         bool wave_layout) {
  constexpr int E = 8;
  const ModelView mv = P.mv;
  const size_t n = (size_t)mv.n, U = (size_t)mv.U;
  const double *dx0 = P.dx0 ? P.dx0 + (size_t)mem * n : nullptr;
  double *lam0 = P.lam0 ? P.lam0 + (size_t)mem * n : nullptr;
  Real *f = P.f ? reinterpret_cast<Real *>(P.f) + (size_t)mem * U : nullptr;
  const Real *fsrc = reinterpret_cast<const Real *>(P.fsrc);
  if (wave_layout) {
    Member<Real, E, true> M(mv, lds, l);
    M.run(mode, dx0, lam0, f, fsrc);
  } else {
    Member<Real, E, false> M(mv, lds, l);
    M.run(mode, dx0, lam0, f, fsrc);
  }
}

template <typename Real>
__global__ void __launch_bounds__(256)
    tlad_persistent_kernel(int mode, const TladProb *__restrict__ probs,
                           const TladTile *__restrict__ wg_tiles, int n_wg,
                           const TladTile *__restrict__ wave_tiles, int n_wave,
                           int *__restrict__ counters, long long *__restrict__ clk) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  Real *lds = reinterpret_cast<Real *>(lds_raw);
  __shared__ int tile_sh;
  for (;;) {
    if (threadIdx.x == 0) tile_sh = atomicAdd(&counters[0], 1);
    __syncthreads();
    const int t = tile_sh;
    __syncthreads();  // every thread has its tile before thread 0 fetches the next
    if (t >= n_wg) break;
    const TladTile tile = wg_tiles[t];
    const long long c0 = clk ? wall_clock64() : 0;
    run_tile<Real>(mode, probs[tile.prob], tile.mem, lds, threadIdx.x, false);
    __syncthreads();  // the tile's LDS traffic is over before the next tile starts
    if (clk && threadIdx.x == 0) {
      clk[2 * t] = c0;
      clk[2 * t + 1] = wall_clock64();
    }
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  Real *wlds = lds + (size_t)wave * kLdsSlots * 2 * 64;
  for (;;) {
    int t = 0;
    if (lane == 0) t = atomicAdd(&counters[1], 1);
    t = __shfl(t, 0, 64);
    if (t >= n_wave) break;
    const TladTile tile = wave_tiles[t];
    const long long c0 = clk ? wall_clock64() : 0;
    run_tile<Real>(mode, probs[tile.prob], tile.mem, wlds, lane, true);
    if (clk && lane == 0) {
      clk[2 * (n_wg + t)] = c0;
      clk[2 * (n_wg + t) + 1] = wall_clock64();
    }
  }
}

// ---------------------------------------------------------------------------
// Innovation, gradient forcing and cost.
// ---------------------------------------------------------------------------

template <typename Real>
__global__ void innovation_kernel(ModelView mv, const double *__restrict__ xs64, int U,
                                  const int *__restrict__ obs_step, const int *__restrict__ obs_idx,
                                  const double *__restrict__ y, const double *__restrict__ rinv,
                                  const int *__restrict__ u_optr, const int *__restrict__ u_olist,
                                  double *__restrict__ d, Real *__restrict__ fgrad,
                                  const InnovJob *__restrict__ jobs) {
  if (jobs) {  // batched: blockIdx.y selects the problem
    const InnovJob &J = jobs[blockIdx.y];
    mv = J.mv, xs64 = J.xs64, U = J.mv.U, obs_step = J.obs_step, obs_idx = J.obs_idx, y = J.y;
    rinv = J.rinv, u_optr = J.u_optr, u_olist = J.u_olist, d = J.d;
    fgrad = reinterpret_cast<Real *>(J.fgrad);
  }
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= U) return;
  double acc = 0.0;
  for (int q = u_optr[u]; q < u_optr[u + 1]; ++q) {
    const int o = u_olist[q];
    const int t = obs_step[o];
    const int i = obs_idx[o];
    const int l = i / mv.E, j = i - l * mv.E;
    const double xv = xs64[(size_t)(t * 4) * (size_t)(mv.E + 4) * mv.NT + (size_t)j * mv.NT + l];
    const double dv = y[o] - xv;
    d[o] = dv;
    acc += rinv[o] * dv;
  }
  fgrad[u] = (Real)acc;
}

// Observed values of a stored window segment: out[o] = x_t[i] for the observations whose
// step t lies in (lo, lo + T] (and t = lo when include_lo), read from block (t - lo, 0).
__global__ void obs_value_kernel(ModelView mv, const double *__restrict__ xs64, int nobs,
                                 const int *__restrict__ obs_step, const int *__restrict__ obs_idx,
                                 int lo, int include_lo, double *__restrict__ out) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nobs) return;
  const int t = obs_step[o];
  if (t < lo || t > lo + mv.T || (t == lo && !include_lo)) return;
  const int i = obs_idx[o];
  const int l = i / mv.E, j = i - l * mv.E;
  out[o] = xs64[(size_t)((t - lo) * 4) * (size_t)(mv.E + 4) * mv.NT + (size_t)j * mv.NT + l];
}

// Z[o, j] = f_j[u(o)] : raw TL values back in the caller's observation order, multiplied by
// sqrt(rinv[o]) when rinv is given (the R^{-1/2} factor of the dual operator).
template <typename Real>
__global__ void obs_gather_kernel(int nobs, int U, int m, const int *__restrict__ u_of_o,
                                  const Real *__restrict__ f, double *__restrict__ Z,
                                  const double *__restrict__ rinv) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nobs * m) return;
  const int o = (int)(idx % nobs), j = (int)(idx / nobs);
  const double z = (double)f[(size_t)j * U + u_of_o[o]];
  Z[idx] = rinv ? sqrt(rinv[o]) * z : z;
}

// f_j[u] = sum_{o in u} F[o, j] : observation-space forcing folded onto unique pairs (each
// F[o, j] first multiplied by sqrt(rinv[o]) when rinv is given).
template <typename Real>
__global__ void obs_scatter_kernel(int nobs, int U, int m, const int *__restrict__ u_optr,
                                   const int *__restrict__ u_olist, const double *__restrict__ Fo,
                                   Real *__restrict__ f, const double *__restrict__ rinv) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)U * m) return;
  const int u = (int)(idx % U), j = (int)(idx / U);
  double s = 0.0;
  for (int q = u_optr[u]; q < u_optr[u + 1]; ++q) {
    const int o = u_olist[q];
    const double v = Fo[(size_t)j * nobs + o];
    s += rinv ? sqrt(rinv[o]) * v : v;
  }
  f[idx] = (Real)s;
}

// Dual right-hand side and increment scaling: out[o] = sqrt(rinv[o]) (d[o] - bp[o]) (bp may be
// nullptr), and dw[o] = -sqrt(rinv[o]) t[o] (t from the negated low-rank combination).
__global__ void psas_rhs_kernel(int nobs, const double *__restrict__ rinv,
                                const double *__restrict__ d, const double *__restrict__ bp,
                                double *__restrict__ out) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nobs) return;
  out[o] = sqrt(rinv[o]) * (bp ? d[o] - bp[o] : d[o]);
}

// Perturbed observations of one gradient sample: out[o] = y[o] - eps[o] / sqrt(rinv[o]).
__global__ void obs_perturb_kernel(int nobs, const double *__restrict__ y,
                                   const double *__restrict__ rinv, const double *__restrict__ eps,
                                   double *__restrict__ out) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nobs) return;
  out[o] = y[o] - eps[o] / sqrt(rinv[o]);
}

__global__ void psas_scale_kernel(int nobs, const double *__restrict__ rinv,
                                  const double *__restrict__ t, double *__restrict__ dw) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nobs) return;
  dw[o] = -sqrt(rinv[o]) * t[o];
}

__device__ double block_sum(double v, double *red) {
  // wave reduction then cross-wave through LDS, fixed order
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

__global__ void __launch_bounds__(1024)
    cost_kernel(int n, const double *__restrict__ v, int nobs, const double *__restrict__ d,
                const double *__restrict__ rinv, double *__restrict__ out) {
  __shared__ double red[16];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    if (v) a += v[i] * v[i];
  for (int o = threadIdx.x; o < nobs; o += blockDim.x) b += rinv[o] * d[o] * d[o];
  const double sa = block_sum(a, red);
  const double sb = block_sum(b, red);
  if (threadIdx.x == 0) out[0] = 0.5 * sa + 0.5 * sb;
}

// ---------------------------------------------------------------------------
// L (symmetric circulant, half-kernel taps) applied to columns.
// ---------------------------------------------------------------------------

// Workgroup-cooperative L x for one column; ext must hold n + 2w doubles of LDS
// (or be nullptr to read x from global memory with modular indexing).
__device__ void apply_L_column(int n, int w, const double *__restrict__ taps,
                               const double *__restrict__ x, double *__restrict__ y,
                               const double *__restrict__ z, int mode, double *ext) {
  if (ext) {
    for (int k = threadIdx.x; k < n + 2 * w; k += blockDim.x) {
      int src = (k - w) % n;
      if (src < 0) src += n;
      ext[k] = x[src];
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double acc;
    if (ext) {
      acc = taps[0] * ext[i + w];
      for (int dd = 1; dd <= w; ++dd) acc += taps[dd] * (ext[i + w + dd] + ext[i + w - dd]);
    } else {
      acc = taps[0] * x[i];
      for (int dd = 1; dd <= w; ++dd) {
        int ip = (i + dd) % n;
        int im = (i - dd) % n;
        if (im < 0) im += n;
        acc += taps[dd] * (x[ip] + x[im]);
      }
    }
    if (mode == 1)
      acc += z[i];
    else if (mode == 2)
      acc = (z ? z[i] : 0.0) - acc;
    y[i] = acc;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(256)
    apply_L_kernel(int n, int w, const double *__restrict__ taps, const double *__restrict__ X,
                   double *__restrict__ Y, const double *__restrict__ Z, int mode, int use_lds,
                   const ApplyLJobE *__restrict__ jobs) {
  extern __shared__ double ext[];
  const size_t c = blockIdx.x;
  if (jobs) {  // batched: blockIdx.y selects the problem, blockIdx.x the column
    const ApplyLJobE &J = jobs[blockIdx.y];
    if ((int)c >= J.m) return;
    n = J.n, w = J.w, taps = J.taps, X = J.X, Y = J.Y, Z = J.Z, mode = J.mode;
  }
  apply_L_column(n, w, taps, X + c * n, Y + c * n, Z ? Z + c * n : nullptr, mode,
                 use_lds ? ext : nullptr);
}

// The same product for one segment of kLSeg rows of one column per workgroup (grid: column,
// segment): the segment with its w-row halo on each side is staged in LDS, and the sums run
// in the order of apply_L_column, so results are identical. A column split into segments
// gives a block of m columns n / kLSeg times as many workgroups to hide the LDS latency.
constexpr int kLSeg = 1024;

__global__ void __launch_bounds__(256)
    apply_L_seg_kernel(int n, int w, const double *__restrict__ taps, const double *__restrict__ X,
                       double *__restrict__ Y, const double *__restrict__ Z, int mode) {
  extern __shared__ double ext[];
  const size_t c = blockIdx.x;
  const int r0 = blockIdx.y * kLSeg, len = min(kLSeg, n - r0);
  const double *x = X + c * n;
  const int tot = len + 2 * w;
  auto src_of = [&](int k) {
    int src = (r0 + k - w) % n;
    return src < 0 ? src + n : src;
  };
  if (tot <= 6 * 256 && blockDim.x == 256) {
    // the segment's loads all issued before the first wait (one memory latency, not one per
    // round of 256)
    double v[6];
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      const int k = threadIdx.x + 256 * t;
      v[t] = x[src_of(k < tot ? k : 0)];
    }
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      const int k = threadIdx.x + 256 * t;
      if (k < tot) ext[k] = v[t];
    }
  } else {
    for (int k = threadIdx.x; k < tot; k += blockDim.x) ext[k] = x[src_of(k)];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < len; i += blockDim.x) {
    double acc = taps[0] * ext[i + w];
    for (int dd = 1; dd <= w; ++dd) acc += taps[dd] * (ext[i + w + dd] + ext[i + w - dd]);
    const size_t o = c * n + r0 + i;
    if (mode == 1)
      acc += Z[o];
    else if (mode == 2)
      acc = (Z ? Z[o] : 0.0) - acc;
    Y[o] = acc;
  }
}

// ---------------------------------------------------------------------------
// Conjugate gradients: one workgroup, all iterations in one launch.
// ---------------------------------------------------------------------------

template <typename Real, int E>
__global__ void __launch_bounds__(E >= 8 ? 512 : 1024)
    cg_kernel(ModelView mv, int w, const double *__restrict__ taps, const double *__restrict__ g,
              int iters, double rtol, double *__restrict__ x, double *__restrict__ iterates,
              double *__restrict__ vs, Real *__restrict__ f, int *__restrict__ used,
              int ext_off_bytes, int use_lds_ext) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ double red[16];
  Real *lds = reinterpret_cast<Real *>(lds_raw);
  double *ext = use_lds_ext ? reinterpret_cast<double *>(lds_raw + ext_off_bytes) : nullptr;
  const int n = mv.n;
  double *r = vs, *p = vs + n, *q = vs + 2 * n, *tmp = vs + 3 * n, *lam = vs + 4 * n;
  Member<Real, E> M(mv, lds, threadIdx.x);

  double rr_part = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double ri = -g[i];
    x[i] = 0.0;
    r[i] = ri;
    p[i] = ri;
    rr_part += ri * ri;
  }
  double rr = block_sum(rr_part, red);
  const double r0 = sqrt(rr);
  int it = 0;
  for (; it < iters; ++it) {
    // q = (I + A) p = p + L^T G^T R^{-1} G L p
    apply_L_column(n, w, taps, p, tmp, nullptr, 0, ext);
    M.template run<false>(0, tmp, lam, f, nullptr);
    __syncthreads();
    apply_L_column(n, w, taps, lam, q, p, 1, ext);
    double pq_part = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) pq_part += p[i] * q[i];
    const double pq = block_sum(pq_part, red);
    const double alpha = rr / pq;
    double rn_part = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      x[i] += alpha * p[i];
      const double ri = r[i] - alpha * q[i];
      r[i] = ri;
      rn_part += ri * ri;
      if (iterates) iterates[(size_t)it * n + i] = x[i];
    }
    const double rr_new = block_sum(rn_part, red);
    if (rtol > 0.0 && sqrt(rr_new) <= rtol * r0) {
      ++it;
      break;
    }
    const double beta = rr_new / rr;
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = r[i] + beta * p[i];
    rr = rr_new;
    __syncthreads();
  }
  if (threadIdx.x == 0) used[0] = it;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC 2011) and Box-Muller normals.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t p0 = (uint64_t)M0 * c[0];
    const uint64_t p1 = (uint64_t)M1 * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__global__ void philox_normal_kernel(long long total, uint64_t seed, uint64_t stream,
                                     double *__restrict__ out, const PhiloxJob *__restrict__ jobs) {
  if (jobs) {  // batched: blockIdx.y selects the problem (its own stream)
    const PhiloxJob &J = jobs[blockIdx.y];
    total = J.total, stream = J.stream, out = J.out;
  }
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long pairs = (total + 1) / 2;
  if (j >= pairs) return;
  uint32_t c[4] = {(uint32_t)j, (uint32_t)((unsigned long long)j >> 32), (uint32_t)stream,
                   (uint32_t)(stream >> 32)};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t v1 = (((uint64_t)c[1] << 32) | c[0]) >> 11;
  const uint64_t v2 = (((uint64_t)c[3] << 32) | c[2]) >> 11;
  const double u1 = ((double)v1 + 0.5) * 0x1.0p-53;
  const double u2 = ((double)v2 + 0.5) * 0x1.0p-53;
  const double r = sqrt(-2.0 * log(u1));
  const double th = 2.0 * 3.14159265358979323846 * u2;
  out[2 * j] = r * cos(th);
  if (2 * j + 1 < total) out[2 * j + 1] = r * sin(th);
}

// ---------------------------------------------------------------------------
// Deterministic LRA/LRU choice: candidate states, non-quadratic costs, selection.
// ---------------------------------------------------------------------------

// xc[c] = x + dx[c], vc[c] = v + dz[c] (v = nullptr: zero), c = 0 .. nc-1, n-vectors.
__global__ void cand_state_kernel(int n, int nc, const double *__restrict__ x,
                                  const double *__restrict__ v, const double *__restrict__ dz,
                                  const double *__restrict__ dx, double *__restrict__ xc,
                                  double *__restrict__ vc) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * nc) return;
  const int i = (int)(e % n);
  xc[e] = x[i] + dx[e];
  vc[e] = (v ? v[i] : 0.0) + dz[e];
}

// J[c] = 1/2 vc^T vc + 1/2 sum_o rinv_o (y_o - x_c at o)^2 (eq. 2 in control variables), one
// workgroup per candidate, sums in a fixed order.
__global__ void __launch_bounds__(1024)
    cand_cost_kernel(int n, const double *__restrict__ vc, int nobs, int U,
                     const double *__restrict__ y, const double *__restrict__ rinv,
                     const int *__restrict__ u_of_o, const double *__restrict__ xu,
                     double *__restrict__ J) {
  __shared__ double red[16];
  const int c = blockIdx.x;
  const double *v = vc + (size_t)c * n;
  const double *xo = xu + (size_t)c * U;
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) a += v[i] * v[i];
  for (int o = threadIdx.x; o < nobs; o += blockDim.x) {
    const double d = y[o] - xo[u_of_o[o]];
    b += rinv[o] * d * d;
  }
  const double sa = block_sum(a, red);
  const double sb = block_sum(b, red);
  if (threadIdx.x == 0) J[c] = 0.5 * sa + 0.5 * sb;
}

// The candidate with the lowest cost (the first on a tie; a non-finite cost never beats a
// finite one) is copied to dz, dx; its index is written to mode_out (candidate 0 = LRA,
// 1 = LRU: RIOT_LRA or RIOT_LRU).
__global__ void cand_select_kernel(int n, int nc, const double *__restrict__ J,
                                   const double *__restrict__ dzc, const double *__restrict__ dxc,
                                   double *__restrict__ dz, double *__restrict__ dx,
                                   int *__restrict__ mode_out) {
  int best = 0;
  for (int c = 1; c < nc; ++c)
    if (isfinite(J[c]) && (!isfinite(J[best]) || J[c] < J[best])) best = c;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    dz[i] = dzc[(size_t)best * n + i];
    dx[i] = dxc[(size_t)best * n + i];
  }
  if (i == 0 && mode_out) mode_out[0] = best == 0 ? RIOT_LRA : RIOT_LRU;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

// The ring-staged TL/AD kernel serves the full-member E = 16 products unless RIOT_TLAD_RING=0
// (kept for comparison runs against the register-loading kernel).
static bool tlad_ring_enabled() {
  static const bool on = [] {
    const char *e = getenv("RIOT_TLAD_RING");
    return !(e && e[0] == '0');
  }();
  return on;
}

#define RIOT_DISPATCH_E(E_, CALL) \
  switch (E_) {                   \
    case 1: {                     \
      constexpr int EE = 1;       \
      CALL;                       \
    } break;                      \
    case 2: {                     \
      constexpr int EE = 2;       \
      CALL;                       \
    } break;                      \
    case 4: {                     \
      constexpr int EE = 4;       \
      CALL;                       \
    } break;                      \
    case 8: {                     \
      constexpr int EE = 8;       \
      CALL;                       \
    } break;                      \
    case 16: {                    \
      constexpr int EE = 16;      \
      CALL;                       \
    } break;                      \
    default:                      \
      return hipErrorInvalidValue; \
  }

hipError_t launch_trajectory(const ModelView &mv, int nsteps, const double *x0, double *xout,
                             double *xs64, float *xs32, hipStream_t st) {
  const size_t lds = (size_t)kLdsSlots * 2 * mv.NT * sizeof(double);
  RIOT_DISPATCH_E(mv.E, hipLaunchKernelGGL(trajectory_kernel<EE>, dim3(1), dim3(mv.NT), lds, st,
                                           mv, nsteps, x0, xout, xs64, xs32, nullptr, nullptr));
  return hipGetLastError();
}

hipError_t launch_window_obs(const ModelView &mv, int nstates, const double *x0, double *xu,
                             hipStream_t st) {
  if (nstates <= 0) return hipSuccess;
  const size_t lds = (size_t)kLdsSlots * 2 * mv.NT * sizeof(double);
  RIOT_DISPATCH_E(mv.E, hipLaunchKernelGGL(trajectory_kernel<EE>, dim3(nstates), dim3(mv.NT), lds,
                                           st, mv, mv.T, x0, nullptr, nullptr, nullptr, nullptr,
                                           xu));
  return hipGetLastError();
}

hipError_t launch_cand_state(int n, int nc, const double *x, const double *v, const double *dz,
                             const double *dx, double *xc, double *vc, hipStream_t st) {
  const long long tot = (long long)n * nc;
  hipLaunchKernelGGL(cand_state_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n,
                     nc, x, v, dz, dx, xc, vc);
  return hipGetLastError();
}

hipError_t launch_cand_cost(int n, int nc, const double *vc, int nobs, int U, const double *y,
                            const double *rinv, const int *u_of_o, const double *xu, double *J,
                            hipStream_t st) {
  hipLaunchKernelGGL(cand_cost_kernel, dim3(nc), dim3(1024), 0, st, n, vc, nobs, U, y, rinv,
                     u_of_o, xu, J);
  return hipGetLastError();
}

hipError_t launch_cand_select(int n, int nc, const double *J, const double *dzc, const double *dxc,
                              double *dz, double *dx, int *mode_out, hipStream_t st) {
  hipLaunchKernelGGL(cand_select_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, nc, J, dzc,
                     dxc, dz, dx, mode_out);
  return hipGetLastError();
}

hipError_t launch_innovation(const ModelView &mv, const double *xs64, int nobs, const int *obs_step,
                             const int *obs_idx, const double *y, const double *rinv,
                             const int *u_optr, const int *u_olist, double *d, void *fgrad,
                             bool fp32, hipStream_t st) {
  (void)nobs;
  if (mv.U == 0) return hipSuccess;
  const int bs = 256;
  const int grid = (mv.U + bs - 1) / bs;
  if (fp32)
    hipLaunchKernelGGL(innovation_kernel<float>, dim3(grid), dim3(bs), 0, st, mv, xs64, mv.U,
                       obs_step, obs_idx, y, rinv, u_optr, u_olist, d,
                       reinterpret_cast<float *>(fgrad), nullptr);
  else
    hipLaunchKernelGGL(innovation_kernel<double>, dim3(grid), dim3(bs), 0, st, mv, xs64, mv.U,
                       obs_step, obs_idx, y, rinv, u_optr, u_olist, d,
                       reinterpret_cast<double *>(fgrad), nullptr);
  return hipGetLastError();
}

hipError_t launch_cost(int n, const double *v, int nobs, const double *d, const double *rinv,
                       double *out, hipStream_t st) {
  hipLaunchKernelGGL(cost_kernel, dim3(1), dim3(1024), 0, st, n, v, nobs, d, rinv, out);
  return hipGetLastError();
}

hipError_t launch_tlad(const ModelView &mv, int m, int mode, const double *dx0, double *lam0,
                       void *f, const void *fsrc, bool fp32, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  const bool flags = (mode & ~7) != 0;
  const bool full = mv.A == mv.NT;
  if (mode == 0 && full && mv.E == 16 && mv.NT == kRingNT && mv.T >= 1 && tlad_ring_enabled()) {
    const dim3 grid((m + kRingMembers - 1) / kRingMembers), block(kRingMembers * kRingNT);
    if (fp32)
      hipLaunchKernelGGL((tlad_ring_kernel<float, 16>), grid, block, 0, st, mv, m, dx0, lam0,
                         reinterpret_cast<float *>(f), mv.stepk, mv.ustart, mv.umask,
                         reinterpret_cast<const float *>(mv.wgt));
    else
      hipLaunchKernelGGL((tlad_ring_kernel<double, 16>), grid, block, 0, st, mv, m, dx0, lam0,
                         reinterpret_cast<double *>(f), mv.stepk, mv.ustart, mv.umask,
                         reinterpret_cast<const double *>(mv.wgt));
    return hipGetLastError();
  }
#define RIOT_TLAD(R_, F_, U_)                                                                   \
  RIOT_DISPATCH_E(mv.E, hipLaunchKernelGGL((tlad_kernel<R_, EE, F_, U_>), dim3(m), dim3(mv.NT), \
                                           lds, st, mv, mode, dx0, lam0,                        \
                                           reinterpret_cast<R_ *>(f),                           \
                                           reinterpret_cast<const R_ *>(fsrc)))
  if (fp32) {
    const size_t lds = (size_t)kLdsSlots * 2 * mv.NT * sizeof(float);
    if (flags) {
      RIOT_TLAD(float, true, false);
    } else if (full) {
      RIOT_TLAD(float, false, true);
    } else {
      RIOT_TLAD(float, false, false);
    }
  } else {
    const size_t lds = (size_t)kLdsSlots * 2 * mv.NT * sizeof(double);
    if (flags) {
      RIOT_TLAD(double, true, false);
    } else if (full) {
      RIOT_TLAD(double, false, true);
    } else {
      RIOT_TLAD(double, false, false);
    }
  }
#undef RIOT_TLAD
  return hipGetLastError();
}

hipError_t launch_obs_value(const ModelView &mv, const double *xs64, int nobs, const int *obs_step,
                            const int *obs_idx, int lo, bool include_lo, double *out,
                            hipStream_t st) {
  if (nobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(obs_value_kernel, dim3((nobs + 255) / 256), dim3(256), 0, st, mv, xs64, nobs,
                     obs_step, obs_idx, lo, include_lo ? 1 : 0, out);
  return hipGetLastError();
}

hipError_t launch_obs_gather(int nobs, int U, int m, const int *u_of_o, const void *f, double *Z,
                             bool fp32, hipStream_t st, const double *rinv) {
  const size_t tot = (size_t)nobs * m;
  if (tot == 0) return hipSuccess;
  const unsigned grid = (unsigned)((tot + 255) / 256);
  if (fp32)
    hipLaunchKernelGGL(obs_gather_kernel<float>, dim3(grid), dim3(256), 0, st, nobs, U, m, u_of_o,
                       reinterpret_cast<const float *>(f), Z, rinv);
  else
    hipLaunchKernelGGL(obs_gather_kernel<double>, dim3(grid), dim3(256), 0, st, nobs, U, m, u_of_o,
                       reinterpret_cast<const double *>(f), Z, rinv);
  return hipGetLastError();
}

hipError_t launch_obs_scatter(int nobs, int U, int m, const int *u_optr, const int *u_olist,
                              const double *Fo, void *f, bool fp32, hipStream_t st,
                              const double *rinv) {
  const size_t tot = (size_t)U * m;
  if (tot == 0) return hipSuccess;
  const unsigned grid = (unsigned)((tot + 255) / 256);
  if (fp32)
    hipLaunchKernelGGL(obs_scatter_kernel<float>, dim3(grid), dim3(256), 0, st, nobs, U, m, u_optr,
                       u_olist, Fo, reinterpret_cast<float *>(f), rinv);
  else
    hipLaunchKernelGGL(obs_scatter_kernel<double>, dim3(grid), dim3(256), 0, st, nobs, U, m, u_optr,
                       u_olist, Fo, reinterpret_cast<double *>(f), rinv);
  return hipGetLastError();
}

hipError_t launch_psas_rhs(int nobs, const double *rinv, const double *d, const double *bp,
                           double *out, hipStream_t st) {
  if (nobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(psas_rhs_kernel, dim3((nobs + 255) / 256), dim3(256), 0, st, nobs, rinv, d, bp,
                     out);
  return hipGetLastError();
}

hipError_t launch_obs_perturb(int nobs, const double *y, const double *rinv, const double *eps,
                              double *out, hipStream_t st) {
  if (nobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(obs_perturb_kernel, dim3((nobs + 255) / 256), dim3(256), 0, st, nobs, y, rinv,
                     eps, out);
  return hipGetLastError();
}

hipError_t launch_psas_scale(int nobs, const double *rinv, const double *t, double *dw,
                             hipStream_t st) {
  if (nobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(psas_scale_kernel, dim3((nobs + 255) / 256), dim3(256), 0, st, nobs, rinv, t,
                     dw);
  return hipGetLastError();
}

hipError_t launch_apply_L(int n, int w, const double *taps, int m, const double *X, double *Y,
                          const double *Z, int mode, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  const size_t seg_lds = (size_t)(kLSeg + 2 * w) * sizeof(double);
  if (seg_lds <= 60 * 1024) {
    const unsigned nseg = (unsigned)((n + kLSeg - 1) / kLSeg);
    hipLaunchKernelGGL(apply_L_seg_kernel, dim3(m, nseg), dim3(256), seg_lds, st, n, w, taps, X, Y,
                       Z, mode);
    return hipGetLastError();
  }
  const size_t lds = (size_t)(n + 2 * w) * sizeof(double);
  const int use_lds = lds <= 60 * 1024 ? 1 : 0;
  hipLaunchKernelGGL(apply_L_kernel, dim3(m), dim3(256), use_lds ? lds : 0, st, n, w, taps, X, Y,
                     Z, mode, use_lds, nullptr);
  return hipGetLastError();
}

hipError_t launch_cg(const ModelView &mv, int w, const double *taps, const double *g, int iters,
                     double rtol, double *x, double *iterates, double *vec_scratch, void *f,
                     int *used, bool fp32, hipStream_t st) {
  const size_t xb = (size_t)kLdsSlots * 2 * mv.NT * (fp32 ? sizeof(float) : sizeof(double));
  const size_t ext_off = (xb + 255) / 256 * 256;
  const size_t ext_bytes = (size_t)(mv.n + 2 * w) * sizeof(double);
  const int use_ext = (ext_off + ext_bytes) <= 60 * 1024 ? 1 : 0;
  const size_t lds = use_ext ? ext_off + ext_bytes : xb;
  if (fp32) {
    RIOT_DISPATCH_E(mv.E, hipLaunchKernelGGL((cg_kernel<float, EE>), dim3(1), dim3(mv.NT), lds, st,
                                             mv, w, taps, g, iters, rtol, x, iterates, vec_scratch,
                                             reinterpret_cast<float *>(f), used, (int)ext_off,
                                             use_ext));
  } else {
    RIOT_DISPATCH_E(mv.E, hipLaunchKernelGGL((cg_kernel<double, EE>), dim3(1), dim3(mv.NT), lds,
                                             st, mv, w, taps, g, iters, rtol, x, iterates,
                                             vec_scratch, reinterpret_cast<double *>(f), used,
                                             (int)ext_off, use_ext));
  }
  return hipGetLastError();
}

hipError_t launch_philox_normal(long long total, uint64_t seed, uint64_t stream, double *out,
                                hipStream_t st) {
  if (total <= 0) return hipSuccess;
  const long long pairs = (total + 1) / 2;
  const int bs = 256;
  const long long grid = (pairs + bs - 1) / bs;
  hipLaunchKernelGGL(philox_normal_kernel, dim3((unsigned)grid), dim3(bs), 0, st, total, seed,
                     stream, out, nullptr);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Batched launchers (E = 8, workgroups of 256 threads, NT <= 256 per problem)
// ---------------------------------------------------------------------------

constexpr int kBatchThreads = 256;

hipError_t launch_trajectory_batched(int nprob, const TrajJob *jobs, hipStream_t st) {
  if (nprob <= 0) return hipSuccess;
  const size_t lds = (size_t)kLdsSlots * 2 * kBatchThreads * sizeof(double);
  hipLaunchKernelGGL(trajectory_kernel<8>, dim3(nprob), dim3(kBatchThreads), lds, st, ModelView{}, 0,
                     nullptr, nullptr, nullptr, nullptr, jobs, nullptr);
  return hipGetLastError();
}

hipError_t launch_innovation_batched(int nprob, int maxU, const InnovJob *jobs, bool fp32,
                                     hipStream_t st) {
  if (nprob <= 0 || maxU <= 0) return hipSuccess;
  const dim3 grid((maxU + 255) / 256, nprob);
  if (fp32)
    hipLaunchKernelGGL(innovation_kernel<float>, grid, dim3(256), 0, st, ModelView{}, nullptr, 0,
                       nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, jobs);
  else
    hipLaunchKernelGGL(innovation_kernel<double>, grid, dim3(256), 0, st, ModelView{}, nullptr, 0,
                       nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, jobs);
  return hipGetLastError();
}

hipError_t launch_tlad_persistent(int nwg, int mode, const TladProb *probs, const TladTile *wg_tiles,
                                  int n_wg, const TladTile *wave_tiles, int n_wave, int *counters,
                                  bool fp32, hipStream_t st, long long *clk) {
  if (nwg <= 0 || (n_wg <= 0 && n_wave <= 0)) return hipSuccess;
  hipError_t e = launch_zero_ints(counters, 2, st);
  if (e != hipSuccess) return e;
  const size_t lds =
      (size_t)kLdsSlots * 2 * kBatchThreads * (fp32 ? sizeof(float) : sizeof(double));
  if (fp32)
    hipLaunchKernelGGL(tlad_persistent_kernel<float>, dim3(nwg), dim3(kBatchThreads), lds, st, mode,
                       probs, wg_tiles, n_wg, wave_tiles, n_wave, counters, clk);
  else
    hipLaunchKernelGGL(tlad_persistent_kernel<double>, dim3(nwg), dim3(kBatchThreads), lds, st,
                       mode, probs, wg_tiles, n_wg, wave_tiles, n_wave, counters, clk);
  return hipGetLastError();
}

int tlad_persistent_resident_per_cu(bool fp32) {
  int nb = 0;
  const size_t lds =
      (size_t)kLdsSlots * 2 * kBatchThreads * (fp32 ? sizeof(float) : sizeof(double));
  const hipError_t e =
      fp32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, tlad_persistent_kernel<float>,
                                                          kBatchThreads, lds)
           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, tlad_persistent_kernel<double>,
                                                          kBatchThreads, lds);
  return e == hipSuccess ? nb : 0;
}

hipError_t launch_apply_L_batched(int nprob, int maxm, int maxext, const ApplyLJobE *jobs,
                                  hipStream_t st) {
  if (nprob <= 0 || maxm <= 0) return hipSuccess;
  const size_t lds = (size_t)maxext * sizeof(double);
  if (lds > 60 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(apply_L_kernel, dim3(maxm, nprob), dim3(256), lds, st, 0, 0, nullptr, nullptr,
                     nullptr, nullptr, 0, 1, jobs);
  return hipGetLastError();
}

hipError_t launch_philox_batched(int nprob, long long maxtotal, uint64_t seed,
                                 const PhiloxJob *jobs, hipStream_t st) {
  if (nprob <= 0 || maxtotal <= 0) return hipSuccess;
  const long long pairs = (maxtotal + 1) / 2;
  hipLaunchKernelGGL(philox_normal_kernel, dim3((unsigned)((pairs + 255) / 256), nprob), dim3(256),
                     0, st, 0LL, seed, 0ULL, nullptr, jobs);
  return hipGetLastError();
}

}  // namespace riot
