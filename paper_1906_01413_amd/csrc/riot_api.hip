// C ABI of the RIOT inner loop: handle, workspace carve-up, call sequencing.
//
// The calls follow Alg. 3 (precond = false) of arXiv 1906.01413: linearise
// (trajectory, innovation, gradient), Hessian-probe products of the whole probe
// block, orthonormal basis, K from K (Q^T Omega) = Q^T Y, eigendecomposition,
// adaptive increment (eqs. 8-11) and low-rank posterior covariance.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "riot_internal.h"

using namespace riot;

namespace {

constexpr int kSplitK = 16;

// Scratch of the linear algebra: the split-K partial products of an m x m Gram matrix,
// later reused for the inverses of the Cholesky factor's 32 x 32 diagonal blocks.
// The Gram's partial sums of squares for the in-place Cholesky follow both uses, then 32
// doubles of flags for its workgroups, then the partial sums of its squared distance from I.
inline size_t gram_sq_offset(size_t m) {
  return std::max((size_t)kSplitK * std::max(m * m, m), (m + 31) / 32 * 1024);
}
inline size_t partial_doubles(size_t m) {
  return gram_sq_offset(m) + 2 * ((m * m + 255) / 256) + 32;
}

// Bump allocator over the caller's workspace (base == nullptr: size only).
struct Carver {
  char *base;
  size_t off = 0;
  explicit Carver(void *b) : base(static_cast<char *>(b)) {}
  template <typename T>
  T *take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

int launch_bound_for(int E) { return E >= 8 ? 512 : 1024; }

// Elements per lane: largest E with n % E == 0 and 256 <= n/E <= bound, else
// largest with n/E >= 64, else 1.
int choose_E(int n, int requested) {
  const int cands[5] = {16, 8, 4, 2, 1};
  if (requested) {
    if (n % requested || n / requested > launch_bound_for(requested)) return 0;
    return requested;
  }
  for (int E : cands)
    if (n % E == 0 && n / E >= 256 && n / E <= launch_bound_for(E)) return E;
  for (int E : cands)
    if (n % E == 0 && n / E >= 64 && n / E <= launch_bound_for(E)) return E;
  for (int E : cands)
    if (n % E == 0 && n / E <= launch_bound_for(E)) return E;
  return 0;
}

struct ObsPlan {
  int S = 0, U = 0;
  std::vector<int> stepk, ustart, umask, u_optr, u_olist, u_of_o;
  std::vector<double> wgt;
};

bool build_obs(const riot_desc &d, int E, int NT, ObsPlan &p) {
  const int n = d.n, T = d.nsteps, no = d.nobs;
  std::vector<int> order(no);
  for (int o = 0; o < no; ++o) {
    if (d.obs_step[o] < 0 || d.obs_step[o] > T || d.obs_idx[o] < 0 || d.obs_idx[o] >= n)
      return false;
    if (!(d.rinv[o] > 0.0) || !std::isfinite(d.rinv[o]) || !std::isfinite(d.y[o])) return false;
    order[o] = o;
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (d.obs_step[a] != d.obs_step[b]) return d.obs_step[a] < d.obs_step[b];
    return d.obs_idx[a] < d.obs_idx[b];
  });
  p.stepk.assign(T + 1, -1);
  p.u_of_o.assign(std::max(no, 1), 0);
  std::vector<int> ustep, uidx;
  for (int q = 0; q < no; ++q) {
    const int o = order[q];
    const int t = d.obs_step[o], i = d.obs_idx[o];
    if (p.U == 0 || ustep.back() != t || uidx.back() != i) {
      ustep.push_back(t);
      uidx.push_back(i);
      p.wgt.push_back(0.0);
      p.u_optr.push_back(q);
      ++p.U;
    }
    p.wgt.back() += d.rinv[o];
    p.u_olist.push_back(o);
    p.u_of_o[o] = p.U - 1;
  }
  p.u_optr.push_back(no);
  for (int u = 0; u < p.U; ++u)
    if (p.stepk[ustep[u]] < 0) p.stepk[ustep[u]] = p.S++;
  p.ustart.assign((size_t)std::max(p.S, 1) * NT, 0);
  p.umask.assign((size_t)std::max(p.S, 1) * NT, 0);
  std::vector<char> seen((size_t)std::max(p.S, 1) * NT, 0);
  for (int u = 0; u < p.U; ++u) {
    const int k = p.stepk[ustep[u]];
    const int l = uidx[u] / E, j = uidx[u] % E;
    const size_t s = (size_t)k * NT + l;
    if (!seen[s]) {
      seen[s] = 1;
      p.ustart[s] = u;
    }
    p.umask[s] |= 1 << j;
  }
  return true;
}

}  // namespace

struct riot_handle {
  riot_desc d{};
  hipStream_t st = nullptr;
  int E = 0, NT = 0, A = 0, S = 0, U = 0, w = 0;
  int cus = 256;  // compute units of the device the handle was created on
  bool fp32 = false;
  bool linearized = false;
  double base_diag = 0.0;
  // device regions
  double *taps = nullptr, *brow = nullptr;
  int *stepk = nullptr, *ustart = nullptr, *umask = nullptr;
  double *wgt64 = nullptr;
  float *wgt32 = nullptr;
  int *obs_step = nullptr, *obs_idx = nullptr, *u_optr = nullptr, *u_olist = nullptr,
      *u_of_o = nullptr;
  double *y = nullptr, *rinv = nullptr;
  double *xs64 = nullptr;
  float *xs32 = nullptr;
  void *fgrad = nullptr, *f = nullptr;
  double *LW = nullptr, *LAM = nullptr;
  double *Om = nullptr, *Y = nullptr, *Q = nullptr, *Q0 = nullptr;
  double *G = nullptr, *R = nullptr, *B1 = nullptr, *B2 = nullptr, *K = nullptr, *Zs = nullptr,
         *sywork = nullptr;
  double *partial = nullptr, *cvec = nullptr, *scal = nullptr, *cgv = nullptr;
  double *sel = nullptr;  // candidate increments, states and observed values (2 n x 4, 2 U, 2)
  double *pso = nullptr;  // observation-space vectors of the dual solve (2 nobs)
  int *flags = nullptr;
  ModelView mv{};
  // deferred gradient: lambda_0 of the gradient's adjoint sweep, and a second stream with
  // its fork / done events (created on the first deferred linearisation)
  double *LAM0 = nullptr;
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_grad = nullptr;
  bool grad_pending = false;
  // host-mapped word through which a CholeskyQR pass reports whether the next one runs
  // (pinned host memory; nullptr if it could not be had), and whether the host uses it
  int *hflag = nullptr, *hflag_dev = nullptr;
  unsigned pass_seq = 0;
  bool pass_sync = true;
  ~riot_handle() {
    if (side) {
      (void)hipStreamSynchronize(side);
      (void)hipStreamDestroy(side);
    }
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_grad) (void)hipEventDestroy(ev_grad);
    if (hflag) {
      (void)hipStreamSynchronize(st);
      (void)hipHostFree(hflag);
    }
  }
};

// Buffers of the RSVD linear algebra (CholeskyQR, projections, K, eigen-solve), shared by
// a problem handle and a standalone sketch handle.
struct LaSpace {
  hipStream_t st;
  double *Q, *G, *R, *B1, *B2, *K, *Zs, *sywork, *partial, *scal, *cvec;
  int *flags;
  int *cq;  // CholeskyQR pass control (kMaxCholQRPasses + 1 ints), after the 16 flags
  // host-read pass control (see cholqr): the host-mapped word (host and device addresses)
  // and the handle's sequence counter; nullptr: every pass is launched, predicated
  int *hflag = nullptr, *hflag_dev = nullptr;
  unsigned *seq = nullptr;
};

inline LaSpace la_of(riot_handle *h) {
  LaSpace la{h->st, h->Q, h->G, h->R, h->B1, h->B2, h->K, h->Zs, h->sywork, h->partial, h->scal,
             h->cvec, h->flags, h->flags + 16};
  if (h->pass_sync && h->hflag) la.hflag = h->hflag, la.hflag_dev = h->hflag_dev, la.seq = &h->pass_seq;
  return la;
}

namespace {

// Carve (or size) every region of the workspace.
size_t carve(riot_handle &h, void *base) {
  Carver c(base);
  const riot_desc &d = h.d;
  const int n = d.n, T = d.nsteps, mm = d.m_max;
  const size_t Rs = h.fp32 ? sizeof(float) : sizeof(double);
  const size_t U1 = (size_t)std::max(h.U, 1);
  h.taps = c.take<double>(h.w + 1);
  h.brow = c.take<double>(n);
  h.stepk = c.take<int>(T + 1);
  h.ustart = c.take<int>((size_t)std::max(h.S, 1) * h.NT);
  h.umask = c.take<int>((size_t)std::max(h.S, 1) * h.NT);
  h.wgt64 = c.take<double>(U1);
  h.wgt32 = h.fp32 ? c.take<float>(U1) : nullptr;
  h.obs_step = c.take<int>(std::max(d.nobs, 1));
  h.obs_idx = c.take<int>(std::max(d.nobs, 1));
  h.u_optr = c.take<int>(U1 + 1);
  h.u_olist = c.take<int>(std::max(d.nobs, 1));
  h.u_of_o = c.take<int>(std::max(d.nobs, 1));
  h.y = c.take<double>(std::max(d.nobs, 1));
  h.rinv = c.take<double>(std::max(d.nobs, 1));
  // the whole window's stage blocks, or one checkpoint segment's
  const int Tst = d.ckpt_stride > 0 ? d.ckpt_stride : T;
  const size_t blk = (size_t)(Tst + 1) * 4 * stage_block_elems(h.E, h.NT);
  h.xs64 = c.take<double>(blk);
  h.xs32 = h.fp32 ? c.take<float>(blk) : nullptr;
  h.fgrad = c.take<char>(U1 * Rs);
  h.f = c.take<char>((size_t)(mm + 1) * U1 * Rs);
  const size_t nm = (size_t)n * mm;
  h.LW = c.take<double>(nm);
  h.LAM = c.take<double>(nm);
  h.LAM0 = c.take<double>(n);
  h.Om = c.take<double>(nm);
  h.Y = c.take<double>(nm);
  h.Q = c.take<double>(nm);
  h.Q0 = c.take<double>(nm);
  const size_t m2 = (size_t)mm * mm;
  h.G = c.take<double>(m2);
  h.R = c.take<double>(m2);
  h.B1 = c.take<double>(m2);
  h.B2 = c.take<double>(m2);
  h.K = c.take<double>(m2);
  h.Zs = c.take<double>(m2);
  h.sywork = c.take<double>(eig_work_doubles(mm));
  h.partial = c.take<double>(partial_doubles(mm));
  h.cvec = c.take<double>(mm);
  h.scal = c.take<double>(16);
  h.cgv = c.take<double>((size_t)5 * n);
  h.sel = c.take<double>((size_t)8 * n + 2 * U1 + 2);
  h.pso = c.take<double>((size_t)2 * std::max(d.nobs, 1));
  h.flags = c.take<int>(32);  // 16 flags, then the CholeskyQR pass control
  return c.off + 256;
}

bool desc_valid(const riot_desc *d) {
  if (!d) return false;
  if (d->n < 4 || d->n > 16384 || d->nsteps < 0 || d->nobs < 0 || d->m_max < 1) return false;
  if (!(d->dt > 0.0) || !std::isfinite(d->dt) || !std::isfinite(d->forcing)) return false;
  if (d->l_halfwidth < 0 || !d->l_taps) return false;
  if (d->nobs > 0 && (!d->obs_step || !d->obs_idx || !d->y || !d->rinv)) return false;
  if (d->prec != RIOT_FP64 && d->prec != RIOT_FP32_TLAD) return false;
  if (choose_E(d->n, d->elems_per_lane) == 0) return false;
  if (d->m_max > 1088) return false;
  if (d->ckpt_stride < 0 || d->ckpt_stride > std::max(d->nsteps, 1)) return false;
  return true;
}

bool prepare(riot_handle &h, const riot_desc *d, ObsPlan *plan) {
  h.d = *d;
  h.fp32 = d->prec == RIOT_FP32_TLAD;
  h.E = choose_E(d->n, d->elems_per_lane);
  h.A = d->n / h.E;
  h.NT = (h.A + 63) / 64 * 64;
  h.w = d->l_halfwidth;
  ObsPlan local;
  ObsPlan &p = plan ? *plan : local;
  if (!build_obs(*d, h.E, h.NT, p)) return false;
  h.S = p.S;
  h.U = p.U;
  return true;
}

void fill_view(riot_handle &h) {
  ModelView &mv = h.mv;
  mv.n = h.d.n;
  mv.T = h.d.nsteps;
  mv.E = h.E;
  mv.NT = h.NT;
  mv.A = h.A;
  mv.h = h.d.dt;
  mv.F = h.d.forcing;
  mv.S = h.S;
  mv.U = h.U;
  mv.xs = h.fp32 ? (const void *)h.xs32 : (const void *)h.xs64;
  mv.stepk = h.stepk;
  mv.ustart = h.ustart;
  mv.umask = h.umask;
  mv.wgt = h.fp32 ? (const void *)h.wgt32 : (const void *)h.wgt64;
}

#define RIOT_HIP(call)                             \
  do {                                             \
    if ((call) != hipSuccess) return RIOT_E_HIP;   \
  } while (0)

riot_status read_flag(riot_handle *h, int idx, int *out) {
  RIOT_HIP(hipMemcpyAsync(out, h->flags + idx, sizeof(int), hipMemcpyDeviceToHost, h->st));
  RIOT_HIP(hipStreamSynchronize(h->st));
  return RIOT_OK;
}

// Q = orth(Xin) (rows x m, leading dimension rows) by CholeskyQR. Each pass computes
// G = X^T X, G (+ s I) = L L^T and X <- X L^{-T}; a companion C (mc x m, ld mc) receives
// the same right factors, C <- C L^{-T}, so that X_in M = Q and C_in M = C_out for one M.
// The first pass is shifted when `shifted` (s = 11 (m rows + m (m+1)) u ||G||_F, which
// never breaks down); later passes replace any pivot below that shift by it. Passes repeat
// on the device until two in a row are plain with no pivot replaced, which leaves Q
// orthonormal to rounding; a pass whose Gram is within sqrt(u) of I in the Frobenius norm
// (usually the last: the one before it already left Q orthonormal to about 1e-11) takes
// the first-order factor instead of a factorization. At most kMaxCholQRPasses: a sketch
// whose singular values span more than the FP64 range of one shifted pass (graded spectra,
// numerically rank-deficient blocks) gets further passes instead of a non-orthonormal Q.
// Each pass's kernels read its run flag, set by the previous pass's Cholesky, and return at
// once when it is 0. Two ways to launch them:
//  - host-read control (la.hflag set and the stream not being captured): the passes that
//    always run (three after a shifted first pass, which is never clean; two otherwise) are
//    launched, then one at a time, each after the previous pass's Cholesky has stored its
//    decision in the host-mapped word; the host waits for that store only, while the pass's
//    solve still runs, so the device does not idle, and no pass beyond the last is launched;
//  - otherwise all kMaxCholQRPasses are launched and the unneeded ones return at once.
constexpr int kMaxCholQRPasses = 8;
static_assert(kMaxCholQRPasses + 1 <= 16, "the pass control fits after the 16 flags");

// Wait for the host-mapped word to carry sequence number `seq`, and return the decision it
// holds. Should the stream drain without it (no pass left to report), the decision is read
// from the device's run flag `cq_next` instead; a stream error is returned as RIOT_E_HIP.
riot_status wait_pass(const LaSpace &h, int seq, const int *cq_next, int *next) {
  for (unsigned it = 1;; ++it) {
    const int v = __atomic_load_n(h.hflag, __ATOMIC_ACQUIRE);
    if ((v >> 1) == seq) {
      *next = v & 1;
      return RIOT_OK;
    }
    if ((it & 127) == 0) {
      const hipError_t q = hipStreamQuery(h.st);
      if (q == hipSuccess) {
        const int w = __atomic_load_n(h.hflag, __ATOMIC_ACQUIRE);
        if ((w >> 1) == seq) {
          *next = w & 1;
          return RIOT_OK;
        }
        RIOT_HIP(hipMemcpy(next, cq_next, sizeof(int), hipMemcpyDeviceToHost));
        return RIOT_OK;
      }
      if (q != hipErrorNotReady) return RIOT_E_HIP;
    }
#if defined(__x86_64__)
    __builtin_ia32_pause();
#endif
  }
}

riot_status cholqr(const LaSpace &h, int rows, int m, const double *Xin, double *Qout,
                   bool shifted, int flag_idx, double *comp = nullptr, int mc = 0,
                   int *count = nullptr) {
  hipStream_t st = h.st;
  const double u = 0x1.0p-53;
  const double srel = 11.0 * ((double)m * rows + (double)m * (m + 1)) * u;
  int *cq = h.cq;
  bool host_ctl = h.hflag != nullptr;
  if (host_ctl) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
      host_ctl = false;
  }
  const int always = shifted ? 3 : 2;  // passes that run whatever the data
  for (int pass = 0; pass < kMaxCholQRPasses; ++pass) {
    const bool sh = shifted && pass == 0;
    // pass 0 always runs, on Xin (its solve writes Qout); pass p > 0 runs when the Cholesky
    // of pass p - 1 set run flag p (a pass that does not run clears the next one's flag)
    int *run = pass == 0 ? nullptr : cq + pass;
    const double *src = pass == 0 ? Xin : Qout;
    // the Gram goes straight into R (lower triangle, zero upper) with the partial sums of
    // its squared Frobenius norm and distance from I, and is factored there in place; the
    // Cholesky also writes its diagonal blocks' inverses into the Gram's split-K buffer,
    // free by then, and decides whether the next pass runs
    double *gsq = h.partial + gram_sq_offset(m);
    RIOT_HIP(gemm_f64(1, 0, m, m, rows, 1.0, src, rows, src, rows, 0.0, h.R, m, h.partial,
                      kSplitK, st, run, true, gsq));
    CholQrCtl ctl;
    ctl.cq = cq, ctl.pass = pass, ctl.npass = kMaxCholQRPasses, ctl.count = count;
    const bool wait = host_ctl && pass + 1 >= always && pass + 1 < kMaxCholQRPasses;
    if (wait) {
      ctl.host = h.hflag_dev;
      ctl.seq = (int)(++*h.seq & 0x3fffffffu);
    }
    RIOT_HIP(launch_chol_blocked(m, h.R, h.R, srel, sh ? 1 : 2, h.flags + flag_idx, h.flags + 4,
                                 st, nullptr, nullptr, gsq, h.partial, ctl));
    // X and its companion in one launch
    RIOT_HIP(launch_trsm_rlt_inv(rows, m, Qout, rows, h.R, h.partial, st, run, comp ? mc : 0,
                                 comp, comp ? mc : 1, pass == 0 ? Xin : nullptr));
    if (wait) {
      int next = 1;
      const riot_status ws = wait_pass(h, ctl.seq, cq + pass + 1, &next);
      if (ws != RIOT_OK) return ws;
      if (!next) break;
    }
  }
  return RIOT_OK;
}

// Alg. 3 from a finished sketch: Q = orth(Y); B1 = Q^T Y, B2 = Q^T Omega_eff; K solves
// K B2 = B1 (CholeskyQR of the square B2 carrying B1 as companion: B2 M = Q2, B1 M -> B1',
// so B2^{-1} = M Q2^T and K = B1' Q2^T); K <- (K + K^T)/2 = Z diag(lambda) Z^T; V = Q Z.
// The caller zeroes la.flags first.
riot_status sketch_eig(const LaSpace &la, int n, int m, const double *Y, const double *Om_eff,
                       double *lambda, double *V, riot_rsvd_info *info) {
  hipStream_t st = la.st;
  riot_status rs = cholqr(la, n, m, Y, la.Q, true, 0, nullptr, 0, la.flags + 5);
  if (rs != RIOT_OK) return rs;
  // B1 and B2 in one launch (half the K splits: the partial buffer holds both products)
  RIOT_HIP(gemm_f64(1, 0, m, m, n, 1.0, la.Q, n, Y, n, 0.0, la.B1, m, la.partial, kSplitK / 2,
                    st, nullptr, false, nullptr, Om_eff, la.B2));
  rs = cholqr(la, m, m, la.B2, la.Zs, false, 1, la.B1, m);
  if (rs != RIOT_OK) return rs;
  if (info) {  // ||K - K^T|| / ||K|| (reported) needs K before symmetrisation
    RIOT_HIP(gemm_f64(0, 1, m, m, m, 1.0, la.B1, m, la.Zs, m, 0.0, la.K, m, la.partial, kSplitK,
                      st));
    RIOT_HIP(launch_symmetrize(m, la.K, la.scal + 1, la.partial, st));
  } else {  // K <- (K + K^T) / 2 as the product's split-K reduction forms it
    RIOT_HIP(gemm_f64(0, 1, m, m, m, 1.0, la.B1, m, la.Zs, m, 0.0, la.K, m, la.partial, kSplitK,
                      st, nullptr, false, nullptr, nullptr, nullptr, true));
  }
  RIOT_HIP(launch_eig(m, la.K, lambda, la.Zs, la.sywork, la.flags + 2, st));
  RIOT_HIP(gemm_f64(0, 0, n, m, m, 1.0, la.Q, n, la.Zs, m, 0.0, V, n, nullptr, 1, st));
  RIOT_HIP(launch_check_finite(m, lambda, la.flags + 3, st, (long long)n * m, V));
  if (info) {
    RIOT_HIP(gemm_f64(1, 0, m, m, n, 1.0, la.Q, n, la.Q, n, 0.0, la.G, m, la.partial, kSplitK, st));
    RIOT_HIP(launch_orth_err(m, la.G, la.scal + 2, st));
    // residual of the defining equation with the symmetrised K: ||K B2 - B1|| / ||B1||
    // (B1 = Q^T Y formed again: the solve above overwrote it; B2 and K are intact)
    RIOT_HIP(gemm_f64(1, 0, m, m, n, 1.0, la.Q, n, Y, n, 0.0, la.R, m, la.partial, kSplitK, st));
    RIOT_HIP(gemm_f64(0, 0, m, m, m, 1.0, la.K, m, la.B2, m, 0.0, la.G, m, nullptr, 1, st));
    RIOT_HIP(launch_axpby((long long)m * m, 1.0, la.G, -1.0, la.R, st));
    RIOT_HIP(launch_fro_ratio((long long)m * m, la.G, la.R, la.scal + 7, st));
    int fl[6];
    double sc[8], lend[2];
    RIOT_HIP(hipMemcpyAsync(fl, la.flags, 6 * sizeof(int), hipMemcpyDeviceToHost, st));
    RIOT_HIP(hipMemcpyAsync(sc, la.scal, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
    RIOT_HIP(hipMemcpyAsync(&lend[0], lambda, sizeof(double), hipMemcpyDeviceToHost, st));
    RIOT_HIP(hipMemcpyAsync(&lend[1], lambda + (m - 1), sizeof(double), hipMemcpyDeviceToHost, st));
    RIOT_HIP(hipStreamSynchronize(st));
    info->chol_shifts = fl[4];
    info->qr_passes = fl[5];
    info->k_asym = sc[1];
    info->orth_err = sc[2];
    info->kappa_est = (1.0 + lend[0]) / (1.0 + std::max(lend[1], 0.0));
    info->resid_est = sc[7];
    if (fl[0]) return RIOT_E_NOT_SPD;
    if (fl[1]) return RIOT_E_SINGULAR;
    if (fl[2]) return RIOT_E_NOCONV;
    if (fl[3]) return RIOT_E_NONFINITE;
  }
  return RIOT_OK;
}

// dz from the k leading Ritz pairs (eqs. 8-11; no L): c = V^T g, then the LRA/LRU combination.
riot_status sketch_increment(const LaSpace &la, int n, int k, const double *lambda,
                             const double *V, const double *grad, riot_update mode, double *dz,
                             double *dofs_host, int32_t *mode_used) {
  hipStream_t st = la.st;
  RIOT_HIP(gemm_f64(1, 0, k, 1, n, 1.0, V, n, grad, n, 0.0, la.cvec, k, la.partial, kSplitK, st));
  const int ml = mode == RIOT_LRA ? 0 : (mode == RIOT_LRU ? 1 : 2);
  RIOT_HIP(launch_increment_combine(n, k, lambda, V, la.cvec, grad, ml, dz, la.scal + 4, st));
  if (mode_used) RIOT_HIP(launch_choose_mode(k, lambda, la.flags + 8, st));
  if (dofs_host || mode_used) {
    int mu = 0;
    if (dofs_host)
      RIOT_HIP(hipMemcpyAsync(dofs_host, la.scal + 4, sizeof(double), hipMemcpyDeviceToHost, st));
    if (mode_used)
      RIOT_HIP(hipMemcpyAsync(&mu, la.flags + 8, sizeof(int), hipMemcpyDeviceToHost, st));
    RIOT_HIP(hipStreamSynchronize(st));
    if (mode_used) *mode_used = (mode == RIOT_ADAPTIVE) ? mu : (int32_t)mode;
  }
  return RIOT_OK;
}

// Projected residual rho = ||A Q - Q Q^T A Q||_F / ||A Q||_F of an orthonormal block Q
// (Q and AQ n x m, column-major): how far span(Q) is from an invariant subspace of A.
riot_status proj_residual(const LaSpace &la, int n, int m, const double *Q, const double *AQ,
                          double *rho_host) {
  hipStream_t st = la.st;
  RIOT_HIP(gemm_f64(1, 0, m, m, n, 1.0, Q, n, AQ, n, 0.0, la.K, m, la.partial, kSplitK, st));
  RIOT_HIP(hipMemcpyAsync(la.Q, AQ, (size_t)n * m * sizeof(double), hipMemcpyDeviceToDevice, st));
  RIOT_HIP(gemm_f64(0, 0, n, m, m, -1.0, Q, n, la.K, m, 1.0, la.Q, n, la.partial, 1, st));
  RIOT_HIP(launch_fro_ratio((long long)n * m, la.Q, AQ, la.scal + 6, st));
  RIOT_HIP(hipMemcpyAsync(rho_host, la.scal + 6, sizeof(double), hipMemcpyDeviceToHost, st));
  RIOT_HIP(hipStreamSynchronize(st));
  return RIOT_OK;
}

riot_status hess_apply_impl(riot_handle *h, int m, const double *W, double *Y, int add_identity) {
  const int n = h->d.n;
  hipStream_t st = h->st;
  RIOT_HIP(launch_apply_L(n, h->w, h->taps, m, W, h->LW, nullptr, 0, st));
  RIOT_HIP(launch_tlad(h->mv, m, 0, h->LW, h->LAM, h->f, nullptr, h->fp32, st));
  RIOT_HIP(launch_apply_L(n, h->w, h->taps, m, h->LAM, Y, add_identity ? W : nullptr,
                          add_identity ? 1 : 0, st));
  return RIOT_OK;
}

}  // namespace

extern "C" {

size_t riot_workspace_bytes(const riot_desc *desc) {
  if (!desc_valid(desc)) return 0;
  riot_handle h;
  if (!prepare(h, desc, nullptr)) return 0;
  return carve(h, nullptr);
}

// Set up a handle in `workspace` (shared by riot_init and the batch): carve, host tables,
// uploads. Synchronises the stream before returning (the host tables are local).
static riot_status init_handle(riot_handle *h, const riot_desc *desc, void *workspace,
                               size_t bytes, hipStream_t st) {
  ObsPlan plan;
  if (!prepare(*h, desc, &plan)) return RIOT_E_ARG;
  const size_t need = carve(*h, nullptr);
  if (bytes < need) return RIOT_E_WORKSPACE;
  carve(*h, workspace);
  h->st = st;
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        cus > 0)
      h->cus = cus;
  }
  fill_view(*h);
  const riot_desc &d = h->d;
  const int n = d.n, w = h->w;
  // host-side tables: the first row of L (wrapped taps) and of B = L L^T
  std::vector<double> lrow(n, 0.0), brow(n, 0.0);
  for (int dd = -w; dd <= w; ++dd) {
    int j = dd % n;
    if (j < 0) j += n;
    lrow[j] += d.l_taps[std::abs(dd)];
  }
  std::vector<int> nz;
  for (int j = 0; j < n; ++j)
    if (lrow[j] != 0.0) nz.push_back(j);
  for (int dd = 0; dd < n; ++dd) {
    double s = 0.0;
    for (int j : nz) s += lrow[j] * lrow[(j + dd) % n];
    brow[dd] = s;
  }
  h->base_diag = brow[0];
  std::vector<float> wgt32(plan.wgt.begin(), plan.wgt.end());
  riot_status rs = RIOT_OK;
  auto cp = [&](void *dst, const void *src, size_t b) {
    if (b && hipMemcpyAsync(dst, src, b, hipMemcpyHostToDevice, st) != hipSuccess) rs = RIOT_E_HIP;
  };
  cp(h->taps, d.l_taps, (size_t)(w + 1) * sizeof(double));
  cp(h->brow, brow.data(), (size_t)n * sizeof(double));
  cp(h->stepk, plan.stepk.data(), plan.stepk.size() * sizeof(int));
  cp(h->ustart, plan.ustart.data(), plan.ustart.size() * sizeof(int));
  cp(h->umask, plan.umask.data(), plan.umask.size() * sizeof(int));
  cp(h->wgt64, plan.wgt.data(), plan.wgt.size() * sizeof(double));
  if (h->fp32) cp(h->wgt32, wgt32.data(), wgt32.size() * sizeof(float));
  cp(h->obs_step, d.obs_step, (size_t)d.nobs * sizeof(int));
  cp(h->obs_idx, d.obs_idx, (size_t)d.nobs * sizeof(int));
  cp(h->u_optr, plan.u_optr.data(), plan.u_optr.size() * sizeof(int));
  cp(h->u_olist, plan.u_olist.data(), plan.u_olist.size() * sizeof(int));
  cp(h->u_of_o, plan.u_of_o.data(), (size_t)d.nobs * sizeof(int));
  cp(h->y, d.y, (size_t)d.nobs * sizeof(double));
  cp(h->rinv, d.rinv, (size_t)d.nobs * sizeof(double));
  if (launch_zero_ints(h->flags, 16, st) != hipSuccess) rs = RIOT_E_HIP;
  // the host vectors above go out of scope: wait for the copies
  if (hipStreamSynchronize(st) != hipSuccess) rs = RIOT_E_HIP;
  // the descriptor's host pointers are not kept
  h->d.obs_step = nullptr;
  h->d.obs_idx = nullptr;
  h->d.y = nullptr;
  h->d.rinv = nullptr;
  h->d.l_taps = nullptr;
  return rs;
}

riot_status riot_init(const riot_desc *desc, void *workspace, size_t bytes, void *hip_stream,
                      riot_handle **out) {
  if (!out) return RIOT_E_ARG;
  *out = nullptr;
  if (!desc_valid(desc) || !workspace) return RIOT_E_ARG;
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return RIOT_E_WORKSPACE;
  riot_handle *h = new (std::nothrow) riot_handle();
  if (!h) return RIOT_E_ARG;
  const riot_status rs =
      init_handle(h, desc, workspace, bytes, static_cast<hipStream_t>(hip_stream));
  if (rs != RIOT_OK) {
    delete h;
    return rs;
  }
  // the host-mapped word of the CholeskyQR pass control (without it, every pass is launched)
  void *hp = nullptr, *dp = nullptr;
  if (hipHostMalloc(&hp, 64, hipHostMallocCoherent | hipHostMallocMapped) == hipSuccess) {
    if (hipHostGetDevicePointer(&dp, hp, 0) == hipSuccess) {
      h->hflag = static_cast<int *>(hp);
      h->hflag_dev = static_cast<int *>(dp);
      __atomic_store_n(h->hflag, -1, __ATOMIC_RELEASE);
    } else {
      (void)hipHostFree(hp);
    }
  }
  (void)hipGetLastError();  // a failed pinned allocation only turns the host-read control off
  *out = h;
  return RIOT_OK;
}

void riot_free(riot_handle *h) { delete h; }

riot_status riot_set_pass_sync(riot_handle *h, int32_t on) {
  if (!h) return RIOT_E_ARG;
  h->pass_sync = on != 0;
  return RIOT_OK;
}

const char *riot_status_str(riot_status s) {
  switch (s) {
    case RIOT_OK: return "RIOT_OK";
    case RIOT_E_ARG: return "RIOT_E_ARG: invalid argument";
    case RIOT_E_HIP: return "RIOT_E_HIP: HIP runtime error";
    case RIOT_E_NOT_SPD: return "RIOT_E_NOT_SPD: Cholesky breakdown";
    case RIOT_E_SINGULAR: return "RIOT_E_SINGULAR: singular projected probe matrix";
    case RIOT_E_NONFINITE: return "RIOT_E_NONFINITE: non-finite result";
    case RIOT_E_NOCONV: return "RIOT_E_NOCONV: iteration cap reached";
    case RIOT_E_STATE: return "RIOT_E_STATE: call order violated";
    case RIOT_E_WORKSPACE: return "RIOT_E_WORKSPACE: workspace too small or misaligned";
    case RIOT_E_SCRATCH:
      return "RIOT_E_SCRATCH: problem larger than the no-allocation entry point's static scratch";
  }
  return "unknown riot_status";
}

// The handle's stream waits for a deferred gradient (no-op when none is pending).
static riot_status join_gradient(riot_handle *h) {
  if (h->grad_pending) {
    h->grad_pending = false;
    RIOT_HIP(hipStreamWaitEvent(h->st, h->ev_grad, 0));
  }
  return RIOT_OK;
}

riot_status riot_set_obs(riot_handle *h, const double *y) {
  if (!h || (h->d.nobs > 0 && !y)) return RIOT_E_ARG;
  if (riot_status js = join_gradient(h); js != RIOT_OK) return js;
  if (h->d.nobs > 0)
    RIOT_HIP(hipMemcpyAsync(h->y, y, (size_t)h->d.nobs * sizeof(double),
                            hipMemcpyDeviceToDevice, h->st));
  h->linearized = false;  // the stored innovation belongs to the old values
  return RIOT_OK;
}

// Trajectory, innovation and the gradient g = v - L lambda_0 with lambda_0 the adjoint sweep
// forced by R^{-1} d; with defer, the gradient's sweep and L run on the handle's second
// stream, beside whatever the caller enqueues next.
static riot_status linearize_impl(riot_handle *h, const double *x, const double *v, double *d,
                           double *grad, double *J_host, bool defer) {
  if (!h || !x || !grad || (h->d.nobs > 0 && !d)) return RIOT_E_ARG;
  if (h->d.ckpt_stride > 0) return RIOT_E_STATE;  // only a segment of the window fits
  riot_status rs = join_gradient(h);
  if (rs != RIOT_OK) return rs;
  const riot_desc &ds = h->d;
  hipStream_t st = h->st;
  RIOT_HIP(launch_trajectory(h->mv, ds.nsteps, x, nullptr, h->xs64, h->xs32, st));
  if (ds.nobs > 0)
    RIOT_HIP(launch_innovation(h->mv, h->xs64, ds.nobs, h->obs_step, h->obs_idx, h->y, h->rinv,
                               h->u_optr, h->u_olist, d, h->fgrad, h->fp32, st));
  hipStream_t gs = st;
  if (defer) {
    if (!h->side) {
      // default priority, no implicit synchronisation with the null stream
      RIOT_HIP(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
      RIOT_HIP(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
      RIOT_HIP(hipEventCreateWithFlags(&h->ev_grad, hipEventDisableTiming));
    }
    RIOT_HIP(hipEventRecord(h->ev_fork, st));
    RIOT_HIP(hipStreamWaitEvent(h->side, h->ev_fork, 0));
    gs = h->side;
  }
  RIOT_HIP(launch_tlad(h->mv, 1, 1, nullptr, h->LAM0, nullptr, h->fgrad, h->fp32, gs));
  RIOT_HIP(launch_apply_L(ds.n, h->w, h->taps, 1, h->LAM0, grad, v, 2, gs));
  if (defer) {
    RIOT_HIP(hipEventRecord(h->ev_grad, gs));
    h->grad_pending = true;
  }
  h->linearized = true;
  if (J_host) {
    RIOT_HIP(launch_cost(ds.n, v, ds.nobs, d, h->rinv, h->scal, st));
    RIOT_HIP(hipMemcpyAsync(J_host, h->scal, sizeof(double), hipMemcpyDeviceToHost, st));
    RIOT_HIP(hipStreamSynchronize(st));
  }
  return RIOT_OK;
}

riot_status riot_linearize(riot_handle *h, const double *x, const double *v, double *d,
                           double *grad, double *J_host) {
  return linearize_impl(h, x, v, d, grad, J_host, false);
}

riot_status riot_linearize_deferred(riot_handle *h, const double *x, const double *v, double *d,
                                    double *grad, double *J_host) {
  return linearize_impl(h, x, v, d, grad, J_host, true);
}

riot_status riot_join(riot_handle *h) {
  if (!h) return RIOT_E_ARG;
  return join_gradient(h);
}

riot_status riot_hess_apply(riot_handle *h, int32_t m, const double *W, double *Y,
                            int32_t add_identity) {
  if (!h || !W || !Y || m < 1 || m > h->d.m_max || W == Y) return RIOT_E_ARG;
  if (!h->linearized) return RIOT_E_STATE;
  return hess_apply_impl(h, m, W, Y, add_identity);
}

riot_status riot_rsvd(riot_handle *h, int32_t k, int32_t p_os, int32_t q, const double *Omega,
                      uint64_t seed, double *lambda, double *V, riot_rsvd_info *info) {
  if (!h || !lambda || !V || k < 1 || p_os < 0 || q < 0) return RIOT_E_ARG;
  const int n = h->d.n;
  const int m = k + p_os;
  if (m > h->d.m_max || m > n) return RIOT_E_ARG;
  if (!h->linearized) return RIOT_E_STATE;
  hipStream_t st = h->st;
  RIOT_HIP(launch_zero_ints(h->flags, 16, st));
  const double *Om = Omega;
  if (!Om) {
    RIOT_HIP(launch_philox_normal((long long)n * m, seed, 0, h->Om, st));
    Om = h->Om;
  }
  riot_status rs = hess_apply_impl(h, m, Om, h->Y, 0);
  if (rs != RIOT_OK) return rs;
  const double *Om_eff = Om;
  for (int it = 0; it < q; ++it) {
    rs = cholqr(la_of(h), n, m, h->Y, h->Q0, true, 0);
    if (rs != RIOT_OK) return rs;
    rs = hess_apply_impl(h, m, h->Q0, h->Y, 0);
    if (rs != RIOT_OK) return rs;
    Om_eff = h->Q0;
  }
  return sketch_eig(la_of(h), n, m, h->Y, Om_eff, lambda, V, info);
}

riot_status riot_proj_residual(riot_handle *h, int32_t m, const double *Q, const double *AQ,
                               double *rho_host) {
  if (!h || !Q || !AQ || !rho_host || m < 1 || m > h->d.m_max || m > h->d.n) return RIOT_E_ARG;
  if (Q == h->Q || AQ == h->Q) return RIOT_E_ARG;
  return proj_residual(la_of(h), h->d.n, m, Q, AQ, rho_host);
}

riot_status riot_increment(riot_handle *h, int32_t k, const double *lambda, const double *V,
                           const double *grad, riot_update mode, double *dz, double *dx,
                           double *dofs_host, int32_t *mode_used) {
  if (!h || !lambda || !V || !grad || !dz || !dx || dz == dx || k < 1 || k > h->d.n ||
      k > h->d.m_max)
    return RIOT_E_ARG;
  if (riot_status js = join_gradient(h); js != RIOT_OK) return js;
  if (mode != RIOT_ADAPTIVE && mode != RIOT_LRA && mode != RIOT_LRU) return RIOT_E_ARG;
  const int n = h->d.n;
  // dx = L dz is enqueued before any host synchronisation of the increment
  riot_status rs = sketch_increment(la_of(h), n, k, lambda, V, grad, mode, dz, nullptr, nullptr);
  if (rs != RIOT_OK) return rs;
  RIOT_HIP(launch_apply_L(n, h->w, h->taps, 1, dz, dx, nullptr, 0, h->st));
  if (dofs_host || mode_used) {
    LaSpace la = la_of(h);
    hipStream_t st = h->st;
    int mu = 0;
    if (mode_used) RIOT_HIP(launch_choose_mode(k, lambda, la.flags + 8, st));
    if (dofs_host)
      RIOT_HIP(hipMemcpyAsync(dofs_host, la.scal + 4, sizeof(double), hipMemcpyDeviceToHost, st));
    if (mode_used)
      RIOT_HIP(hipMemcpyAsync(&mu, la.flags + 8, sizeof(int), hipMemcpyDeviceToHost, st));
    RIOT_HIP(hipStreamSynchronize(st));
    if (mode_used) *mode_used = (mode == RIOT_ADAPTIVE) ? mu : (int32_t)mode;
  }
  return RIOT_OK;
}

// Deterministic LRA/LRU choice (Sec. 3.2.1): both increments from the same Ritz pairs, the
// nonlinear window from both updated states in one launch (one workgroup each), the
// non-quadratic costs, and the increment with the lower cost.
riot_status riot_increment_select(riot_handle *h, int32_t k, const double *lambda,
                                  const double *V, const double *grad, const double *x,
                                  const double *v, double *dz, double *dx, double *J_host,
                                  int32_t *mode_used) {
  if (!h || !lambda || !V || !grad || !x || !dz || !dx || k < 1 || k > h->d.m_max ||
      k > h->d.n)
    return RIOT_E_ARG;
  if (h->d.ckpt_stride > 0) return RIOT_E_STATE;
  if (dz == dx || dz == grad || dx == grad || dz == x || dx == x) return RIOT_E_ARG;
  riot_status rs = join_gradient(h);
  if (rs != RIOT_OK) return rs;
  const int n = h->d.n;
  const size_t U1 = (size_t)std::max(h->U, 1);
  hipStream_t st = h->st;
  double *dzc = h->sel, *dxc = dzc + 2 * (size_t)n, *xc = dxc + 2 * (size_t)n;
  double *vc = xc + 2 * (size_t)n, *xu = vc + 2 * (size_t)n, *J = xu + 2 * U1;
  RIOT_HIP(gemm_f64(1, 0, k, 1, n, 1.0, V, n, grad, n, 0.0, h->cvec, k, h->partial, kSplitK, st));
  RIOT_HIP(launch_increment_combine(n, k, lambda, V, h->cvec, grad, 0, dzc, h->scal + 4, st));
  RIOT_HIP(launch_increment_combine(n, k, lambda, V, h->cvec, grad, 1, dzc + n, h->scal + 4, st));
  RIOT_HIP(launch_apply_L(n, h->w, h->taps, 2, dzc, dxc, nullptr, 0, st));
  RIOT_HIP(launch_cand_state(n, 2, x, v, dzc, dxc, xc, vc, st));
  RIOT_HIP(launch_window_obs(h->mv, 2, xc, xu, st));
  RIOT_HIP(launch_cand_cost(n, 2, vc, h->d.nobs, h->U, h->y, h->rinv, h->u_of_o, xu, J, st));
  RIOT_HIP(launch_cand_select(n, 2, J, dzc, dxc, dz, dx, h->flags + 11, st));
  if (J_host || mode_used) {
    double jj[2];
    int mu = 0;
    RIOT_HIP(hipMemcpyAsync(jj, J, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    RIOT_HIP(hipMemcpyAsync(&mu, h->flags + 11, sizeof(int), hipMemcpyDeviceToHost, st));
    RIOT_HIP(hipStreamSynchronize(st));
    if (J_host) J_host[0] = jj[0], J_host[1] = jj[1];
    if (mode_used) *mode_used = mu;
  }
  return RIOT_OK;
}

riot_status riot_posterior_cov(riot_handle *h, int32_t k, const double *lambda, const double *V,
                               riot_update mode, double *W, double *coef, double *diag,
                               double *dense, int32_t *mode_used) {
  if (!h || !lambda || !V || !W || !coef || W == V || k < 1 || k > h->d.n) return RIOT_E_ARG;
  if (riot_status js = join_gradient(h); js != RIOT_OK) return js;
  if (mode != RIOT_ADAPTIVE && mode != RIOT_LRA && mode != RIOT_LRU) return RIOT_E_ARG;
  if (k > h->d.m_max) return RIOT_E_ARG;
  const int n = h->d.n;
  hipStream_t st = h->st;
  const int ml = mode == RIOT_LRA ? 0 : (mode == RIOT_LRU ? 1 : 2);
  RIOT_HIP(launch_apply_L(n, h->w, h->taps, k, V, W, nullptr, 0, st));
  RIOT_HIP(launch_postcov_diag(n, k, lambda, W, ml, h->base_diag, coef, diag, st));
  RIOT_HIP(launch_choose_mode(k, lambda, h->flags + 9, st));
  if (mode == RIOT_LRA) RIOT_HIP(launch_zero_ints(h->flags + 9, 1, st));
  if (dense) {
    RIOT_HIP(launch_scale_cols(n, k, W, coef, h->LAM, st));
    RIOT_HIP(gemm_f64(0, 1, n, n, k, 1.0, h->LAM, n, W, n, 0.0, dense, n, nullptr, 1, st));
    RIOT_HIP(launch_dense_B(n, h->brow, 1.0, dense, mode == RIOT_LRU ? nullptr : h->flags + 9, st));
  }
  if (mode_used) {
    int mu = 0;
    RIOT_HIP(hipMemcpyAsync(&mu, h->flags + 9, sizeof(int), hipMemcpyDeviceToHost, st));
    RIOT_HIP(hipStreamSynchronize(st));
    *mode_used = (mode == RIOT_ADAPTIVE) ? mu : (int32_t)mode;
  }
  return RIOT_OK;
}

riot_status riot_cg(riot_handle *h, const double *grad, int32_t iters, double rtol, double *dz,
                    double *iterates, int32_t *used) {
  if (!h || !grad || !dz || iters < 0) return RIOT_E_ARG;
  if (riot_status js = join_gradient(h); js != RIOT_OK) return js;
  if (!h->linearized) return RIOT_E_STATE;
  hipStream_t st = h->st;
  RIOT_HIP(launch_cg(h->mv, h->w, h->taps, grad, iters, rtol, dz, iterates, h->cgv, h->f,
                     h->flags + 10, h->fp32, st));
  if (used) {
    int u = 0;
    RIOT_HIP(hipMemcpyAsync(&u, h->flags + 10, sizeof(int), hipMemcpyDeviceToHost, st));
    RIOT_HIP(hipStreamSynchronize(st));
    *used = u;
  }
  return RIOT_OK;
}

riot_status riot_tl_apply(riot_handle *h, int32_t m, const double *X, double *Z) {
  if (!h || !X || (!Z && h->d.nobs > 0) || m < 1 || m > h->d.m_max) return RIOT_E_ARG;
  if (riot_status js = join_gradient(h); js != RIOT_OK) return js;
  if (!h->linearized) return RIOT_E_STATE;
  hipStream_t st = h->st;
  RIOT_HIP(launch_tlad(h->mv, m, 2, X, nullptr, h->f, nullptr, h->fp32, st));
  RIOT_HIP(launch_obs_gather(h->d.nobs, h->U, m, h->u_of_o, h->f, Z, h->fp32, st));
  return RIOT_OK;
}

riot_status riot_ad_apply(riot_handle *h, int32_t m, const double *Fo, double *X) {
  if (!h || !X || (!Fo && h->d.nobs > 0) || m < 1 || m > h->d.m_max) return RIOT_E_ARG;
  if (riot_status js = join_gradient(h); js != RIOT_OK) return js;
  if (!h->linearized) return RIOT_E_STATE;
  hipStream_t st = h->st;
  RIOT_HIP(launch_obs_scatter(h->d.nobs, h->U, m, h->u_optr, h->u_olist, Fo, h->f, h->fp32, st));
  RIOT_HIP(launch_tlad(h->mv, m, 3, nullptr, X, h->f, nullptr, h->fp32, st));
  return RIOT_OK;
}

// ---------------------------------------------------------------------------
// Spectral preconditioner and rotation across outer loops (Alg. 3, precond / rotation).
// ---------------------------------------------------------------------------

static riot_status precond_apply_impl(riot_handle *h, int nlev, const double *const *V,
                                      const int32_t *mj, const double *const *lam, int op, int m,
                                      double *X) {
  const int n = h->d.n;
  hipStream_t st = h->st;
  const double power = op == 2 ? 0.5 : -0.5;
  for (int q = 0; q < nlev; ++q) {
    const int j = op == 0 ? nlev - 1 - q : q;  // P applies the last factor first
    const int k = mj[j];
    RIOT_HIP(gemm_f64(1, 0, k, m, n, 1.0, V[j], n, X, n, 0.0, h->B1, k, h->partial, kSplitK, st));
    RIOT_HIP(launch_precond_scale(k, m, lam[j], power, h->B1, st));
    RIOT_HIP(gemm_f64(0, 0, n, m, k, 1.0, V[j], n, h->B1, k, 1.0, X, n, nullptr, 1, st));
  }
  return RIOT_OK;
}

static bool precond_args_ok(const riot_handle *h, int nlev, const double *const *V,
                            const int32_t *mj, const double *const *lam, int m) {
  if (nlev < 0 || m < 1 || m > h->d.m_max) return false;
  if (nlev > 0 && (!V || !mj || !lam)) return false;
  for (int j = 0; j < nlev; ++j)
    if (!V[j] || !lam[j] || mj[j] < 1 || mj[j] > h->d.m_max || mj[j] > h->d.n) return false;
  return true;
}

riot_status riot_precond_apply(riot_handle *h, int32_t nlev, const double *const *V,
                               const int32_t *mj, const double *const *lam, int32_t op,
                               int32_t m, double *X) {
  if (!h || !X || op < 0 || op > 2 || !precond_args_ok(h, nlev, V, mj, lam, m)) return RIOT_E_ARG;
  if (riot_status js = join_gradient(h); js != RIOT_OK) return js;
  return precond_apply_impl(h, nlev, V, mj, lam, op, m, X);
}

riot_status riot_precond_hess_apply(riot_handle *h, int32_t nlev, const double *const *V,
                                    const int32_t *mj, const double *const *lam, int32_t m,
                                    const double *W, double *Y) {
  if (!h || !W || !Y || W == Y || !precond_args_ok(h, nlev, V, mj, lam, m)) return RIOT_E_ARG;
  if (h->d.ckpt_stride > 0) return RIOT_E_STATE;
  if (riot_status js = join_gradient(h); js != RIOT_OK) return js;
  if (!h->linearized) return RIOT_E_STATE;
  const int n = h->d.n;
  hipStream_t st = h->st;
  // T = P W; Y = (I + A) T; Y <- P^T Y - W
  RIOT_HIP(hipMemcpyAsync(h->Q0, W, (size_t)n * m * sizeof(double), hipMemcpyDeviceToDevice, st));
  riot_status rs = precond_apply_impl(h, nlev, V, mj, lam, 0, m, h->Q0);
  if (rs != RIOT_OK) return rs;
  rs = hess_apply_impl(h, m, h->Q0, Y, 1);
  if (rs != RIOT_OK) return rs;
  rs = precond_apply_impl(h, nlev, V, mj, lam, 1, m, Y);
  if (rs != RIOT_OK) return rs;
  RIOT_HIP(launch_axpby((long long)n * m, 1.0, Y, -1.0, W, st));
  return RIOT_OK;
}

riot_status riot_orth(riot_handle *h, int32_t m, const double *X, double *Q) {
  if (!h || !X || !Q || m < 1 || m > h->d.m_max || m > h->d.n) return RIOT_E_ARG;
  if (Q == h->Q) return RIOT_E_ARG;
  if (riot_status js = join_gradient(h); js != RIOT_OK) return js;
  LaSpace la = la_of(h);
  RIOT_HIP(launch_zero_ints(la.flags, 16, h->st));
  return cholqr(la, h->d.n, m, X, Q, true, 0);
}

riot_status riot_project_out(riot_handle *h, int32_t r, const double *U, int32_t m, double *X) {
  if (!h || !U || !X || r < 1 || m < 1 || r > h->d.m_max || m > h->d.m_max || r > h->d.n)
    return RIOT_E_ARG;
  if (riot_status js = join_gradient(h); js != RIOT_OK) return js;
  const int n = h->d.n;
  hipStream_t st = h->st;
  for (int pass = 0; pass < 2; ++pass) {  // twice: classical Gram-Schmidt to rounding level
    RIOT_HIP(gemm_f64(1, 0, r, m, n, 1.0, U, n, X, n, 0.0, h->B2, r, h->partial, kSplitK, st));
    RIOT_HIP(gemm_f64(0, 0, n, m, r, -1.0, U, n, h->B2, r, 1.0, X, n, nullptr, 1, st));
  }
  return RIOT_OK;
}

riot_status riot_outer_update(riot_handle *h, const double *dv, double *v, double *x) {
  if (!h || !dv || !v || !x || dv == v || dv == x || v == x) return RIOT_E_ARG;
  if (riot_status js = join_gradient(h); js != RIOT_OK) return js;
  const int n = h->d.n;
  hipStream_t st = h->st;
  RIOT_HIP(launch_apply_L(n, h->w, h->taps, 1, dv, h->LW, nullptr, 0, st));
  RIOT_HIP(launch_axpby(n, 1.0, x, 1.0, h->LW, st));
  RIOT_HIP(launch_axpby(n, 1.0, v, 1.0, dv, st));
  return RIOT_OK;
}

// ---------------------------------------------------------------------------
// VarBL (Alg. 2): perturbed gradient samples and the block Lanczos inner loop.
// ---------------------------------------------------------------------------

riot_status riot_gradient_sample(riot_handle *h, const double *x, const double *v,
                                 const double *eps_b, const double *eps_o, double *grad) {
  if (!h || !x || !grad || (h->d.nobs > 0 && !eps_o)) return RIOT_E_ARG;
  if (grad == x || grad == v || grad == eps_b) return RIOT_E_ARG;
  if (h->d.ckpt_stride > 0) return RIOT_E_STATE;
  if (riot_status js = join_gradient(h); js != RIOT_OK) return js;
  const riot_desc &ds = h->d;
  const int n = ds.n, no = ds.nobs;
  hipStream_t st = h->st;
  const double *xj = x, *vj = v;
  if (eps_b) {
    double *xb_ = h->sel, *vb_ = h->sel + n;
    RIOT_HIP(launch_apply_L(n, h->w, h->taps, 1, eps_b, h->LW, nullptr, 0, st));
    RIOT_HIP(hipMemcpyAsync(xb_, x, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
    RIOT_HIP(launch_axpby(n, 1.0, xb_, 1.0, h->LW, st));
    RIOT_HIP(hipMemcpyAsync(vb_, eps_b, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (v) RIOT_HIP(launch_axpby(n, 1.0, vb_, 1.0, v, st));
    xj = xb_, vj = vb_;
  }
  // the handle's trajectory becomes the perturbed one: it must be linearised again
  h->linearized = false;
  RIOT_HIP(launch_trajectory(h->mv, ds.nsteps, xj, nullptr, h->xs64, h->xs32, st));
  if (no > 0) {
    RIOT_HIP(launch_obs_perturb(no, h->y, h->rinv, eps_o, h->pso, st));
    RIOT_HIP(launch_innovation(h->mv, h->xs64, no, h->obs_step, h->obs_idx, h->pso, h->rinv,
                               h->u_optr, h->u_olist, h->pso + no, h->fgrad, h->fp32, st));
  }
  RIOT_HIP(launch_tlad(h->mv, 1, 1, nullptr, h->LAM0, nullptr, h->fgrad, h->fp32, st));
  RIOT_HIP(launch_apply_L(n, h->w, h->taps, 1, h->LAM0, grad, vj, 2, st));
  return RIOT_OK;
}

riot_status riot_block_lanczos(riot_handle *h, int32_t l, int32_t iters, const double *B,
                               const double *grad, double *lambda, double *U, double *dz,
                               double *dx) {
  if (!h || !B || !grad || !lambda || !U || !dz || !dx || l < 1 || iters < 1) return RIOT_E_ARG;
  const int n = h->d.n, ml = l * iters;
  if (ml > h->d.m_max || ml > n || dz == dx || dz == grad || dx == grad) return RIOT_E_ARG;
  if (h->d.ckpt_stride > 0) return RIOT_E_STATE;
  if (riot_status js = join_gradient(h); js != RIOT_OK) return js;
  if (!h->linearized) return RIOT_E_STATE;
  hipStream_t st = h->st;
  LaSpace la = la_of(h);
  RIOT_HIP(launch_zero_ints(la.flags, 16, st));
  double *Q = h->Q, *Y = h->Y, *T = h->K;
  auto blk = [&](int i, int j) { return T + (size_t)j * l * ml + (size_t)i * l; };
  riot_status rs = cholqr(la, n, l, B, Q, true, 0);
  if (rs != RIOT_OK) return rs;
  for (int i = 0; i < iters; ++i) {
    double *Qi = Q + (size_t)i * l * n;
    rs = hess_apply_impl(h, l, Qi, Y, 0);
    if (rs != RIOT_OK) return rs;
    // M_i = Q_i^T Y_i
    RIOT_HIP(gemm_f64(1, 0, l, l, n, 1.0, Qi, n, Y, n, 0.0, blk(i, i), ml, h->partial, kSplitK, st));
    if (i == iters - 1) break;
    // R = Y_i - Q_i M_i - Q_{i-1} W_{i-1}^T, orthogonalised against every block so far
    RIOT_HIP(gemm_f64(0, 0, n, l, l, -1.0, Qi, n, blk(i, i), ml, 1.0, Y, n, nullptr, 1, st));
    if (i > 0)
      RIOT_HIP(gemm_f64(0, 0, n, l, l, -1.0, Qi - (size_t)l * n, n, blk(i - 1, i), ml, 1.0, Y, n,
                        nullptr, 1, st));
    const int done = (i + 1) * l;
    for (int pass = 0; pass < 2; ++pass) {
      RIOT_HIP(gemm_f64(1, 0, done, l, n, 1.0, Q, n, Y, n, 0.0, h->B2, done, h->partial, kSplitK,
                        st));
      RIOT_HIP(gemm_f64(0, 0, n, l, done, -1.0, Q, n, h->B2, done, 1.0, Y, n, nullptr, 1, st));
    }
    // Q_{i+1} W_i = R: orthonormal block by CholeskyQR, W_i = Q_{i+1}^T R (and its transpose)
    double *Qn = Qi + (size_t)l * n;
    rs = cholqr(la, n, l, Y, Qn, true, 0);
    if (rs != RIOT_OK) return rs;
    RIOT_HIP(gemm_f64(1, 0, l, l, n, 1.0, Qn, n, Y, n, 0.0, blk(i + 1, i), ml, h->partial, kSplitK,
                      st));
    RIOT_HIP(gemm_f64(1, 0, l, l, n, 1.0, Y, n, Qn, n, 0.0, blk(i, i + 1), ml, h->partial, kSplitK,
                      st));
  }
  // blocks outside the band are zero
  RIOT_HIP(launch_block_band_zero(ml, l, T, st));
  RIOT_HIP(launch_symmetrize(ml, T, la.scal + 1, la.partial, st));
  RIOT_HIP(launch_eig(ml, T, lambda, la.Zs, la.sywork, la.flags + 2, st));
  RIOT_HIP(gemm_f64(0, 0, n, ml, ml, 1.0, Q, n, la.Zs, ml, 0.0, U, n, nullptr, 1, st));
  // dz = -sum (1 + l_i)^{-1} u_i u_i^T g (LRA), dx = L dz
  RIOT_HIP(gemm_f64(1, 0, ml, 1, n, 1.0, U, n, grad, n, 0.0, la.cvec, ml, la.partial, kSplitK, st));
  RIOT_HIP(launch_increment_combine(n, ml, lambda, U, la.cvec, grad, 0, dz, la.scal + 4, st));
  RIOT_HIP(launch_apply_L(n, h->w, h->taps, 1, dz, dx, nullptr, 0, st));
  return RIOT_OK;
}

// ---------------------------------------------------------------------------
// RIOT-PSAS (Appendix algorithm): the randomized solve in observation space.
// ---------------------------------------------------------------------------

riot_status riot_psas_hess_apply(riot_handle *h, int32_t m, const double *W, double *Y) {
  if (!h || !W || !Y || W == Y || m < 1 || m > h->d.m_max || h->d.nobs < 1) return RIOT_E_ARG;
  if (h->d.ckpt_stride > 0) return RIOT_E_STATE;
  if (riot_status js = join_gradient(h); js != RIOT_OK) return js;
  if (!h->linearized) return RIOT_E_STATE;
  const int n = h->d.n, no = h->d.nobs;
  hipStream_t st = h->st;
  // X = G^T R^{-1/2} W, then B X = L (L X), then R^{-1/2} G B X at the observations
  RIOT_HIP(launch_obs_scatter(no, h->U, m, h->u_optr, h->u_olist, W, h->f, h->fp32, st, h->rinv));
  RIOT_HIP(launch_tlad(h->mv, m, 3, nullptr, h->LAM, h->f, nullptr, h->fp32, st));
  RIOT_HIP(launch_apply_L(n, h->w, h->taps, m, h->LAM, h->LW, nullptr, 0, st));
  RIOT_HIP(launch_apply_L(n, h->w, h->taps, m, h->LW, h->LAM, nullptr, 0, st));
  RIOT_HIP(launch_tlad(h->mv, m, 2, h->LAM, nullptr, h->f, nullptr, h->fp32, st));
  RIOT_HIP(launch_obs_gather(no, h->U, m, h->u_of_o, h->f, Y, h->fp32, st, h->rinv));
  return RIOT_OK;
}

riot_status riot_psas_rhs(riot_handle *h, const double *d, const double *xb_minus_x,
                          double *rhs) {
  if (!h || !d || !rhs || d == rhs || h->d.nobs < 1) return RIOT_E_ARG;
  if (h->d.ckpt_stride > 0) return RIOT_E_STATE;
  if (riot_status js = join_gradient(h); js != RIOT_OK) return js;
  if (!h->linearized) return RIOT_E_STATE;
  const int no = h->d.nobs;
  hipStream_t st = h->st;
  const double *bp = nullptr;
  if (xb_minus_x) {
    RIOT_HIP(launch_tlad(h->mv, 1, 2, xb_minus_x, nullptr, h->f, nullptr, h->fp32, st));
    RIOT_HIP(launch_obs_gather(no, h->U, 1, h->u_of_o, h->f, h->pso, h->fp32, st));
    bp = h->pso;
  }
  RIOT_HIP(launch_psas_rhs(no, h->rinv, d, bp, rhs, st));
  return RIOT_OK;
}

riot_status riot_psas_increment(riot_handle *h, int32_t k, const double *lambda, const double *U,
                                const double *rhs, riot_update mode, double *dw, double *dx,
                                int32_t *mode_used) {
  const int no = h ? h->d.nobs : 0;
  if (!h || !lambda || !U || !rhs || !dw || !dx || no < 1 || k < 1 || k > no ||
      k > h->d.m_max)
    return RIOT_E_ARG;
  if (mode != RIOT_ADAPTIVE && mode != RIOT_LRA && mode != RIOT_LRU) return RIOT_E_ARG;
  if (dw == rhs || (const double *)dx == U) return RIOT_E_ARG;
  if (h->d.ckpt_stride > 0) return RIOT_E_STATE;
  if (riot_status js = join_gradient(h); js != RIOT_OK) return js;
  if (!h->linearized) return RIOT_E_STATE;
  const int n = h->d.n;
  hipStream_t st = h->st;
  double *t = h->pso + no;
  // c = U^T rhs; t = -(LRA or LRU combination of rhs); dw = -R^{-1/2} t
  RIOT_HIP(gemm_f64(1, 0, k, 1, no, 1.0, U, no, rhs, no, 0.0, h->cvec, k, h->partial, kSplitK, st));
  const int ml = mode == RIOT_LRA ? 0 : (mode == RIOT_LRU ? 1 : 2);
  RIOT_HIP(launch_increment_combine(no, k, lambda, U, h->cvec, rhs, ml, t, h->scal + 4, st));
  RIOT_HIP(launch_psas_scale(no, h->rinv, t, dw, st));
  // dx = B G^T dw = L (L (G^T dw))
  RIOT_HIP(launch_obs_scatter(no, h->U, 1, h->u_optr, h->u_olist, dw, h->f, h->fp32, st));
  RIOT_HIP(launch_tlad(h->mv, 1, 3, nullptr, h->LAM, h->f, nullptr, h->fp32, st));
  RIOT_HIP(launch_apply_L(n, h->w, h->taps, 1, h->LAM, h->LW, nullptr, 0, st));
  RIOT_HIP(launch_apply_L(n, h->w, h->taps, 1, h->LW, dx, nullptr, 0, st));
  if (mode_used) {
    int mu = 0;
    RIOT_HIP(launch_choose_mode(k, lambda, h->flags + 8, st));
    RIOT_HIP(hipMemcpyAsync(&mu, h->flags + 8, sizeof(int), hipMemcpyDeviceToHost, st));
    RIOT_HIP(hipStreamSynchronize(st));
    *mode_used = (mode == RIOT_ADAPTIVE) ? mu : (int32_t)mode;
  }
  return RIOT_OK;
}

// ---------------------------------------------------------------------------
// Checkpointed observation map, tangent and adjoint
// ---------------------------------------------------------------------------

static ModelView segment_view(const riot_handle *h, int s, int steps) {
  ModelView mv = h->mv;
  mv.T = steps;
  mv.stepk = h->stepk + (size_t)s * h->d.ckpt_stride;
  return mv;
}

static int segment_steps(const riot_handle *h, int s) {
  const int c = h->d.ckpt_stride, T = h->d.nsteps;
  return std::min(c, T - s * c);
}

static int segment_count(const riot_handle *h) {
  const int c = h->d.ckpt_stride, T = h->d.nsteps;
  return T > 0 ? (T + c - 1) / c : 0;
}

riot_status riot_ckpt_forward(riot_handle *h, const double *x0, double *ckpt, double *obs) {
  if (!h || !x0 || !ckpt || (h->d.nobs > 0 && !obs)) return RIOT_E_ARG;
  if (riot_status js = join_gradient(h); js != RIOT_OK) return js;
  if (h->d.ckpt_stride <= 0) return RIOT_E_STATE;
  const int n = h->d.n, c = h->d.ckpt_stride, ns = segment_count(h);
  hipStream_t st = h->st;
  RIOT_HIP(hipMemcpyAsync(ckpt, x0, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (ns == 0) {
    RIOT_HIP(launch_trajectory(segment_view(h, 0, 0), 0, x0, nullptr, h->xs64, h->xs32, st));
    RIOT_HIP(launch_obs_value(segment_view(h, 0, 0), h->xs64, h->d.nobs, h->obs_step, h->obs_idx,
                              0, true, obs, st));
    return RIOT_OK;
  }
  for (int s = 0; s < ns; ++s) {
    const int steps = segment_steps(h, s);
    const ModelView mv = segment_view(h, s, steps);
    RIOT_HIP(launch_trajectory(mv, steps, ckpt + (size_t)s * n, ckpt + (size_t)(s + 1) * n,
                               h->xs64, h->xs32, st));
    RIOT_HIP(launch_obs_value(mv, h->xs64, h->d.nobs, h->obs_step, h->obs_idx, s * c, s == 0, obs,
                              st));
  }
  return RIOT_OK;
}

riot_status riot_ckpt_tangent(riot_handle *h, int32_t m, const double *ckpt, const double *dX0,
                              double *dObs) {
  if (!h || !ckpt || !dX0 || (h->d.nobs > 0 && !dObs) || m < 1 || m > h->d.m_max)
    return RIOT_E_ARG;
  if (riot_status js = join_gradient(h); js != RIOT_OK) return js;
  if (h->d.ckpt_stride <= 0) return RIOT_E_STATE;
  const int n = h->d.n, ns = std::max(segment_count(h), 1);
  hipStream_t st = h->st;
  // tangent states ping-pong between two n x m blocks of the workspace
  const double *cur = dX0;
  double *bufs[2] = {h->LW, h->LAM};
  for (int s = 0; s < ns; ++s) {
    const int steps = segment_count(h) ? segment_steps(h, s) : 0;
    const ModelView mv = segment_view(h, s, steps);
    RIOT_HIP(launch_trajectory(mv, steps, ckpt + (size_t)s * n, nullptr, h->xs64, h->xs32, st));
    double *next = bufs[s & 1];
    RIOT_HIP(launch_tlad(mv, m, 2 | kTladOutState | (s > 0 ? kTladSkip0 : 0), cur, next, h->f,
                         nullptr, h->fp32, st));
    cur = next;
  }
  RIOT_HIP(launch_obs_gather(h->d.nobs, h->U, m, h->u_of_o, h->f, dObs, h->fp32, st));
  return RIOT_OK;
}

riot_status riot_ckpt_adjoint(riot_handle *h, int32_t m, const double *ckpt, const double *gObs,
                              double *gX0) {
  if (!h || !ckpt || !gX0 || (h->d.nobs > 0 && !gObs) || m < 1 || m > h->d.m_max)
    return RIOT_E_ARG;
  if (riot_status js = join_gradient(h); js != RIOT_OK) return js;
  if (h->d.ckpt_stride <= 0) return RIOT_E_STATE;
  const int n = h->d.n, ns = std::max(segment_count(h), 1);
  hipStream_t st = h->st;
  RIOT_HIP(launch_obs_scatter(h->d.nobs, h->U, m, h->u_optr, h->u_olist, gObs, h->f, h->fp32, st));
  // adjoint states ping-pong between two n x m blocks; the last segment starts from zero
  double *bufs[2] = {h->LW, h->LAM};
  const double *cur = nullptr;
  for (int s = ns - 1, i = 0; s >= 0; --s, ++i) {
    const int steps = segment_count(h) ? segment_steps(h, s) : 0;
    const ModelView mv = segment_view(h, s, steps);
    RIOT_HIP(launch_trajectory(mv, steps, ckpt + (size_t)s * n, nullptr, h->xs64, h->xs32, st));
    double *next = s == 0 ? gX0 : bufs[i & 1];
    const int mode = 3 | (cur ? kTladInitLam : 0) | (s > 0 ? kTladSkip0 : 0);
    RIOT_HIP(launch_tlad(mv, m, mode, cur, next, h->f, nullptr, h->fp32, st));
    cur = next;
  }
  return RIOT_OK;
}

riot_status riot_gn_apply(riot_handle *h, int32_t m, const double *X, double *Y) {
  if (!h || !X || !Y || X == Y || m < 1 || m > h->d.m_max) return RIOT_E_ARG;
  if (riot_status js = join_gradient(h); js != RIOT_OK) return js;
  if (!h->linearized) return RIOT_E_STATE;
  RIOT_HIP(launch_tlad(h->mv, m, 0, X, Y, h->f, nullptr, h->fp32, h->st));
  return RIOT_OK;
}

riot_status riot_forecast(riot_handle *h, const double *x0, int32_t nsteps, double *xout) {
  if (!h || !x0 || !xout || nsteps < 0) return RIOT_E_ARG;
  if (riot_status js = join_gradient(h); js != RIOT_OK) return js;
  RIOT_HIP(launch_trajectory(h->mv, nsteps, x0, xout, nullptr, nullptr, h->st));
  return RIOT_OK;
}

riot_status riot_apply_L(riot_handle *h, int32_t m, const double *X, double *Y) {
  if (!h || !X || !Y || m < 1 || X == Y) return RIOT_E_ARG;
  if (riot_status js = join_gradient(h); js != RIOT_OK) return js;
  RIOT_HIP(launch_apply_L(h->d.n, h->w, h->taps, m, X, Y, nullptr, 0, h->st));
  return RIOT_OK;
}

riot_status riot_philox_normal(riot_handle *h, int32_t n, int32_t m, uint64_t seed,
                               uint64_t stream, double *out) {
  if (!h || !out || n < 1 || m < 1) return RIOT_E_ARG;
  RIOT_HIP(launch_philox_normal((long long)n * m, seed, stream, out, h->st));
  return RIOT_OK;
}


// ===========================================================================
// Batches of independent problems (a persistent TL/AD launch over all probes of all
// problems, batched linear algebra, graph capture of the whole inner loop).
// ===========================================================================

}  // extern "C"

namespace {

constexpr int kBatchMaxN = 2048;  // NT <= 256 threads at 8 elements per lane
constexpr int kBatchMaxM = 278;   // within the register-tile tridiagonalisation bound (279)

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

struct riot_batch {
  int nprob = 0;
  hipStream_t st = nullptr;
  bool fp32 = false;
  int cus = 256;
  std::vector<riot_handle *> hs;
  std::vector<int> n, m, T, nobs;
  std::vector<size_t> off_n, off_m, off_nm, off_obs;
  size_t tot_n = 0, tot_m = 0, tot_nm = 0, tot_obs = 0;
  int maxn = 0, maxm = 0, maxU = 0, maxext = 0;
  // packed caller-visible buffers
  double *X = nullptr, *Gr = nullptr, *Lam = nullptr, *V = nullptr, *Dz = nullptr, *Dx = nullptr,
         *D = nullptr;
  // device job tables
  riot::TrajJob *traj = nullptr;
  riot::InnovJob *innov = nullptr;
  riot::TladProb *grad_probs = nullptr, *hvp_probs = nullptr;
  riot::TladTile *tiles = nullptr;  // [grad wg | grad wave | hvp wg | hvp wave]
  int n_grad_wg = 0, n_grad_wave = 0, n_hvp_wg = 0, n_hvp_wave = 0, tile_cap = 0;
  int *counters = nullptr;
  long long *clk = nullptr;  // per-tile start/end clocks of riot_batch_profile (2 per tile)
  riot::ApplyLJobE *aL_grad = nullptr, *aL_in = nullptr, *aL_out = nullptr, *aL_dx = nullptr;
  riot::PhiloxJob *philox = nullptr;
  riot::CopyJob *cp_Y = nullptr, *cp_B2 = nullptr;
  riot::CqJob *cq_Y = nullptr, *cq_B2 = nullptr;
  riot::GemmJob *gram_Q = nullptr, *gram_Z = nullptr, *g_B1 = nullptr, *g_B2 = nullptr,
                *g_K = nullptr, *g_V = nullptr, *g_c = nullptr;
  riot::CholJob *ch_Q = nullptr, *ch_Z = nullptr;
  riot::TrsmJob *tr_Q = nullptr, *tr_Z = nullptr, *tr_B1 = nullptr;
  riot::SymJob *sym = nullptr;
  riot::EigJob *eig = nullptr;
  riot::IncJob *inc = nullptr;
  // layout chosen by riot_batch_autotune (or the defaults)
  int nwg = 0;
  int wave_max_nt = 64;  // problems with NT <= this use member-per-wave tiles (0: none)
  uint64_t seed = 0;
  hipGraphExec_t graph = nullptr;
  ~riot_batch() {
    if (graph) (void)hipGraphExecDestroy(graph);
    for (auto *h : hs) delete h;
  }
};

namespace {

template <typename T>
riot_status upload(T *dst, const std::vector<T> &src, hipStream_t st) {
  if (src.empty()) return RIOT_OK;
  return hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st) ==
                 hipSuccess
             ? RIOT_OK
             : RIOT_E_HIP;
}

bool batch_desc_ok(const riot_desc &d) {
  return desc_valid(&d) && d.n % 8 == 0 && d.n <= kBatchMaxN && d.m_max <= kBatchMaxM &&
         d.m_max <= d.n && d.ckpt_stride == 0;
}

// Workspace of the batch-level part: packed buffers and job tables.
struct BatchCarve {
  size_t off = 0;
  char *base;
  explicit BatchCarve(void *b) : base(static_cast<char *>(b)) {}
  template <typename T>
  T *take(size_t count) {
    off = align256(off);
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += std::max<size_t>(count, 1) * sizeof(T);
    return p;
  }
};

size_t batch_carve(riot_batch &b, void *base, size_t tiles_cap) {
  BatchCarve c(base);
  const size_t P = b.nprob;
  b.X = c.take<double>(b.tot_n);
  b.Gr = c.take<double>(b.tot_n);
  b.Dz = c.take<double>(b.tot_n);
  b.Dx = c.take<double>(b.tot_n);
  b.Lam = c.take<double>(b.tot_m);
  b.V = c.take<double>(b.tot_nm);
  b.D = c.take<double>(b.tot_obs);
  b.traj = c.take<riot::TrajJob>(P);
  b.innov = c.take<riot::InnovJob>(P);
  b.grad_probs = c.take<riot::TladProb>(P);
  b.hvp_probs = c.take<riot::TladProb>(P);
  b.tiles = c.take<riot::TladTile>(tiles_cap);
  b.counters = c.take<int>(4);
  b.clk = c.take<long long>(2 * tiles_cap);
  b.aL_grad = c.take<riot::ApplyLJobE>(P);
  b.aL_in = c.take<riot::ApplyLJobE>(P);
  b.aL_out = c.take<riot::ApplyLJobE>(P);
  b.aL_dx = c.take<riot::ApplyLJobE>(P);
  b.philox = c.take<riot::PhiloxJob>(P);
  b.cp_Y = c.take<riot::CopyJob>(P);
  b.cp_B2 = c.take<riot::CopyJob>(P);
  b.cq_Y = c.take<riot::CqJob>(P);
  b.cq_B2 = c.take<riot::CqJob>(P);
  b.gram_Q = c.take<riot::GemmJob>(P);
  b.gram_Z = c.take<riot::GemmJob>(P);
  b.g_B1 = c.take<riot::GemmJob>(P);
  b.g_B2 = c.take<riot::GemmJob>(P);
  b.g_K = c.take<riot::GemmJob>(P);
  b.g_V = c.take<riot::GemmJob>(P);
  b.g_c = c.take<riot::GemmJob>(P);
  b.ch_Q = c.take<riot::CholJob>(P);
  b.ch_Z = c.take<riot::CholJob>(P);
  b.tr_Q = c.take<riot::TrsmJob>(P);
  b.tr_Z = c.take<riot::TrsmJob>(P);
  b.tr_B1 = c.take<riot::TrsmJob>(P);
  b.sym = c.take<riot::SymJob>(P);
  b.eig = c.take<riot::EigJob>(P);
  b.inc = c.take<riot::IncJob>(P);
  return align256(c.off);
}

// Tile lists of the two persistent launches for the current layout: longest first.
riot_status batch_build_tiles(riot_batch &b) {
  std::vector<int> order(b.nprob);
  for (int j = 0; j < b.nprob; ++j) order[j] = j;
  auto cost = [&](int j) { return (double)b.T[j] * (double)b.n[j]; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cost(a) > cost(c); });
  std::vector<riot::TladTile> gw, gv, hw, hv;
  for (int j : order) {
    const bool wave = b.hs[j]->NT <= b.wave_max_nt;
    (wave ? gv : gw).push_back({j, 0});
    for (int i = 0; i < b.m[j]; ++i) (wave ? hv : hw).push_back({j, i});
  }
  std::vector<riot::TladTile> all;
  all.insert(all.end(), gw.begin(), gw.end());
  all.insert(all.end(), gv.begin(), gv.end());
  all.insert(all.end(), hw.begin(), hw.end());
  all.insert(all.end(), hv.begin(), hv.end());
  if ((int)all.size() > b.tile_cap) return RIOT_E_ARG;
  b.n_grad_wg = (int)gw.size();
  b.n_grad_wave = (int)gv.size();
  b.n_hvp_wg = (int)hw.size();
  b.n_hvp_wave = (int)hv.size();
  return upload(b.tiles, all, b.st);
}

riot_status batch_tables(riot_batch &b) {
  const int P = b.nprob;
  std::vector<riot::TrajJob> traj(P);
  std::vector<riot::InnovJob> innov(P);
  std::vector<riot::TladProb> gp(P), hp(P);
  std::vector<riot::ApplyLJobE> aG(P), aI(P), aO(P), aD(P);
  std::vector<riot::PhiloxJob> ph(P);
  std::vector<riot::CopyJob> cY(P), cB(P);
  std::vector<riot::CqJob> qY(P), qB(P);
  std::vector<riot::GemmJob> gQ(P), gZ(P), g1(P), g2(P), gK(P), gV(P), gc(P);
  std::vector<riot::CholJob> hQ(P), hZ(P);
  std::vector<riot::TrsmJob> tQ(P), tZ(P), t1(P);
  std::vector<riot::SymJob> sy(P);
  std::vector<riot::EigJob> eg(P);
  std::vector<riot::IncJob> ic(P);
  const double u = 0x1.0p-53;
  for (int j = 0; j < P; ++j) {
    riot_handle &h = *b.hs[j];
    const int n = b.n[j], m = b.m[j];
    double *x = b.X + b.off_n[j], *g = b.Gr + b.off_n[j];
    double *lam = b.Lam + b.off_m[j], *V = b.V + b.off_nm[j];
    double *d = b.D + b.off_obs[j];
    traj[j] = {h.mv, x, h.xs64, h.xs32};
    innov[j] = {h.mv, h.xs64, h.obs_step, h.obs_idx, h.u_optr, h.u_olist, h.y, h.rinv, d, h.fgrad};
    gp[j] = {h.mv, nullptr, h.LAM, nullptr, h.fgrad};
    hp[j] = {h.mv, h.LW, h.LAM, h.f, nullptr};
    aG[j] = {n, h.w, 1, h.taps, h.LAM, g, nullptr, 2};
    aI[j] = {n, h.w, m, h.taps, h.Om, h.LW, nullptr, 0};
    aO[j] = {n, h.w, m, h.taps, h.LAM, h.Y, nullptr, 0};
    aD[j] = {n, h.w, 1, h.taps, b.Dz + b.off_n[j], b.Dx + b.off_n[j], nullptr, 0};
    ph[j] = {(long long)n * m, (unsigned long long)j, h.Om};
    cY[j] = {(long long)n * m, h.Y, h.Q};
    cB[j] = {(long long)m * m, h.B2, h.Zs};
    int *cq1 = h.flags + 12, *cq2 = h.flags + 12;
    qY[j] = {cq1, h.flags + 5};
    qB[j] = {cq2, nullptr};
    gQ[j] = {m, m, n, h.Q, n, h.Q, n, h.G, m, cq1};
    gZ[j] = {m, m, m, h.Zs, m, h.Zs, m, h.G, m, cq2};
    g1[j] = {m, m, n, h.Q, n, h.Y, n, h.B1, m, nullptr};
    g2[j] = {m, m, n, h.Q, n, h.Om, n, h.B2, m, nullptr};
    gK[j] = {m, m, m, h.B1, m, h.Zs, m, h.K, m, nullptr};
    gV[j] = {n, m, m, h.Q, n, h.Zs, m, V, n, nullptr};
    gc[j] = {m, 1, n, V, n, g, n, h.cvec, m, nullptr};
    const double srelY = 11.0 * ((double)m * n + (double)m * (m + 1)) * u;
    const double srelZ = 11.0 * ((double)m * m + (double)m * (m + 1)) * u;
    hQ[j] = {m, h.G, h.R, srelY, h.flags + 0, h.flags + 4, cq1, cq1 + 2};
    hZ[j] = {m, h.G, h.R, srelZ, h.flags + 1, h.flags + 4, cq2, cq2 + 2};
    tQ[j] = {n, m, h.Q, n, h.R, cq1};
    tZ[j] = {m, m, h.Zs, m, h.R, cq2};
    t1[j] = {m, m, h.B1, m, h.R, cq2};
    sy[j] = {m, h.K};
    eg[j] = {m, h.K, lam, h.Zs, h.sywork, h.flags + 2};
    ic[j] = {n, m, lam, V, h.cvec, g, b.Dz + b.off_n[j], h.scal + 4};
  }
  riot_status rs = RIOT_OK;
  auto up = [&](auto *dst, const auto &src) {
    if (rs == RIOT_OK) rs = upload(dst, src, b.st);
  };
  up(b.traj, traj);
  up(b.innov, innov);
  up(b.grad_probs, gp);
  up(b.hvp_probs, hp);
  up(b.aL_grad, aG);
  up(b.aL_in, aI);
  up(b.aL_out, aO);
  up(b.aL_dx, aD);
  up(b.philox, ph);
  up(b.cp_Y, cY);
  up(b.cp_B2, cB);
  up(b.cq_Y, qY);
  up(b.cq_B2, qB);
  up(b.gram_Q, gQ);
  up(b.gram_Z, gZ);
  up(b.g_B1, g1);
  up(b.g_B2, g2);
  up(b.g_K, gK);
  up(b.g_V, gV);
  up(b.g_c, gc);
  up(b.ch_Q, hQ);
  up(b.ch_Z, hZ);
  up(b.tr_Q, tQ);
  up(b.tr_Z, tZ);
  up(b.tr_B1, t1);
  up(b.sym, sy);
  up(b.eig, eg);
  up(b.inc, ic);
  if (rs == RIOT_OK) rs = batch_build_tiles(b);
  if (hipStreamSynchronize(b.st) != hipSuccess) rs = RIOT_E_HIP;
  return rs;
}

#define RIOT_BHIP(call)                        \
  do {                                         \
    if ((call) != hipSuccess) return RIOT_E_HIP; \
  } while (0)

riot_status batch_hvp(riot_batch &b, int mode, long long *clk = nullptr) {
  const riot::TladTile *t = b.tiles;
  if (mode == 1)
    return riot::launch_tlad_persistent(b.nwg, 1, b.grad_probs, t, b.n_grad_wg, t + b.n_grad_wg,
                                        b.n_grad_wave, b.counters, b.fp32, b.st) == hipSuccess
               ? RIOT_OK
               : RIOT_E_HIP;
  const riot::TladTile *th = t + b.n_grad_wg + b.n_grad_wave;
  return riot::launch_tlad_persistent(b.nwg, mode, b.hvp_probs, th, b.n_hvp_wg, th + b.n_hvp_wg,
                                      b.n_hvp_wave, b.counters + 2, b.fp32, b.st, clk) == hipSuccess
             ? RIOT_OK
             : RIOT_E_HIP;
}

// Adaptive CholeskyQR of every problem's block (see cholqr): X_j <- orth(X_j), companion
// C_j receiving the same right factors.
riot_status batch_cholqr(riot_batch &b, const riot::CqJob *cq, const riot::GemmJob *gram,
                         const riot::CholJob *ch, const riot::TrsmJob *tr, const riot::TrsmJob *comp,
                         int maxrows, bool shifted) {
  hipStream_t st = b.st;
  RIOT_BHIP(riot::launch_cholqr_reset_batched(b.nprob, cq, st));
  for (int pass = 0; pass < 8; ++pass) {
    const bool sh = shifted && pass == 0;
    RIOT_BHIP(riot::launch_gemm_batched(1, 0, b.nprob, b.maxm, b.maxm, 1.0, 0.0, gram, st));
    RIOT_BHIP(riot::launch_chol_batched(b.nprob, sh ? 1 : 2, ch, st));
    RIOT_BHIP(riot::launch_trsm_batched(b.nprob, maxrows, tr, st));
    if (comp) RIOT_BHIP(riot::launch_trsm_batched(b.nprob, b.maxm, comp, st));
    RIOT_BHIP(riot::launch_cholqr_ctrl_batched(b.nprob, sh ? 1 : 0, cq, st));
  }
  return RIOT_OK;
}

riot_status batch_pipeline(riot_batch &b) {
  hipStream_t st = b.st;
  riot_status rs;
  // a1-a2: trajectories, innovations, gradients g = -L G^T R^{-1} d (first outer loop)
  RIOT_BHIP(riot::launch_trajectory_batched(b.nprob, b.traj, st));
  RIOT_BHIP(riot::launch_innovation_batched(b.nprob, b.maxU, b.innov, b.fp32, st));
  if ((rs = batch_hvp(b, 1)) != RIOT_OK) return rs;
  RIOT_BHIP(riot::launch_apply_L_batched(b.nprob, 1, b.maxext, b.aL_grad, st));
  // a3-a4: probes and Hessian-probe products
  RIOT_BHIP(riot::launch_philox_batched(b.nprob, (long long)b.maxn * b.maxm, b.seed, b.philox, st));
  RIOT_BHIP(riot::launch_apply_L_batched(b.nprob, b.maxm, b.maxext, b.aL_in, st));
  if ((rs = batch_hvp(b, 0)) != RIOT_OK) return rs;
  RIOT_BHIP(riot::launch_apply_L_batched(b.nprob, b.maxm, b.maxext, b.aL_out, st));
  // a6: Q = orth(Y)
  RIOT_BHIP(riot::launch_copy_batched(b.nprob, (long long)b.maxn * b.maxm, b.cp_Y, st));
  if ((rs = batch_cholqr(b, b.cq_Y, b.gram_Q, b.ch_Q, b.tr_Q, nullptr, b.maxn, true)) != RIOT_OK)
    return rs;
  // a7: projections and K
  RIOT_BHIP(riot::launch_gemm_batched(1, 0, b.nprob, b.maxm, b.maxm, 1.0, 0.0, b.g_B1, st));
  RIOT_BHIP(riot::launch_gemm_batched(1, 0, b.nprob, b.maxm, b.maxm, 1.0, 0.0, b.g_B2, st));
  RIOT_BHIP(riot::launch_copy_batched(b.nprob, (long long)b.maxm * b.maxm, b.cp_B2, st));
  if ((rs = batch_cholqr(b, b.cq_B2, b.gram_Z, b.ch_Z, b.tr_Z, b.tr_B1, b.maxm, false)) != RIOT_OK)
    return rs;
  RIOT_BHIP(riot::launch_gemm_batched(0, 1, b.nprob, b.maxm, b.maxm, 1.0, 0.0, b.g_K, st));
  RIOT_BHIP(riot::launch_symmetrize_batched(b.nprob, b.sym, st));
  // a8: eigen-solve and Ritz vectors
  RIOT_BHIP(riot::launch_eig_batched(b.nprob, b.maxm, b.eig, st));
  RIOT_BHIP(riot::launch_gemm_batched(0, 0, b.nprob, b.maxn, b.maxm, 1.0, 0.0, b.g_V, st));
  // a9: adaptive increment from all m Ritz pairs, dx = L dz
  RIOT_BHIP(riot::launch_gemm_batched(1, 0, b.nprob, b.maxm, 1, 1.0, 0.0, b.g_c, st));
  RIOT_BHIP(riot::launch_increment_batched(b.nprob, b.maxn, 2, b.inc, st));
  RIOT_BHIP(riot::launch_apply_L_batched(b.nprob, 1, b.maxext, b.aL_dx, st));
  return RIOT_OK;
}

}  // namespace

extern "C" {

size_t riot_batch_workspace_bytes(int32_t nprob, const riot_desc *descs) {
  if (nprob < 1 || !descs) return 0;
  size_t tot = 0, tn = 0, tm = 0, tnm = 0, tobs = 0, tiles = 0;
  for (int j = 0; j < nprob; ++j) {
    riot_desc d = descs[j];
    d.elems_per_lane = 8;
    if (!batch_desc_ok(d)) return 0;
    const size_t w = riot_workspace_bytes(&d);
    if (!w) return 0;
    tot += align256(w);
    tn += d.n;
    tm += d.m_max;
    tnm += (size_t)d.n * d.m_max;
    tobs += std::max(d.nobs, 1);
    tiles += 1 + d.m_max;
  }
  riot_batch b;
  b.nprob = nprob;
  b.tot_n = tn, b.tot_m = tm, b.tot_nm = tnm, b.tot_obs = tobs;
  return tot + batch_carve(b, nullptr, tiles) + 256;
}

riot_status riot_batch_init(int32_t nprob, const riot_desc *descs, void *workspace, size_t bytes,
                            void *hip_stream, riot_batch **out) {
  if (!out) return RIOT_E_ARG;
  *out = nullptr;
  if (nprob < 1 || !descs || !workspace) return RIOT_E_ARG;
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return RIOT_E_WORKSPACE;
  const size_t need = riot_batch_workspace_bytes(nprob, descs);
  if (!need) return RIOT_E_ARG;
  if (bytes < need) return RIOT_E_WORKSPACE;
  riot_batch *b = new (std::nothrow) riot_batch();
  if (!b) return RIOT_E_ARG;
  b->nprob = nprob;
  b->st = static_cast<hipStream_t>(hip_stream);
  b->fp32 = descs[0].prec == RIOT_FP32_TLAD;
  char *base = static_cast<char *>(workspace);
  size_t off = 0;
  riot_status rs = RIOT_OK;
  for (int j = 0; j < nprob && rs == RIOT_OK; ++j) {
    riot_desc d = descs[j];
    d.elems_per_lane = 8;
    if ((d.prec == RIOT_FP32_TLAD) != b->fp32) {
      rs = RIOT_E_ARG;
      break;
    }
    riot_handle *h = new (std::nothrow) riot_handle();
    if (!h) {
      rs = RIOT_E_ARG;
      break;
    }
    b->hs.push_back(h);
    const size_t w = riot_workspace_bytes(&d);
    rs = init_handle(h, &d, base + off, w, b->st);
    off += align256(w);
    b->n.push_back(d.n);
    b->m.push_back(d.m_max);
    b->T.push_back(d.nsteps);
    b->nobs.push_back(d.nobs);
    b->off_n.push_back(b->tot_n);
    b->off_m.push_back(b->tot_m);
    b->off_nm.push_back(b->tot_nm);
    b->off_obs.push_back(b->tot_obs);
    b->tot_n += d.n;
    b->tot_m += d.m_max;
    b->tot_nm += (size_t)d.n * d.m_max;
    b->tot_obs += std::max(d.nobs, 1);
    b->maxn = std::max(b->maxn, d.n);
    b->maxm = std::max(b->maxm, d.m_max);
    b->maxU = std::max(b->maxU, h->U);
    b->maxext = std::max(b->maxext, d.n + 2 * h->w);
    b->cus = h->cus;
  }
  if (rs == RIOT_OK) {
    for (int j = 0; j < nprob; ++j) b->tile_cap += 1 + b->m[j];
    batch_carve(*b, base + off, b->tile_cap);
    b->nwg = 2 * b->cus;
    rs = batch_tables(*b);
  }
  if (rs != RIOT_OK) {
    delete b;
    return rs;
  }
  *out = b;
  return RIOT_OK;
}

void riot_batch_free(riot_batch *b) { delete b; }

riot_status riot_batch_buffers(riot_batch *b, riot_batch_io *io) {
  if (!b || !io) return RIOT_E_ARG;
  io->x = b->X;
  io->grad = b->Gr;
  io->lambda = b->Lam;
  io->V = b->V;
  io->dz = b->Dz;
  io->dx = b->Dx;
  io->d = b->D;
  return RIOT_OK;
}

riot_status riot_batch_run(riot_batch *b, uint64_t seed) {
  if (!b) return RIOT_E_ARG;
  if (b->graph) return RIOT_E_STATE;
  b->seed = seed;
  const riot_status rs = batch_pipeline(*b);
  if (rs == RIOT_OK)
    for (auto *h : b->hs) h->linearized = true;  // trajectories are stored for every problem
  return rs;
}

riot_status riot_batch_set_layout(riot_batch *b, int32_t workgroups, int32_t wave_max_threads) {
  if (!b || workgroups < 1 || wave_max_threads < 0 || wave_max_threads > 64) return RIOT_E_ARG;
  if (b->graph) return RIOT_E_STATE;
  b->nwg = workgroups;
  b->wave_max_nt = wave_max_threads;
  const riot_status rs = batch_build_tiles(*b);
  if (rs != RIOT_OK) return rs;
  return hipStreamSynchronize(b->st) == hipSuccess ? RIOT_OK : RIOT_E_HIP;
}

riot_status riot_batch_autotune(riot_batch *b, int32_t *workgroups_out,
                                int32_t *wave_max_threads_out, float *ms_out) {
  if (!b) return RIOT_E_ARG;
  if (b->graph) return RIOT_E_STATE;
  // inputs of the timed launches: the current trajectories and deterministic probes
  b->seed = 0x5eedULL;
  RIOT_BHIP(riot::launch_trajectory_batched(b->nprob, b->traj, b->st));
  RIOT_BHIP(riot::launch_philox_batched(b->nprob, (long long)b->maxn * b->maxm, b->seed, b->philox,
                                        b->st));
  RIOT_BHIP(riot::launch_apply_L_batched(b->nprob, b->maxm, b->maxext, b->aL_in, b->st));
  hipEvent_t e0, e1;
  RIOT_BHIP(hipEventCreate(&e0));
  RIOT_BHIP(hipEventCreate(&e1));
  const int cand_wg[3] = {b->cus, 2 * b->cus, 3 * b->cus};
  const int cand_wave[2] = {0, 64};
  float best = 1e30f;
  int best_wg = b->nwg, best_wave = b->wave_max_nt;
  riot_status rs = RIOT_OK;
  for (int wv : cand_wave) {
    for (int wg : cand_wg) {
      b->nwg = wg;
      b->wave_max_nt = wv;
      if ((rs = batch_build_tiles(*b)) != RIOT_OK) break;
      float ms = 1e30f;
      for (int rep = 0; rep < 3 && rs == RIOT_OK; ++rep) {
        if (hipEventRecord(e0, b->st) != hipSuccess) rs = RIOT_E_HIP;
        if (rs == RIOT_OK) rs = batch_hvp(*b, 0);
        if (rs == RIOT_OK && hipEventRecord(e1, b->st) != hipSuccess) rs = RIOT_E_HIP;
        if (rs == RIOT_OK && hipEventSynchronize(e1) != hipSuccess) rs = RIOT_E_HIP;
        float t = 0.f;
        if (rs == RIOT_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rs = RIOT_E_HIP;
        if (rep > 0) ms = std::min(ms, t);  // the first run is a warm-up
      }
      if (rs != RIOT_OK) break;
      if (ms < best) best = ms, best_wg = wg, best_wave = wv;
    }
    if (rs != RIOT_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rs != RIOT_OK) return rs;
  b->nwg = best_wg;
  b->wave_max_nt = best_wave;
  if ((rs = batch_build_tiles(*b)) != RIOT_OK) return rs;
  if (hipStreamSynchronize(b->st) != hipSuccess) return RIOT_E_HIP;
  if (workgroups_out) *workgroups_out = best_wg;
  if (wave_max_threads_out) *wave_max_threads_out = best_wave;
  if (ms_out) *ms_out = best;
  return RIOT_OK;
}

riot_status riot_batch_capture(riot_batch *b, uint64_t seed) {
  if (!b) return RIOT_E_ARG;
  if (b->graph) {
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
  }
  if (b->st == nullptr) return RIOT_E_STATE;  // the legacy default stream cannot be captured
  b->seed = seed;
  RIOT_BHIP(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
  const riot_status rs = batch_pipeline(*b);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(b->st, &g);
  if (rs != RIOT_OK || ec != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return rs != RIOT_OK ? rs : RIOT_E_HIP;
  }
  for (auto *h : b->hs) h->linearized = true;
  hipGraphExec_t ex = nullptr;
  const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) return RIOT_E_HIP;
  b->graph = ex;
  return RIOT_OK;
}

riot_status riot_batch_replay(riot_batch *b) {
  if (!b || !b->graph) return RIOT_E_STATE;
  return hipGraphLaunch(b->graph, b->st) == hipSuccess ? RIOT_OK : RIOT_E_HIP;
}

riot_status riot_batch_profile(riot_batch *b, float *ms, double *busy_frac, int32_t *tiles) {
  if (!b) return RIOT_E_ARG;
  if (b->graph) return RIOT_E_STATE;
  const int nt = b->n_hvp_wg + b->n_hvp_wave;
  if (nt == 0) return RIOT_E_STATE;
  long long *clk = b->clk;  // carved from the batch's workspace (2 clocks per tile)
  hipEvent_t e0, e1;
  riot_status rs = RIOT_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rs = RIOT_E_HIP;
  if (rs == RIOT_OK && hipEventRecord(e0, b->st) != hipSuccess) rs = RIOT_E_HIP;
  if (rs == RIOT_OK) rs = batch_hvp(*b, 0, clk);
  if (rs == RIOT_OK && hipEventRecord(e1, b->st) != hipSuccess) rs = RIOT_E_HIP;
  std::vector<long long> t(2 * (size_t)nt);
  if (rs == RIOT_OK && hipMemcpyAsync(t.data(), clk, t.size() * sizeof(long long),
                                      hipMemcpyDeviceToHost, b->st) != hipSuccess)
    rs = RIOT_E_HIP;
  if (rs == RIOT_OK && hipStreamSynchronize(b->st) != hipSuccess) rs = RIOT_E_HIP;
  float el = 0.f;
  if (rs == RIOT_OK && hipEventElapsedTime(&el, e0, e1) != hipSuccess) rs = RIOT_E_HIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rs != RIOT_OK) return rs;
  // busy time of every slot (a workgroup tile occupies four waves, a wave tile one) over
  // the slots available (four waves per workgroup that can be resident) times the makespan
  long long lo = t[0], hi = t[1];
  double busy = 0.0;
  for (int i = 0; i < nt; ++i) {
    lo = std::min(lo, t[2 * i]);
    hi = std::max(hi, t[2 * i + 1]);
    busy += (double)(t[2 * i + 1] - t[2 * i]) * (i < b->n_hvp_wg ? 4.0 : 1.0);
  }
  // workgroups resident at once: the launch's, capped by what the compute units hold
  const int per_cu = riot::tlad_persistent_resident_per_cu(b->fp32);
  const double slots = 4.0 * std::min(b->nwg, per_cu > 0 ? per_cu * b->cus : b->nwg);
  if (ms) *ms = el;
  if (busy_frac) *busy_frac = hi > lo ? busy / (slots * (double)(hi - lo)) : 0.0;
  if (tiles) *tiles = nt;
  return RIOT_OK;
}

riot_status riot_exp_corr_sqrt(int32_t n, double ell, double *L1) {
  if (n < 1 || !(ell > 0.0) || !L1) return RIOT_E_ARG;
  // C1[i,j] = exp(-d/ell) with periodic d is a symmetric circulant: its eigenvalues are
  // the cosine transform of its first row, its eigenvectors the Fourier modes, so
  // L1[i,j] = (1/n) sum_k sqrt(max(l_k, 0)) cos(2 pi k (i - j) / n).
  const double tw = 2.0 * 3.14159265358979323846 / n;
  std::vector<double> row(n), lam(n), col(n);
  for (int d = 0; d < n; ++d) row[d] = std::exp(-std::min(d, n - d) / ell);
  for (int k = 0; k < n; ++k) {
    double s = 0.0;
    for (int d = 0; d < n; ++d) s += row[d] * std::cos(tw * ((long long)k * d % n));
    lam[k] = std::sqrt(std::max(s, 0.0));
  }
  for (int d = 0; d < n; ++d) {
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += lam[k] * std::cos(tw * ((long long)k * d % n));
    col[d] = s / n;
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) L1[(size_t)i * n + j] = col[(i - j + n) % n];
  return RIOT_OK;
}

int32_t riot_gaussian_taps(double ell, double sigma_b, int32_t max_taps, double *taps) {
  if (!(ell > 0.0) || !(sigma_b > 0.0) || !std::isfinite(ell) || !std::isfinite(sigma_b))
    return -1;
  const int w = (int)std::ceil(6.25 * ell);
  if (!taps) return w;
  if (max_taps < w + 1) return -1;
  double s2 = 0.0;
  for (int d = -w; d <= w; ++d) {
    const double k = std::exp(-(double)d * d / (ell * ell));
    s2 += k * k;
  }
  const double c = sigma_b / std::sqrt(s2);
  for (int d = 0; d <= w; ++d) taps[d] = c * std::exp(-(double)d * d / (ell * ell));
  return w;
}

riot_status riot_batch_problem(riot_batch *b, int32_t j, riot_handle **h) {
  if (!b || !h || j < 0 || j >= b->nprob) return RIOT_E_ARG;
  *h = b->hs[j];
  return RIOT_OK;
}


// ---------------------------------------------------------------------------
// Standalone sketch handle: Alg. 3's steps after the Hessian-probe products, for any
// operator whose products the caller computes (another model, a learned probe basis).
// ---------------------------------------------------------------------------

}  // extern "C"

struct riot_sketch {
  LaSpace la{};
  int n = 0, m_max = 0;
};

namespace {

size_t sketch_carve(riot_sketch &s, void *base) {
  Carver c(base);
  const size_t n = s.n, m = s.m_max, m2 = m * m;
  LaSpace &la = s.la;
  la.Q = c.take<double>(n * m);
  la.G = c.take<double>(m2);
  la.R = c.take<double>(m2);
  la.B1 = c.take<double>(m2);
  la.B2 = c.take<double>(m2);
  la.K = c.take<double>(m2);
  la.Zs = c.take<double>(m2);
  la.sywork = c.take<double>(eig_work_doubles((int)m));
  la.partial = c.take<double>(partial_doubles(m));
  la.cvec = c.take<double>(m);
  la.scal = c.take<double>(16);
  la.flags = c.take<int>(32);  // 16 flags, then the CholeskyQR pass control
  la.cq = la.flags + 16;
  return c.off + 256;
}

}  // namespace

extern "C" {

size_t riot_sketch_workspace_bytes(int32_t n, int32_t m_max) {
  if (n < 1 || m_max < 1 || m_max > 1088 || m_max > n) return 0;
  riot_sketch s;
  s.n = n, s.m_max = m_max;
  return sketch_carve(s, nullptr);
}

riot_status riot_sketch_init(int32_t n, int32_t m_max, void *workspace, size_t bytes,
                             void *hip_stream, riot_sketch **out) {
  if (!out) return RIOT_E_ARG;
  *out = nullptr;
  const size_t need = riot_sketch_workspace_bytes(n, m_max);
  if (!need || !workspace) return RIOT_E_ARG;
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return RIOT_E_WORKSPACE;
  if (bytes < need) return RIOT_E_WORKSPACE;
  riot_sketch *s = new (std::nothrow) riot_sketch();
  if (!s) return RIOT_E_ARG;
  s->n = n, s->m_max = m_max;
  sketch_carve(*s, workspace);
  s->la.st = static_cast<hipStream_t>(hip_stream);
  *out = s;
  return RIOT_OK;
}

void riot_sketch_free(riot_sketch *s) { delete s; }

riot_status riot_sketch_eig(riot_sketch *s, int32_t m, const double *Omega, const double *Y,
                            double *lambda, double *V, riot_rsvd_info *info) {
  if (!s || !Omega || !Y || !lambda || !V || m < 1 || m > s->m_max) return RIOT_E_ARG;
  RIOT_HIP(launch_zero_ints(s->la.flags, 16, s->la.st));
  return sketch_eig(s->la, s->n, m, Y, Omega, lambda, V, info);
}

riot_status riot_sketch_residual(riot_sketch *s, int32_t m, const double *Q, const double *AQ,
                                 double *rho_host) {
  if (!s || !Q || !AQ || !rho_host || m < 1 || m > s->m_max) return RIOT_E_ARG;
  if (Q == s->la.Q || AQ == s->la.Q) return RIOT_E_ARG;
  return proj_residual(s->la, s->n, m, Q, AQ, rho_host);
}

riot_status riot_sketch_increment(riot_sketch *s, int32_t k, const double *lambda,
                                  const double *V, const double *grad, riot_update mode,
                                  double *dz, double *dofs_host, int32_t *mode_used) {
  if (!s || !lambda || !V || !grad || !dz || k < 1 || k > s->m_max) return RIOT_E_ARG;
  if (mode != RIOT_ADAPTIVE && mode != RIOT_LRA && mode != RIOT_LRU) return RIOT_E_ARG;
  return sketch_increment(s->la, s->n, k, lambda, V, grad, mode, dz, dofs_host, mode_used);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// riot_sketch_eig without a workspace argument, for callers that cannot allocate device
// memory: the sketch's scratch regions are carved from one static device array instead.
// Every call on a device shares that device's copy of the array, so calls that overlap on
// one device race; the flags the eigen-solve reads are cleared by a kernel on every call.
// ---------------------------------------------------------------------------

constexpr size_t kNoallocScratchBytes = (size_t)32 << 20;  // 32 MiB per device
static __device__ __align__(256) char scratch[kNoallocScratchBytes];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxScratchDevices];  // device address of `scratch` per device

// Device address of `scratch` on the current device, looked up once per device (the
// array's name in host code is only a host-side handle, never a device address).
riot_status scratch_address(void **out) {
  int dev = -1;
  RIOT_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices) return RIOT_E_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    RIOT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return RIOT_E_HIP;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return RIOT_OK;
}

}  // namespace

extern "C" {

size_t riot_sketch_noalloc_max_bytes(void) { return kNoallocScratchBytes; }

riot_status riot_sketch_eig_noalloc(int32_t n, int32_t m, const double *Omega, const double *Y,
                                    double *lambda, double *V, void *hip_stream,
                                    riot_rsvd_info *info) {
  if (!Omega || !Y || !lambda || !V || n < 1 || m < 1 || m > n || m > 1088) return RIOT_E_ARG;
  riot_sketch s;
  s.n = n, s.m_max = m;
  if (sketch_carve(s, nullptr) > kNoallocScratchBytes) return RIOT_E_SCRATCH;
  void *base = nullptr;
  const riot_status rs = scratch_address(&base);
  if (rs != RIOT_OK) return rs;
  sketch_carve(s, base);
  s.la.st = static_cast<hipStream_t>(hip_stream);
  RIOT_HIP(launch_zero_ints(s.la.flags, 16, s.la.st));
  return sketch_eig(s.la, n, m, Y, Omega, lambda, V, info);
}

}  // extern "C"
