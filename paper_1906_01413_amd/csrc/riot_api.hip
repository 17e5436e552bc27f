// C ABI of the RIOT inner loop: handle, workspace carve-up, call sequencing.
//
// The calls follow Alg. 3 (precond = false) of arXiv 1906.01413: linearise
// (trajectory, innovation, gradient), Hessian-probe products of the whole probe
// block, orthonormal basis, K from K (Q^T Omega) = Q^T Y, eigendecomposition,
// adaptive increment (eqs. 8-11) and low-rank posterior covariance.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "riot_internal.h"

using namespace riot;

namespace {

constexpr int kSplitK = 16;

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
  double *Om = nullptr, *Y = nullptr, *Q = nullptr, *Q0 = nullptr, *Qt = nullptr;
  double *G = nullptr, *R = nullptr, *Rinv = nullptr, *B1 = nullptr, *B2 = nullptr,
         *B2i = nullptr, *K = nullptr, *Zs = nullptr, *gjw = nullptr, *sywork = nullptr;
  double *partial = nullptr, *cvec = nullptr, *scal = nullptr, *cgv = nullptr;
  int *flags = nullptr;
  ModelView mv{};
};

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
  const size_t blk = (size_t)(T + 1) * 4 * stage_block_elems(h.E, h.NT);
  h.xs64 = c.take<double>(blk);
  h.xs32 = h.fp32 ? c.take<float>(blk) : nullptr;
  h.fgrad = c.take<char>(U1 * Rs);
  h.f = c.take<char>((size_t)(mm + 1) * U1 * Rs);
  const size_t nm = (size_t)n * mm;
  h.LW = c.take<double>(nm);
  h.LAM = c.take<double>(nm);
  h.Om = c.take<double>(nm);
  h.Y = c.take<double>(nm);
  h.Q = c.take<double>(nm);
  h.Q0 = c.take<double>(nm);
  h.Qt = c.take<double>(nm);
  const size_t m2 = (size_t)mm * mm;
  h.G = c.take<double>(m2);
  h.R = c.take<double>(m2);
  h.Rinv = c.take<double>(m2);
  h.B1 = c.take<double>(m2);
  h.B2 = c.take<double>(m2);
  h.B2i = c.take<double>(m2);
  h.K = c.take<double>(m2);
  h.Zs = c.take<double>(m2);
  h.gjw = c.take<double>(2 * m2);
  h.sywork = c.take<double>(eig_work_doubles(mm));
  h.partial = c.take<double>(std::max((size_t)kSplitK * m2, (size_t)kSplitK * mm));
  h.cvec = c.take<double>(mm);
  h.scal = c.take<double>(16);
  h.cgv = c.take<double>((size_t)5 * n);
  h.flags = c.take<int>(16);
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
// orthonormal to rounding, at most kMaxCholQRPasses: a sketch whose singular values span
// more than the FP64 range of one shifted pass (graded spectra, numerically rank-deficient
// blocks) gets further passes instead of a non-orthonormal Q. Passes beyond the last
// needed one are launched but return at once (device flag), so nothing synchronises.
constexpr int kMaxCholQRPasses = 8;

riot_status cholqr(riot_handle *h, int rows, int m, const double *Xin, double *Qout, bool shifted,
                   int flag_idx, double *comp = nullptr, int mc = 0, int *count = nullptr) {
  hipStream_t st = h->st;
  const double u = 0x1.0p-53;
  const double srel = 11.0 * ((double)m * rows + (double)m * (m + 1)) * u;
  int *cq = h->flags + 12;
  if (Qout != Xin)
    RIOT_HIP(hipMemcpyAsync(Qout, Xin, (size_t)rows * m * sizeof(double), hipMemcpyDeviceToDevice,
                            st));
  RIOT_HIP(launch_cholqr_reset(cq, st));
  for (int pass = 0; pass < kMaxCholQRPasses; ++pass) {
    const bool sh = shifted && pass == 0;
    RIOT_HIP(gemm_f64(1, 0, m, m, rows, 1.0, Qout, rows, Qout, rows, 0.0, h->G, m, h->partial,
                      kSplitK, st, cq));
    RIOT_HIP(launch_chol_blocked(m, h->G, h->R, srel, sh ? 1 : 2, h->flags + flag_idx,
                                 h->flags + 4, st, cq, cq + 2));
    RIOT_HIP(launch_trsm_rlt(rows, m, Qout, rows, h->R, st, cq));
    if (comp) RIOT_HIP(launch_trsm_rlt(mc, m, comp, mc, h->R, st, cq));
    RIOT_HIP(launch_cholqr_ctrl(cq, sh ? 1 : 0, count, st));
  }
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

riot_status riot_init(const riot_desc *desc, void *workspace, size_t bytes, void *hip_stream,
                      riot_handle **out) {
  if (!out) return RIOT_E_ARG;
  *out = nullptr;
  if (!desc_valid(desc) || !workspace) return RIOT_E_ARG;
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return RIOT_E_WORKSPACE;
  riot_handle *h = new (std::nothrow) riot_handle();
  if (!h) return RIOT_E_ARG;
  ObsPlan plan;
  if (!prepare(*h, desc, &plan)) {
    delete h;
    return RIOT_E_ARG;
  }
  const size_t need = carve(*h, nullptr);
  if (bytes < need) {
    delete h;
    return RIOT_E_WORKSPACE;
  }
  carve(*h, workspace);
  h->st = static_cast<hipStream_t>(hip_stream);
  fill_view(*h);
  const riot_desc &d = h->d;
  const int n = d.n, w = h->w;
  // host-side tables
  std::vector<double> lrow(n, 0.0), brow(n, 0.0);
  for (int dd = -w; dd <= w; ++dd) {
    int j = dd % n;
    if (j < 0) j += n;
    lrow[j] += d.l_taps[std::abs(dd)];
  }
  for (int dd = 0; dd < n; ++dd) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += lrow[j] * lrow[(j + dd) % n];
    brow[dd] = s;
  }
  h->base_diag = brow[0];
  std::vector<float> wgt32(plan.wgt.begin(), plan.wgt.end());
  hipStream_t st = h->st;
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
  if (rs != RIOT_OK) {
    delete h;
    return rs;
  }
  *out = h;
  return RIOT_OK;
}

void riot_free(riot_handle *h) { delete h; }

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
  }
  return "unknown riot_status";
}

riot_status riot_linearize(riot_handle *h, const double *x, const double *v, double *d,
                           double *grad, double *J_host) {
  if (!h || !x || !grad || (h->d.nobs > 0 && !d)) return RIOT_E_ARG;
  const riot_desc &ds = h->d;
  hipStream_t st = h->st;
  RIOT_HIP(launch_trajectory(h->mv, ds.nsteps, x, nullptr, h->xs64, h->xs32, st));
  if (ds.nobs > 0)
    RIOT_HIP(launch_innovation(h->mv, h->xs64, ds.nobs, h->obs_step, h->obs_idx, h->y, h->rinv,
                               h->u_optr, h->u_olist, d, h->fgrad, h->fp32, st));
  // gradient: g = v - L lambda_0 with lambda_0 the adjoint sweep forced by R^{-1} d
  RIOT_HIP(launch_tlad(h->mv, 1, 1, nullptr, h->LAM, nullptr, h->fgrad, h->fp32, st));
  RIOT_HIP(launch_apply_L(ds.n, h->w, h->taps, 1, h->LAM, grad, v, 2, st));
  h->linearized = true;
  if (J_host) {
    RIOT_HIP(launch_cost(ds.n, v, ds.nobs, d, h->rinv, h->scal, st));
    RIOT_HIP(hipMemcpyAsync(J_host, h->scal, sizeof(double), hipMemcpyDeviceToHost, st));
    RIOT_HIP(hipStreamSynchronize(st));
  }
  return RIOT_OK;
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
    rs = cholqr(h, n, m, h->Y, h->Q0, true, 0);
    if (rs != RIOT_OK) return rs;
    rs = hess_apply_impl(h, m, h->Q0, h->Y, 0);
    if (rs != RIOT_OK) return rs;
    Om_eff = h->Q0;
  }
  rs = cholqr(h, n, m, h->Y, h->Q, true, 0, nullptr, 0, h->flags + 5);
  if (rs != RIOT_OK) return rs;
  // B1 = Q^T Y, B2 = Q^T Omega_eff. K solves K B2 = B1: with B2 M = Q2 orthogonal (CholeskyQR
  // of the square B2 carrying B1 as companion, B1 M -> B1'), B2^{-1} = M Q2^T and K = B1' Q2^T.
  RIOT_HIP(gemm_f64(1, 0, m, m, n, 1.0, h->Q, n, h->Y, n, 0.0, h->B1, m, h->partial, kSplitK, st));
  RIOT_HIP(gemm_f64(1, 0, m, m, n, 1.0, h->Q, n, Om_eff, n, 0.0, h->B2, m, h->partial, kSplitK, st));
  rs = cholqr(h, m, m, h->B2, h->Zs, false, 1, h->B1, m);
  if (rs != RIOT_OK) return rs;
  RIOT_HIP(gemm_f64(0, 1, m, m, m, 1.0, h->B1, m, h->Zs, m, 0.0, h->K, m, nullptr, 1, st));
  RIOT_HIP(launch_symmetrize(m, h->K, h->scal + 1, h->partial, st));
  RIOT_HIP(launch_eig(m, h->K, lambda, h->Zs, h->sywork, h->flags + 2, st));
  RIOT_HIP(gemm_f64(0, 0, n, m, m, 1.0, h->Q, n, h->Zs, m, 0.0, V, n, nullptr, 1, st));
  RIOT_HIP(launch_check_finite(m, lambda, h->flags + 3, st));
  RIOT_HIP(launch_check_finite((long long)n * m, V, h->flags + 3, st));
  if (info) {
    RIOT_HIP(gemm_f64(1, 0, m, m, n, 1.0, h->Q, n, h->Q, n, 0.0, h->G, m, h->partial, kSplitK, st));
    RIOT_HIP(launch_orth_err(m, h->G, h->scal + 2, st));
    int fl[6];
    double sc[3];
    RIOT_HIP(hipMemcpyAsync(fl, h->flags, 6 * sizeof(int), hipMemcpyDeviceToHost, st));
    RIOT_HIP(hipMemcpyAsync(sc, h->scal, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    RIOT_HIP(hipStreamSynchronize(st));
    info->chol_shifts = fl[4];
    info->qr_passes = fl[5];
    info->k_asym = sc[1];
    info->orth_err = sc[2];
    if (fl[0]) return RIOT_E_NOT_SPD;
    if (fl[1]) return RIOT_E_SINGULAR;
    if (fl[2]) return RIOT_E_NOCONV;
    if (fl[3]) return RIOT_E_NONFINITE;
  }
  return RIOT_OK;
}

riot_status riot_increment(riot_handle *h, int32_t k, const double *lambda, const double *V,
                           const double *grad, riot_update mode, double *dz, double *dx,
                           double *dofs_host, int32_t *mode_used) {
  if (!h || !lambda || !V || !grad || !dz || !dx || k < 1 || k > h->d.n || k > h->d.m_max)
    return RIOT_E_ARG;
  if (mode != RIOT_ADAPTIVE && mode != RIOT_LRA && mode != RIOT_LRU) return RIOT_E_ARG;
  const int n = h->d.n;
  hipStream_t st = h->st;
  RIOT_HIP(gemm_f64(1, 0, k, 1, n, 1.0, V, n, grad, n, 0.0, h->cvec, k, h->partial, kSplitK, st));
  const int ml = mode == RIOT_LRA ? 0 : (mode == RIOT_LRU ? 1 : 2);
  RIOT_HIP(launch_increment_combine(n, k, lambda, V, h->cvec, grad, ml, dz, h->scal + 4, st));
  RIOT_HIP(launch_apply_L(n, h->w, h->taps, 1, dz, dx, nullptr, 0, st));
  if (mode_used) RIOT_HIP(launch_choose_mode(k, lambda, h->flags + 8, st));
  if (dofs_host || mode_used) {
    int mu = 0;
    if (dofs_host)
      RIOT_HIP(hipMemcpyAsync(dofs_host, h->scal + 4, sizeof(double), hipMemcpyDeviceToHost, st));
    if (mode_used)
      RIOT_HIP(hipMemcpyAsync(&mu, h->flags + 8, sizeof(int), hipMemcpyDeviceToHost, st));
    RIOT_HIP(hipStreamSynchronize(st));
    if (mode_used) *mode_used = (mode == RIOT_ADAPTIVE) ? mu : (int32_t)mode;
  }
  return RIOT_OK;
}

riot_status riot_posterior_cov(riot_handle *h, int32_t k, const double *lambda, const double *V,
                               riot_update mode, double *W, double *coef, double *diag,
                               double *dense, int32_t *mode_used) {
  if (!h || !lambda || !V || !W || !coef || k < 1 || k > h->d.n) return RIOT_E_ARG;
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
  if (!h->linearized) return RIOT_E_STATE;
  hipStream_t st = h->st;
  RIOT_HIP(launch_tlad(h->mv, m, 2, X, nullptr, h->f, nullptr, h->fp32, st));
  RIOT_HIP(launch_obs_gather(h->d.nobs, h->U, m, h->u_of_o, h->f, Z, h->fp32, st));
  return RIOT_OK;
}

riot_status riot_ad_apply(riot_handle *h, int32_t m, const double *Fo, double *X) {
  if (!h || !X || (!Fo && h->d.nobs > 0) || m < 1 || m > h->d.m_max) return RIOT_E_ARG;
  if (!h->linearized) return RIOT_E_STATE;
  hipStream_t st = h->st;
  RIOT_HIP(launch_obs_scatter(h->d.nobs, h->U, m, h->u_optr, h->u_olist, Fo, h->f, h->fp32, st));
  RIOT_HIP(launch_tlad(h->mv, m, 3, nullptr, X, h->f, nullptr, h->fp32, st));
  return RIOT_OK;
}

riot_status riot_gn_apply(riot_handle *h, int32_t m, const double *X, double *Y) {
  if (!h || !X || !Y || X == Y || m < 1 || m > h->d.m_max) return RIOT_E_ARG;
  if (!h->linearized) return RIOT_E_STATE;
  RIOT_HIP(launch_tlad(h->mv, m, 0, X, Y, h->f, nullptr, h->fp32, h->st));
  return RIOT_OK;
}

riot_status riot_forecast(riot_handle *h, const double *x0, int32_t nsteps, double *xout) {
  if (!h || !x0 || !xout || nsteps < 0) return RIOT_E_ARG;
  RIOT_HIP(launch_trajectory(h->mv, nsteps, x0, xout, nullptr, nullptr, h->st));
  return RIOT_OK;
}

riot_status riot_apply_L(riot_handle *h, int32_t m, const double *X, double *Y) {
  if (!h || !X || !Y || m < 1 || X == Y) return RIOT_E_ARG;
  RIOT_HIP(launch_apply_L(h->d.n, h->w, h->taps, m, X, Y, nullptr, 0, h->st));
  return RIOT_OK;
}

riot_status riot_philox_normal(riot_handle *h, int32_t n, int32_t m, uint64_t seed,
                               uint64_t stream, double *out) {
  if (!h || !out || n < 1 || m < 1) return RIOT_E_ARG;
  RIOT_HIP(launch_philox_normal((long long)n * m, seed, stream, out, h->st));
  return RIOT_OK;
}

}  // extern "C"
