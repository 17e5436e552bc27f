// Learned sketch proposal: a 1-D periodic convolutional network (FP32) that maps a
// background state to k probe vectors, its backward pass, Adam, and the subspace-capture
// loss of the leading Hessian eigenvectors with its gradient (FP64 on the MFMA GEMMs).
//
// Network: input = the standardized state (one channel); L layers of periodic conv1d of
// odd width 2r+1, ReLU after all but the last; output channel c is probe vector c.
// Layout: activations [sample][channel][grid point]; parameters flat, per layer the
// weights [cout][cin][width] then the biases [cout].

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "riot_internal.h"

namespace riot {
namespace {

constexpr int kCX = 64;   // grid points per tile
constexpr int kCC = 16;   // output channels per tile
constexpr int kMaxWidth = 11;  // keeps a tile's LDS within 64 KiB at 64 channels

// Per-row standardization (x - mean) / std of FP64 input rows (one workgroup per sample and
// input channel) into FP32.
__global__ void __launch_bounds__(256)
    standardize_kernel(int n, const double *__restrict__ x, float *__restrict__ out) {
  __shared__ double red[256];
  const double *xs = x + (size_t)blockIdx.x * n;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += xs[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  const double mean = red[0] / n;
  __syncthreads();
  double q = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) q += (xs[i] - mean) * (xs[i] - mean);
  red[threadIdx.x] = q;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  const double inv = 1.0 / sqrt(red[0] / n);
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    out[(size_t)blockIdx.x * n + i] = (float)((xs[i] - mean) * inv);
}

// z[c, i] = b[c] + sum_{c', j} W[c, c', j] h[c', (i + j - r) mod n], ReLU when relu != 0.
// Tile: kCX grid points x kCC output channels; the input rows (all cin, with the halo)
// and the tile's weights are staged in LDS; each thread computes four grid points.
__global__ void __launch_bounds__(256)
    conv_fwd_kernel(int n, int cin, int cout, int width, const float *__restrict__ h,
                    const float *__restrict__ W, const float *__restrict__ b,
                    float *__restrict__ z, int relu) {
  extern __shared__ float sh[];
  const int r = width / 2, span = kCX + width - 1;
  float *Xs = sh;                       // [cin][span]
  float *Ws = sh + (size_t)cin * span;  // [kCC][cin][width]
  const int x0 = blockIdx.x * kCX, c0 = blockIdx.y * kCC, s = blockIdx.z;
  const float *hs = h + (size_t)s * cin * n;
  for (int k = threadIdx.x; k < cin * span; k += blockDim.x) {
    const int ci = k / span, xx = k - ci * span;
    int g = x0 + xx - r;
    g = g < 0 ? g + n : (g >= n ? g - n : g);
    Xs[k] = hs[(size_t)ci * n + g];
  }
  const int wsz = cin * width;
  for (int k = threadIdx.x; k < kCC * wsz; k += blockDim.x) {
    const int cl = k / wsz;
    Ws[k] = (c0 + cl < cout) ? W[(size_t)(c0 + cl) * wsz + (k - cl * wsz)] : 0.f;
  }
  __syncthreads();
  const int cl = threadIdx.x / 16, xq = threadIdx.x % 16;
  const int c = c0 + cl;
  if (c >= cout) return;
  const float bias = b ? b[c] : 0.f;
  float acc[4] = {bias, bias, bias, bias};
  const float *wr = Ws + (size_t)cl * wsz;
  for (int ci = 0; ci < cin; ++ci) {
    const float *xr = Xs + (size_t)ci * span + xq * 4;
    for (int j = 0; j < width; ++j) {
      const float w = wr[ci * width + j];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = fmaf(w, xr[q + j], acc[q]);
    }
  }
  float *zo = z + ((size_t)s * cout + c) * n + x0 + xq * 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) zo[q] = relu ? fmaxf(acc[q], 0.f) : acc[q];
}

// Localized output head: N[s][c S + q][i] = z[s][c][i] for grid points i of segment q
// (n / S consecutive points), 0 elsewhere; z has k / S channels.
__global__ void segment_out_kernel(int n, int kch, int S, long long total,
                                   const float *__restrict__ z, float *__restrict__ N) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int k = kch * S;
  const int i = (int)(e % n), col = (int)((e / n) % k);
  const long long s = e / ((long long)n * k);
  const int c = col / S, q = col - c * S;
  N[e] = (i / (n / S) == q) ? z[(s * kch + c) * n + i] : 0.f;
}

// Its transpose: gz[s][c][i] = gN[s][c S + (segment of i)][i].
__global__ void segment_grad_kernel(int n, int kch, int S, long long total,
                                    const float *__restrict__ gN, float *__restrict__ gz) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int i = (int)(e % n), c = (int)((e / n) % kch);
  const long long s = e / ((long long)n * kch);
  const int q = i / (n / S);
  gz[e] = gN[(s * kch * S + (long long)c * S + q) * n + i];
}

// Wt[ci][co][j'] = W[co][ci][width - 1 - j']: the backward-data pass is a forward
// convolution of the output gradient with these weights.
__global__ void flip_transpose_kernel(int cin, int cout, int width, const float *__restrict__ W,
                                      float *__restrict__ Wt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= cin * cout * width) return;
  const int j = k % width, co = (k / width) % cout, ci = k / (width * cout);
  Wt[k] = W[((size_t)co * cin + ci) * width + (width - 1 - j)];
}

// g *= (act > 0): ReLU derivative applied to the gradient of a hidden layer's output.
__global__ void relu_mask_kernel(long long count, const float *__restrict__ act,
                                 float *__restrict__ g) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count && !(act[i] > 0.f)) g[i] = 0.f;
}

// Weight gradient gW[co][ci][j] = sum_s sum_i g[s][co][i] h[s][ci][(i + j - r) mod n] and
// bias gradient gb[co] = sum_s sum_i g[s][co][i], in two passes with a fixed summation
// order. Pass 1: a workgroup takes one chunk of CP grid points of one sample, 16 output
// and 16 input channels; g rows and h rows (with the halo) are staged in LDS, thread
// (co, ci) slides a W-wide register window along the chunk and keeps W FP32 sums.
// Pass 2 adds the chunks' partial sums in FP64, chunk by chunk.
template <int W>
__global__ void __launch_bounds__(256)
    conv_bwd_weight_part_kernel(int n, int cin, int cout, int CP, int chunks_per_sample,
                                const float *__restrict__ g, const float *__restrict__ h,
                                float *__restrict__ part_w, float *__restrict__ part_b) {
  extern __shared__ float sh[];
  constexpr int r = W / 2;
  const int span = CP + W - 1, hld = span + 1;  // odd row stride: no LDS bank conflicts
  float *Gs = sh;                              // [16][CP]
  float *Hs = sh + 16 * CP;                    // [16][hld]
  const int chunk = blockIdx.x, s = chunk / chunks_per_sample;
  const int i0 = (chunk - s * chunks_per_sample) * CP;
  const int ci0 = blockIdx.y * 16, co0 = blockIdx.z * 16;
  for (int e = threadIdx.x; e < 16 * CP; e += blockDim.x) {
    const int cl = e / CP, p = e - cl * CP;
    Gs[e] = (co0 + cl < cout) ? g[((size_t)s * cout + co0 + cl) * n + i0 + p] : 0.f;
  }
  for (int e = threadIdx.x; e < 16 * span; e += blockDim.x) {
    const int cl = e / span, p = e - cl * span;
    int gi = i0 + p - r;
    gi = gi < 0 ? gi + n : (gi >= n ? gi - n : gi);
    Hs[cl * hld + p] = (ci0 + cl < cin) ? h[((size_t)s * cin + ci0 + cl) * n + gi] : 0.f;
  }
  __syncthreads();
  const int col = threadIdx.x / 16, cil = threadIdx.x % 16;
  const float *gr = Gs + col * CP;
  const float *hr = Hs + cil * hld;
  float acc[W], win[W];
  float accb = 0.f;
#pragma unroll
  for (int q = 0; q < W; ++q) acc[q] = 0.f;
#pragma unroll
  for (int q = 0; q < W - 1; ++q) win[q + 1] = hr[q];
  for (int p = 0; p < CP; ++p) {
#pragma unroll
    for (int q = 0; q < W - 1; ++q) win[q] = win[q + 1];
    win[W - 1] = hr[p + W - 1];
    const float gp = gr[p];
    accb += gp;
#pragma unroll
    for (int q = 0; q < W; ++q) acc[q] = fmaf(gp, win[q], acc[q]);
  }
  const int co = co0 + col, ci = ci0 + cil;
  if (co < cout && ci < cin) {
    float *o = part_w + ((size_t)chunk * cout + co) * cin * W + (size_t)ci * W;
#pragma unroll
    for (int q = 0; q < W; ++q) o[q] = acc[q];
  }
  if (blockIdx.y == 0 && cil == 0 && co < cout) part_b[(size_t)chunk * cout + co] = accb;
}

// out[e] = sum over chunks c = 0, 1, ... of part[c * count + e] (FP64, in chunk order).
__global__ void chunk_sum_kernel(long long count, int chunks, const float *__restrict__ part,
                                 float *__restrict__ out) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  double acc = 0.0;
  for (int c = 0; c < chunks; ++c) acc += (double)part[(size_t)c * count + e];
  out[e] = (float)acc;
}

__global__ void adam_kernel(long long count, float *__restrict__ p, const float *__restrict__ g,
                            float *__restrict__ m, float *__restrict__ v, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void f2d_kernel(long long count, const float *__restrict__ a, double *__restrict__ b) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) b[i] = (double)a[i];
}

// Y[col * ldy + i] = (double) X[col * n + i]: network output columns into an FP64 block.
__global__ void widen_kernel(int n, long long cols, const float *__restrict__ X,
                             double *__restrict__ Y, int ldy) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cols * n) return;
  const long long col = e / n;
  Y[col * ldy + (e - col * n)] = (double)X[e];
}

// identity blocks (k x k per sample)
__global__ void eye_kernel(int k, int batch, double *__restrict__ I) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)k * k * batch) return;
  const int e = (int)(i % ((long long)k * k));
  I[i] = (e % k == e / k) ? 1.0 : 0.0;
}

// WA[s][i][j] = w[s][i] A[s][i][j] (A column-major k x k per sample)
__global__ void scale_rows_kernel(int k, int batch, const double *__restrict__ w,
                                  const double *__restrict__ A, double *__restrict__ WA) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)k * k * batch) return;
  const int s = (int)(i / ((long long)k * k));
  const int row = (int)(i % k);
  WA[i] = w[(size_t)s * k + row] * A[i];
}

// gN[s] = -(2 / sum w) (X - PX) as FP32
__global__ void capture_grad_kernel(int n, int k, const double *__restrict__ w,
                                    const double *__restrict__ X, const double *__restrict__ PX,
                                    float *__restrict__ gN) {
  const int s = blockIdx.y;
  double sw = 0.0;
  for (int i = 0; i < k; ++i) sw += w[(size_t)s * k + i];
  const size_t nk = (size_t)n * k;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < nk;
       e += (size_t)gridDim.x * blockDim.x)
    gN[s * nk + e] = (float)(-(2.0 / sw) * (X[s * nk + e] - PX[s * nk + e]));
}

// loss[s] = -(1 / sum w) sum_i w_i sum_j C_ij A_ij (C, A column-major k x k per sample);
// one workgroup per sample, fixed-order tree reduction.
__global__ void __launch_bounds__(256)
    capture_value_kernel(int k, const double *__restrict__ w, const double *__restrict__ C,
                         const double *__restrict__ A, double *__restrict__ loss) {
  __shared__ double red[256];
  const int s = blockIdx.x;
  const size_t kk = (size_t)k * k;
  double acc = 0.0;
  for (size_t e = threadIdx.x; e < kk; e += blockDim.x)
    acc += w[(size_t)s * k + e % k] * C[s * kk + e] * A[s * kk + e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double sw = 0.0;
    for (int i = 0; i < k; ++i) sw += w[(size_t)s * k + i];
    loss[s] = -red[0] / sw;
  }
}

unsigned nblocks(long long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace
}  // namespace riot

struct riot_net {
  riot_net_desc d{};
  hipStream_t st = nullptr;
  long long nparams = 0;
  std::vector<long long> woff, boff;  // per layer offsets into the flat parameters
  std::vector<int> cin, cout;
  float *params = nullptr, *grads = nullptr, *am = nullptr, *av = nullptr;
  float *x0 = nullptr;               // standardized inputs [batch][in_channels][n]
  std::vector<float *> acts;         // per layer outputs [batch][cout][n]
  float *g0 = nullptr, *g1 = nullptr, *Wt = nullptr, *gN = nullptr;
  float *Nout = nullptr;             // network output after the head [batch][k][n]
  float *wpart = nullptr;            // per-chunk partial weight and bias gradients
  // loss workspace (FP64)
  double *Nd = nullptr, *G = nullptr, *Lc = nullptr, *Z = nullptr, *Gi = nullptr, *A = nullptr,
         *WA = nullptr, *C = nullptr, *Y1 = nullptr, *Y2 = nullptr, *MN = nullptr, *X = nullptr,
         *PX = nullptr, *loss = nullptr;
  int *flags = nullptr;
  riot::CholJob *chol_jobs = nullptr;
  riot::TrsmJob *trsm_jobs = nullptr;
};

namespace {

size_t n256(size_t b) { return (b + 255) / 256 * 256; }

// grid points per chunk of the weight-gradient pass (divides n)
int chunk_points(int n) { return n % 256 == 0 ? 256 : (n % 128 == 0 ? 128 : 64); }

struct NCarve {
  char *base;
  size_t off = 0;
  explicit NCarve(void *b) : base(static_cast<char *>(b)) {}
  template <typename T>
  T *take(size_t n) {
    off = n256(off);
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += std::max<size_t>(n, 1) * sizeof(T);
    return p;
  }
};

bool net_desc_ok(const riot_net_desc *d) {
  return d && d->n >= 64 && d->n % 64 == 0 && d->layers >= 1 && d->layers <= 16 &&
         d->channels >= 1 && d->channels <= 64 && d->k >= 1 && d->k <= 64 && d->k <= d->n &&
         d->width >= 1 && d->width % 2 == 1 && d->width <= riot::kMaxWidth &&
         d->batch_max >= 1 && d->segments >= 1 && d->n % d->segments == 0 &&
         d->k % d->segments == 0 && d->in_channels >= 1 && d->in_channels <= 64;
}

size_t net_carve(riot_net &h, void *base) {
  NCarve c(base);
  const riot_net_desc &d = h.d;
  h.woff.clear(), h.boff.clear(), h.cin.clear(), h.cout.clear();
  long long np = 0;
  int ci = d.in_channels;
  int maxc = 1;
  for (int l = 0; l < d.layers; ++l) {
    const int co = (l == d.layers - 1) ? d.k / d.segments : d.channels;
    h.cin.push_back(ci), h.cout.push_back(co);
    h.woff.push_back(np);
    np += (long long)co * ci * d.width;
    h.boff.push_back(np);
    np += co;
    maxc = std::max(maxc, co);
    ci = co;
  }
  h.nparams = np;
  const size_t B = d.batch_max, n = d.n, k = d.k, kk = (size_t)k * k;
  h.params = c.take<float>(np);
  h.grads = c.take<float>(np);
  h.am = c.take<float>(np);
  h.av = c.take<float>(np);
  h.x0 = c.take<float>(B * d.in_channels * n);
  h.acts.assign(d.layers, nullptr);
  for (int l = 0; l < d.layers; ++l) h.acts[l] = c.take<float>(B * h.cout[l] * n);
  h.g0 = c.take<float>(B * maxc * n);
  h.g1 = c.take<float>(B * maxc * n);
  h.Wt = c.take<float>((size_t)maxc * maxc * d.width);
  h.gN = c.take<float>(B * k * n);
  h.Nout = c.take<float>(B * k * n);
  {
    const size_t chunks = B * (n / chunk_points((int)n));
    size_t mx = 0;
    for (int l = 0; l < d.layers; ++l)
      mx = std::max(mx, (size_t)h.cout[l] * h.cin[l] * d.width + h.cout[l]);
    h.wpart = c.take<float>(chunks * mx);
  }
  h.Nd = c.take<double>(B * n * k);
  h.G = c.take<double>(B * kk);
  h.Lc = c.take<double>(B * kk);
  h.Z = c.take<double>(B * kk);
  h.Gi = c.take<double>(B * kk);
  h.A = c.take<double>(B * kk);
  h.WA = c.take<double>(B * kk);
  h.C = c.take<double>(B * kk);
  h.Y1 = c.take<double>(B * kk);
  h.Y2 = c.take<double>(B * kk);
  h.MN = c.take<double>(B * n * k);
  h.X = c.take<double>(B * n * k);
  h.PX = c.take<double>(B * n * k);
  h.loss = c.take<double>(B);
  h.flags = c.take<int>(2 * B);
  h.chol_jobs = c.take<riot::CholJob>(B);
  h.trsm_jobs = c.take<riot::TrsmJob>(B);
  return n256(c.off) + 256;
}

#define NET_HIP(call)                           \
  do {                                          \
    if ((call) != hipSuccess) return RIOT_E_HIP; \
  } while (0)

riot_status conv_forward(riot_net *h, int batch, const float *in, int cin, int cout,
                         const float *W, const float *b, float *out, bool relu) {
  const int n = h->d.n, width = h->d.width;
  const size_t lds = ((size_t)cin * (riot::kCX + width - 1) + (size_t)riot::kCC * cin * width) *
                     sizeof(float);
  hipLaunchKernelGGL(riot::conv_fwd_kernel, dim3(n / riot::kCX, (cout + riot::kCC - 1) / riot::kCC, batch),
                     dim3(256), lds, h->st, n, cin, cout, width, in, W, b, out, relu ? 1 : 0);
  NET_HIP(hipGetLastError());
  return RIOT_OK;
}

template <int W>
void launch_wgrad_part(dim3 grid, size_t lds, hipStream_t st, int n, int cin, int cout, int CP,
                       int cps, const float *g, const float *hin, float *pw, float *pb) {
  hipLaunchKernelGGL(riot::conv_bwd_weight_part_kernel<W>, grid, dim3(256), lds, st, n, cin, cout,
                     CP, cps, g, hin, pw, pb);
}

riot_status weight_grad(riot_net *h, int batch, int cin, int cout, const float *g,
                        const float *hin, float *gW, float *gb) {
  const int n = h->d.n, W = h->d.width, CP = chunk_points(n), cps = n / CP;
  const int chunks = batch * cps;
  const dim3 grid(chunks, (cin + 15) / 16, (cout + 15) / 16);
  const size_t lds = (16 * (size_t)CP + 16 * (size_t)(CP + W)) * sizeof(float);
  float *pw = h->wpart, *pb = h->wpart + (size_t)chunks * cout * cin * W;
  switch (W) {
    case 1: launch_wgrad_part<1>(grid, lds, h->st, n, cin, cout, CP, cps, g, hin, pw, pb); break;
    case 3: launch_wgrad_part<3>(grid, lds, h->st, n, cin, cout, CP, cps, g, hin, pw, pb); break;
    case 5: launch_wgrad_part<5>(grid, lds, h->st, n, cin, cout, CP, cps, g, hin, pw, pb); break;
    case 7: launch_wgrad_part<7>(grid, lds, h->st, n, cin, cout, CP, cps, g, hin, pw, pb); break;
    case 9: launch_wgrad_part<9>(grid, lds, h->st, n, cin, cout, CP, cps, g, hin, pw, pb); break;
    case 11: launch_wgrad_part<11>(grid, lds, h->st, n, cin, cout, CP, cps, g, hin, pw, pb); break;
    default: return RIOT_E_ARG;
  }
  NET_HIP(hipGetLastError());
  const long long cw = (long long)cout * cin * W;
  hipLaunchKernelGGL(riot::chunk_sum_kernel, dim3(riot::nblocks(cw)), dim3(256), 0, h->st, cw,
                     chunks, pw, gW);
  NET_HIP(hipGetLastError());
  hipLaunchKernelGGL(riot::chunk_sum_kernel, dim3(riot::nblocks(cout)), dim3(256), 0, h->st,
                     (long long)cout, chunks, pb, gb);
  NET_HIP(hipGetLastError());
  return RIOT_OK;
}

}  // namespace

extern "C" {

size_t riot_net_workspace_bytes(const riot_net_desc *desc) {
  if (!net_desc_ok(desc)) return 0;
  riot_net h;
  h.d = *desc;
  return net_carve(h, nullptr);
}

riot_status riot_net_init(const riot_net_desc *desc, void *workspace, size_t bytes,
                          void *hip_stream, riot_net **out) {
  if (!out) return RIOT_E_ARG;
  *out = nullptr;
  if (!net_desc_ok(desc) || !workspace) return RIOT_E_ARG;
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return RIOT_E_WORKSPACE;
  if (bytes < riot_net_workspace_bytes(desc)) return RIOT_E_WORKSPACE;
  riot_net *h = new (std::nothrow) riot_net();
  if (!h) return RIOT_E_ARG;
  h->d = *desc;
  h->st = static_cast<hipStream_t>(hip_stream);
  net_carve(*h, workspace);
  // batched Cholesky / triangular-solve jobs of the loss (k x k per sample)
  const int k = desc->k, B = desc->batch_max;
  const size_t kk = (size_t)k * k;
  std::vector<riot::CholJob> cj(B);
  std::vector<riot::TrsmJob> tj(B);
  for (int s = 0; s < B; ++s) {
    cj[s] = {k, h->G + s * kk, h->Lc + s * kk, 0.0, h->flags + 2 * s, h->flags + 2 * s + 1,
             nullptr, nullptr};
    tj[s] = {k, k, h->Z + s * kk, k, h->Lc + s * kk, nullptr};
  }
  riot_status rs = RIOT_OK;
  if (hipMemcpyAsync(h->chol_jobs, cj.data(), B * sizeof(riot::CholJob), hipMemcpyHostToDevice,
                     h->st) != hipSuccess ||
      hipMemcpyAsync(h->trsm_jobs, tj.data(), B * sizeof(riot::TrsmJob), hipMemcpyHostToDevice,
                     h->st) != hipSuccess ||
      hipStreamSynchronize(h->st) != hipSuccess)
    rs = RIOT_E_HIP;
  if (rs != RIOT_OK) {
    delete h;
    return rs;
  }
  *out = h;
  return RIOT_OK;
}

void riot_net_free(riot_net *h) { delete h; }

int64_t riot_net_param_count(const riot_net *h) { return h ? h->nparams : 0; }

riot_status riot_net_set_params(riot_net *h, const float *params, const float *grads) {
  if (!h) return RIOT_E_ARG;
  if (params)
    NET_HIP(hipMemcpyAsync(h->params, params, h->nparams * sizeof(float),
                           hipMemcpyDeviceToDevice, h->st));
  if (grads)
    NET_HIP(hipMemcpyAsync(h->grads, grads, h->nparams * sizeof(float), hipMemcpyDeviceToDevice,
                           h->st));
  return RIOT_OK;
}

riot_status riot_net_get_params(riot_net *h, float *params, float *grads) {
  if (!h) return RIOT_E_ARG;
  if (params)
    NET_HIP(hipMemcpyAsync(params, h->params, h->nparams * sizeof(float),
                           hipMemcpyDeviceToDevice, h->st));
  if (grads)
    NET_HIP(hipMemcpyAsync(grads, h->grads, h->nparams * sizeof(float), hipMemcpyDeviceToDevice,
                           h->st));
  return RIOT_OK;
}

riot_status riot_net_forward(riot_net *h, int32_t batch, const double *x, float *N,
                             double *N64, int32_t ld64) {
  if (!h || !x || batch < 1 || batch > h->d.batch_max) return RIOT_E_ARG;
  const int n = h->d.n, k = h->d.k;
  if (N64 && ld64 < n) return RIOT_E_ARG;
  hipLaunchKernelGGL(riot::standardize_kernel, dim3(batch * h->d.in_channels), dim3(256), 0, h->st,
                     n, x, h->x0);
  NET_HIP(hipGetLastError());
  const float *in = h->x0;
  for (int l = 0; l < h->d.layers; ++l) {
    const bool last = l == h->d.layers - 1;
    float *out = h->acts[l];
    riot_status rs = conv_forward(h, batch, in, h->cin[l], h->cout[l], h->params + h->woff[l],
                                  h->params + h->boff[l], out, !last);
    if (rs != RIOT_OK) return rs;
    in = out;
  }
  const int S = h->d.segments;
  const long long tot = (long long)batch * k * n;
  float *res = N ? N : h->Nout;
  hipLaunchKernelGGL(riot::segment_out_kernel, dim3(riot::nblocks(tot)), dim3(256), 0, h->st, n,
                     k / S, S, tot, h->acts[h->d.layers - 1], res);
  NET_HIP(hipGetLastError());
  if (N64) {
    hipLaunchKernelGGL(riot::widen_kernel, dim3(riot::nblocks((long long)batch * k * n)), dim3(256),
                       0, h->st, n, (long long)batch * k, res, N64, ld64);
    NET_HIP(hipGetLastError());
  }
  return RIOT_OK;
}

riot_status riot_net_backward(riot_net *h, int32_t batch, const float *gN) {
  if (!h || !gN || batch < 1 || batch > h->d.batch_max) return RIOT_E_ARG;
  const int n = h->d.n, width = h->d.width, L = h->d.layers;
  const int S = h->d.segments, kch = h->d.k / S;
  const long long tot = (long long)batch * kch * n;
  hipLaunchKernelGGL(riot::segment_grad_kernel, dim3(riot::nblocks(tot)), dim3(256), 0, h->st, n,
                     kch, S, tot, gN, h->g0);
  NET_HIP(hipGetLastError());
  float *g = h->g0, *gnext = h->g1;
  for (int l = L - 1; l >= 0; --l) {
    const int ci = h->cin[l], co = h->cout[l];
    if (l < L - 1) {
      hipLaunchKernelGGL(riot::relu_mask_kernel, dim3(riot::nblocks((long long)batch * co * n)),
                         dim3(256), 0, h->st, (long long)batch * co * n, h->acts[l], g);
      NET_HIP(hipGetLastError());
    }
    const float *hin = l == 0 ? h->x0 : h->acts[l - 1];
    {
      riot_status rs = weight_grad(h, batch, ci, co, g, hin, h->grads + h->woff[l],
                                   h->grads + h->boff[l]);
      if (rs != RIOT_OK) return rs;
    }
    if (l > 0) {
      hipLaunchKernelGGL(riot::flip_transpose_kernel, dim3(riot::nblocks((long long)ci * co * width)),
                         dim3(256), 0, h->st, ci, co, width, h->params + h->woff[l], h->Wt);
      NET_HIP(hipGetLastError());
      riot_status rs = conv_forward(h, batch, g, co, ci, h->Wt, nullptr, gnext, false);
      if (rs != RIOT_OK) return rs;
      std::swap(g, gnext);
    }
  }
  return RIOT_OK;
}

riot_status riot_net_adam(riot_net *h, float lr, float beta1, float beta2, float eps, int32_t step) {
  if (!h || step < 1) return RIOT_E_ARG;
  const float c1 = 1.f - std::pow(beta1, (float)step), c2 = 1.f - std::pow(beta2, (float)step);
  if (step == 1) {
    NET_HIP(hipMemsetAsync(h->am, 0, h->nparams * sizeof(float), h->st));
    NET_HIP(hipMemsetAsync(h->av, 0, h->nparams * sizeof(float), h->st));
  }
  hipLaunchKernelGGL(riot::adam_kernel, dim3(riot::nblocks(h->nparams)), dim3(256), 0, h->st,
                     (long long)h->nparams, h->params, h->grads, h->am, h->av, lr, beta1, beta2,
                     eps, c1, c2);
  NET_HIP(hipGetLastError());
  return RIOT_OK;
}

riot_status riot_net_capture_loss(riot_net *h, int32_t batch, const float *N, const double *V,
                                  const double *w, double *loss_host, float *gN) {
  if (!h || !N || !V || !w || !gN || batch < 1 || batch > h->d.batch_max) return RIOT_E_ARG;
  const int n = h->d.n, k = h->d.k;
  const long long nk = (long long)n * k, kk = (long long)k * k;
  hipStream_t st = h->st;
  hipLaunchKernelGGL(riot::f2d_kernel, dim3(riot::nblocks(nk * batch)), dim3(256), 0, st,
                     nk * batch, N, h->Nd);
  NET_HIP(hipGetLastError());
  // G = N^T N = L L^T, Gi = L^{-T} L^{-1}
  NET_HIP(riot::gemm_f64_strided(1, 0, k, k, n, 1.0, h->Nd, n, nk, h->Nd, n, nk, 0.0, h->G, k, kk,
                                 batch, st));
  NET_HIP(riot::launch_chol_batched(batch, 0, h->chol_jobs, st));
  hipLaunchKernelGGL(riot::eye_kernel, dim3(riot::nblocks(kk * batch)), dim3(256), 0, st, k, batch,
                     h->Z);
  NET_HIP(hipGetLastError());
  NET_HIP(riot::launch_trsm_batched(batch, k, h->trsm_jobs, st));  // Z = L^{-T}
  NET_HIP(riot::gemm_f64_strided(0, 1, k, k, k, 1.0, h->Z, k, kk, h->Z, k, kk, 0.0, h->Gi, k, kk,
                                 batch, st));
  // A = V^T N, M N = V diag(w) A, X = M N Gi, P X = N Gi N^T X, C = A Gi
  NET_HIP(riot::gemm_f64_strided(1, 0, k, k, n, 1.0, V, n, nk, h->Nd, n, nk, 0.0, h->A, k, kk,
                                 batch, st));
  hipLaunchKernelGGL(riot::scale_rows_kernel, dim3(riot::nblocks(kk * batch)), dim3(256), 0, st, k,
                     batch, w, h->A, h->WA);
  NET_HIP(hipGetLastError());
  NET_HIP(riot::gemm_f64_strided(0, 0, n, k, k, 1.0, V, n, nk, h->WA, k, kk, 0.0, h->MN, n, nk,
                                 batch, st));
  NET_HIP(riot::gemm_f64_strided(0, 0, n, k, k, 1.0, h->MN, n, nk, h->Gi, k, kk, 0.0, h->X, n, nk,
                                 batch, st));
  NET_HIP(riot::gemm_f64_strided(1, 0, k, k, n, 1.0, h->Nd, n, nk, h->X, n, nk, 0.0, h->Y1, k, kk,
                                 batch, st));
  NET_HIP(riot::gemm_f64_strided(0, 0, k, k, k, 1.0, h->Gi, k, kk, h->Y1, k, kk, 0.0, h->Y2, k, kk,
                                 batch, st));
  NET_HIP(riot::gemm_f64_strided(0, 0, n, k, k, 1.0, h->Nd, n, nk, h->Y2, k, kk, 0.0, h->PX, n, nk,
                                 batch, st));
  NET_HIP(riot::gemm_f64_strided(0, 0, k, k, k, 1.0, h->A, k, kk, h->Gi, k, kk, 0.0, h->C, k, kk,
                                 batch, st));
  hipLaunchKernelGGL(riot::capture_grad_kernel, dim3(64, batch), dim3(256), 0, st, n, k, w, h->X,
                     h->PX, gN);
  NET_HIP(hipGetLastError());
  hipLaunchKernelGGL(riot::capture_value_kernel, dim3(batch), dim3(256), 0, st, k, w, h->C, h->A,
                     h->loss);
  NET_HIP(hipGetLastError());
  if (loss_host) {
    NET_HIP(hipMemcpyAsync(loss_host, h->loss, batch * sizeof(double), hipMemcpyDeviceToHost, st));
    NET_HIP(hipStreamSynchronize(st));
  }
  return RIOT_OK;
}

riot_status riot_net_train_step(riot_net *h, int32_t batch, const double *x, const double *V,
                                const double *w, float lr, int32_t step, double *loss_host) {
  if (!h || !x || !V || !w || batch < 1 || batch > h->d.batch_max || step < 1) return RIOT_E_ARG;
  riot_status rs = riot_net_forward(h, batch, x, nullptr, nullptr, 0);
  if (rs != RIOT_OK) return rs;
  rs = riot_net_capture_loss(h, batch, h->Nout, V, w, loss_host, h->gN);
  if (rs != RIOT_OK) return rs;
  rs = riot_net_backward(h, batch, h->gN);
  if (rs != RIOT_OK) return rs;
  return riot_net_adam(h, lr, 0.9f, 0.999f, 1e-8f, step);
}

}  // extern "C"
