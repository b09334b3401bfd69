// Small convolutional network used as a cheap flexible-GMRES preconditioner
// stage: 3 x 3 cross-correlations with circular padding, no bias, ReLU after
// every layer but the last.  Training and inference kernels:
//   conv_kernel      forward (and backward-data) as an implicit GEMM on MFMA:
//                    rows = 16-pixel row segments, columns = output channels,
//                    reduction = (tap, input channel); ReLU / ReLU-mask fused
//                    into the store;
//   wgrad_kernel     weight gradient per tap, pixels as the reduction axis,
//                    staged transposed in LDS; split over pixel chunks with
//                    deterministic partial sums (wgrad_reduce_kernel);
//   loss / Adam      per-sample relative squared error and its gradient;
//                    Adam on FP32 master weights.
// Activations and gradients are stored as T (bf16 or fp32), channels last
// ([batch][n][n][C]); every MFMA accumulates in FP32 (16x16x32 bf16 or
// 16x16x4 f32).  Weights are kept in FP32 in the (Cout, Cin, 3, 3) layout and
// rounded to T when a kernel stages them in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "spp.h"

namespace spp {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

template <typename T> struct Mma;
template <> struct Mma<__bf16> {
  static constexpr int KS = 32;       // reduction length of one MFMA
  static constexpr int KPL = 8;       // values per lane: k = 8 (lane / 16) + i
  using Frag = bf8;
  __device__ static f4 mma(Frag a, Frag b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};
template <> struct Mma<float> {
  static constexpr int KS = 4;
  static constexpr int KPL = 1;       // k = lane / 16
  using Frag = float;
  __device__ static f4 mma(Frag a, Frag b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};

template <typename T> __device__ inline T to_t(float x);
template <> __device__ inline __bf16 to_t<__bf16>(float x) { return (__bf16)x; }
template <> __device__ inline float to_t<float>(float x) { return x; }
template <typename T> __device__ inline float to_f(T x) { return (float)x; }

template <typename T> __device__ inline void frag_set(typename Mma<T>::Frag& f, int i, T v);
template <> __device__ inline void frag_set<__bf16>(bf8& f, int i, __bf16 v) { f[i] = v; }
template <> __device__ inline void frag_set<float>(float& f, int, float v) { f = v; }

constexpr int kMaxC = 32;   // channels per layer
constexpr int kTaps = 9;

// conv_kernel: out[pix][n] = sum_{tap, k} in[pix shifted by tap][k] * W_tap[n][k]
//   forward:       k = input channel c, n = output channel o, shift +tap,
//                  W_tap[o][c] = w[o][c][tap]; store relu (hidden) or FP32 (last)
//   backward-data: k = o, n = c, shift -tap, W_tap[c][o] = w[o][c][tap];
//                  store g * (mask > 0) with mask = the layer's input activation
// One wave: 16 consecutive pixels of one grid row x all n (<= 32).
template <typename T, bool BWD>
__global__ void __launch_bounds__(256) conv_kernel(const T* __restrict__ in, int kin, const float* __restrict__ w,
                                                   int cout, int cin, int nout, T* __restrict__ out_t,
                                                   float* __restrict__ out_f, const T* __restrict__ mask, int relu,
                                                   int n, int64_t npix) {
  using M = Mma<T>;
  constexpr int KP = kMaxC;   // padded reduction width (a multiple of KS)
  __shared__ T Ws[kTaps][kMaxC][KP + (sizeof(T) == 2 ? 8 : 1)];
  for (int e = threadIdx.x; e < kTaps * kMaxC * KP; e += 256) {
    const int t = e / (kMaxC * KP), r = e - t * kMaxC * KP, nn = r / KP, k = r - nn * KP;
    float v = 0.f;
    if (nn < nout && k < kin) {
      const int o = BWD ? k : nn, c = BWD ? nn : k;
      v = w[((int64_t)o * cin + c) * kTaps + t];
    }
    Ws[t][nn][k] = to_t<T>(v);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t p0 = ((int64_t)blockIdx.x * 4 + wave) * 16;   // first pixel of this wave (16 | n)
  if (p0 >= npix) return;
  const int64_t nn2 = (int64_t)n * n;
  const int64_t b = p0 / nn2;
  const int rem = (int)(p0 - b * nn2);
  const int i0 = rem / n, j0 = rem - i0 * n;
  const int row = lane & 15, kq = lane >> 4;
  const int ntiles = (nout + 15) / 16;
  f4 acc[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
  const int kmax = ((kin + M::KS - 1) / M::KS) * M::KS;
  for (int t = 0; t < kTaps; ++t) {
    int dy = t / 3 - 1, dx = t % 3 - 1;
    if (BWD) { dy = -dy; dx = -dx; }
    const int si = (i0 + dy + n) % n, sj = (j0 + row + dx + n) % n;
    const T* src = in + ((b * n + si) * n + sj) * kin;
    for (int kc = 0; kc < kmax; kc += M::KS) {
      typename M::Frag a, bf[2];
      const int k0 = kc + M::KPL * kq;
#pragma unroll
      for (int i = 0; i < M::KPL; ++i) frag_set<T>(a, i, (k0 + i < kin) ? src[k0 + i] : to_t<T>(0.f));
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int i = 0; i < M::KPL; ++i) frag_set<T>(bf[nt], i, Ws[t][nt * 16 + row][k0 + i]);
      acc[0] = M::mma(a, bf[0], acc[0]);
      if (ntiles > 1) acc[1] = M::mma(a, bf[1], acc[1]);
    }
  }
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    const int ch = nt * 16 + row;
    if (nt >= ntiles || ch >= nout) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t pix = p0 + 4 * kq + r;
      float v = acc[nt][r];
      if (BWD) {
        if (mask && !(to_f(mask[pix * nout + ch]) > 0.f)) v = 0.f;
        out_t[pix * nout + ch] = to_t<T>(v);
      } else if (out_f) {
        out_f[pix * nout + ch] = v;
      } else {
        out_t[pix * nout + ch] = to_t<T>(relu ? fmaxf(v, 0.f) : v);
      }
    }
  }
}

// Weight gradient of one tap over a chunk of pixels:
//   part[chunk][tap][c][o] = sum_{pix in chunk} x[pix + tap][c] * g[pix][o]
// Pixels are staged 64 at a time, transposed in LDS (channel-major), so each
// lane's MFMA fragment is a contiguous run of pixels.
constexpr int kWgPix = 64;

template <typename T>
__global__ void __launch_bounds__(256) wgrad_kernel(const T* __restrict__ x, int cin, const T* __restrict__ g, int cout,
                                                    int n, int64_t npix, int64_t chunk_pix, float* __restrict__ part) {
  using M = Mma<T>;
  constexpr int PAD = (sizeof(T) == 2) ? 8 : 1;
  __shared__ T xs[kMaxC][kWgPix + PAD];
  __shared__ T gs[kMaxC][kWgPix + PAD];
  const int t = blockIdx.y;
  const int dy = t / 3 - 1, dx = t % 3 - 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ct = wave & 1, ot = wave >> 1;    // this wave's 16 x 16 output tile
  const int row = lane & 15, kq = lane >> 4;
  const int64_t nn2 = (int64_t)n * n;
  const int64_t c0 = (int64_t)blockIdx.x * chunk_pix;
  const int64_t c1 = min(npix, c0 + chunk_pix);
  f4 acc = {0, 0, 0, 0};
  for (int64_t q0 = c0; q0 < c1; q0 += kWgPix) {
    for (int e = threadIdx.x; e < kWgPix * kMaxC; e += 256) {
      const int pl = e / kMaxC, ch = e - pl * kMaxC;
      const int64_t pix = q0 + pl;
      T xv = to_t<T>(0.f), gv = to_t<T>(0.f);
      if (pix < c1) {
        if (ch < cin) {
          const int64_t b = pix / nn2;
          const int rem = (int)(pix - b * nn2);
          const int i = rem / n, j = rem - (rem / n) * n;
          const int si = (i + dy + n) % n, sj = (j + dx + n) % n;
          xv = x[((b * n + si) * n + sj) * cin + ch];
        }
        if (ch < cout) gv = g[pix * cout + ch];
      }
      xs[ch][pl] = xv;
      gs[ch][pl] = gv;
    }
    __syncthreads();
    for (int kk = 0; kk < kWgPix; kk += M::KS) {
      typename M::Frag a, bb;
#pragma unroll
      for (int i = 0; i < M::KPL; ++i) {
        frag_set<T>(a, i, xs[ct * 16 + row][kk + M::KPL * kq + i]);
        frag_set<T>(bb, i, gs[ot * 16 + row][kk + M::KPL * kq + i]);
      }
      acc = M::mma(a, bb, acc);
    }
    __syncthreads();
  }
  float* out = part + ((int64_t)blockIdx.x * kTaps + t) * kMaxC * kMaxC;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int c = ct * 16 + 4 * kq + r, o = ot * 16 + row;
    out[c * kMaxC + o] = acc[r];
  }
}

// gw[o][c][tap] = sum over chunks of part[chunk][tap][c][o] (fixed order).
__global__ void wgrad_reduce_kernel(const float* __restrict__ part, int nchunks, int cout, int cin,
                                    float* __restrict__ gw) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cout * cin * kTaps) return;
  const int o = e / (cin * kTaps), r = e - o * cin * kTaps, c = r / kTaps, t = r - c * kTaps;
  float s = 0.f;
  for (int k = 0; k < nchunks; ++k) s += part[((int64_t)k * kTaps + t) * kMaxC * kMaxC + c * kMaxC + o];
  gw[e] = s;
}

// complex128 [batch][N] -> T [batch][N][2] (re, im)
template <typename T>
__global__ void to_channels_kernel(const double2* __restrict__ v, T* __restrict__ x, int64_t count, double scale) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= count) return;
  const double2 z = v[e];
  x[2 * e] = to_t<T>((float)(z.x * scale));
  x[2 * e + 1] = to_t<T>((float)(z.y * scale));
}

__global__ void to_channels_f32_kernel(const double2* __restrict__ v, float* __restrict__ x, int64_t count) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= count) return;
  x[2 * e] = (float)v[e].x;
  x[2 * e + 1] = (float)v[e].y;
}

__global__ void from_channels_kernel(const float* __restrict__ y, double2* __restrict__ v, int64_t count,
                                     double scale) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= count) return;
  v[e] = make_double2((double)y[2 * e] * scale, (double)y[2 * e + 1] * scale);
}

// Per-sample sums of (y - t)^2 and t^2: part[b][blk][2].
__global__ void loss_partial_kernel(const float* __restrict__ y, const float* __restrict__ t, int64_t per,
                                    double* __restrict__ part) {
  const int b = blockIdx.y;
  const float* yb = y + (int64_t)b * per;
  const float* tb = t + (int64_t)b * per;
  double s0 = 0, s1 = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < per; e += (int64_t)gridDim.x * blockDim.x) {
    const double d = (double)yb[e] - (double)tb[e];
    s0 += d * d;
    s1 += (double)tb[e] * tb[e];
  }
  __shared__ double r0[256], r1[256];
  r0[threadIdx.x] = s0;
  r1[threadIdx.x] = s1;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) { r0[threadIdx.x] += r0[threadIdx.x + o]; r1[threadIdx.x] += r1[threadIdx.x + o]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((int64_t)b * gridDim.x + blockIdx.x) * 2] = r0[0];
    part[((int64_t)b * gridDim.x + blockIdx.x) * 2 + 1] = r1[0];
  }
}

// loss = mean_b num_b / den_b; scale_b = 2 / (den_b * batch).
__global__ void loss_final_kernel(const double* __restrict__ part, int nblk, int batch, double* __restrict__ loss,
                                  float* __restrict__ scale) {
  __shared__ double acc[256];
  double l = 0;
  for (int b = threadIdx.x; b < batch; b += blockDim.x) {
    double num = 0, den = 0;
    for (int k = 0; k < nblk; ++k) { num += part[((int64_t)b * nblk + k) * 2]; den += part[((int64_t)b * nblk + k) * 2 + 1]; }
    l += den > 0 ? num / den : 0.0;
    scale[b] = den > 0 ? (float)(2.0 / (den * batch)) : 0.f;
  }
  acc[threadIdx.x] = l;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) acc[threadIdx.x] += acc[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = acc[0] / batch;
}

template <typename T>
__global__ void loss_grad_kernel(const float* __restrict__ y, const float* __restrict__ t, const float* __restrict__ scale,
                                 int64_t per, int64_t count, T* __restrict__ g) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= count) return;
  g[e] = to_t<T>(scale[e / per] * (y[e] - t[e]));
}

__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t count, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= count) return;
  const float gg = g[e];
  const float mm = b1 * m[e] + (1.f - b1) * gg;
  const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
  m[e] = mm;
  v[e] = vv;
  w[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

}  // namespace
}  // namespace spp

using namespace spp;

// A network and its work buffers for up to max_batch samples of an n x n grid.
struct spp_cnn {
  int n = 0, nlayers = 0, dtype = 0, max_batch = 0;
  std::vector<int> ch;               // nlayers + 1 channel counts
  std::vector<int64_t> woff;         // weight offsets per layer (floats)
  int64_t nweights = 0;
  size_t tsize = 2;                  // bytes per activation
  std::vector<void*> allocs;
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr, *yout = nullptr, *tgt = nullptr, *part = nullptr,
        *scale = nullptr;
  double *lpart = nullptr, *lval = nullptr;
  std::vector<void*> act;            // activations: act[0] input, act[l+1] output of hidden layer l
  void *ga = nullptr, *gb = nullptr; // gradient ping-pong buffers
  int64_t part_chunks = 0;
  int adam_t = 0;
  template <typename X> X* dalloc(size_t count) {
    void* p = nullptr;
    SPP_HIP(hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(X)));
    allocs.push_back(p);
    return static_cast<X*>(p);
  }
  ~spp_cnn() {
    for (void* p : allocs) (void)hipFree(p);
  }
};

namespace {

thread_local std::string g_cnn_error;

template <typename F> int cnn_guarded(F&& fn) {
  try {
    return fn();
  } catch (const Error& e) {
    g_cnn_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    g_cnn_error = e.what();
    return SPP_EHIP;
  }
}

int64_t npix_of(const spp_cnn* N, int batch) { return (int64_t)batch * N->n * N->n; }

template <typename T>
void forward_t(spp_cnn* N, int batch, hipStream_t st) {
  const int64_t np = npix_of(N, batch);
  const unsigned grid = ceil_div(np, 64);
  for (int l = 0; l < N->nlayers; ++l) {
    const bool last = l == N->nlayers - 1;
    const int cin = N->ch[l], cout = N->ch[l + 1];
    conv_kernel<T, false><<<grid, 256, 0, st>>>(static_cast<const T*>(N->act[l]), cin, N->w + N->woff[l], cout, cin,
                                                 cout, last ? nullptr : static_cast<T*>(N->act[l + 1]),
                                                 last ? N->yout : nullptr, nullptr, last ? 0 : 1, N->n, np);
    SPP_LAUNCH_CHECK();
  }
}

template <typename T>
void backward_t(spp_cnn* N, int batch, hipStream_t st) {
  const int64_t np = npix_of(N, batch);
  const unsigned grid = ceil_div(np, 64);
  const int64_t chunk = std::max<int64_t>(kWgPix, ((np + 511) / 512 + kWgPix - 1) / kWgPix * kWgPix);
  const int nchunks = (int)ceil_div(np, chunk);
  T* gcur = static_cast<T*>(N->ga);
  T* gnext = static_cast<T*>(N->gb);
  for (int l = N->nlayers - 1; l >= 0; --l) {
    const int cin = N->ch[l], cout = N->ch[l + 1];
    wgrad_kernel<T><<<dim3(nchunks, kTaps), 256, 0, st>>>(static_cast<const T*>(N->act[l]), cin, gcur, cout, N->n, np,
                                                          chunk, N->part);
    SPP_LAUNCH_CHECK();
    const int nw = cout * cin * kTaps;
    wgrad_reduce_kernel<<<ceil_div(nw, 256), 256, 0, st>>>(N->part, nchunks, cout, cin, N->g + N->woff[l]);
    SPP_LAUNCH_CHECK();
    if (l == 0) break;
    // gradient w.r.t. this layer's input, masked by ReLU of that input
    conv_kernel<T, true><<<grid, 256, 0, st>>>(gcur, cout, N->w + N->woff[l], cout, cin, cin, gnext, nullptr,
                                               static_cast<const T*>(N->act[l]), 0, N->n, np);
    SPP_LAUNCH_CHECK();
    std::swap(gcur, gnext);
  }
}

void load_input(spp_cnn* N, const double2* x, int batch, hipStream_t st) {
  const int64_t cnt = npix_of(N, batch);
  if (N->dtype == SPP_CNN_BF16)
    to_channels_kernel<__bf16><<<ceil_div(cnt, 256), 256, 0, st>>>(x, static_cast<__bf16*>(N->act[0]), cnt, 1.0);
  else
    to_channels_kernel<float><<<ceil_div(cnt, 256), 256, 0, st>>>(x, static_cast<float*>(N->act[0]), cnt, 1.0);
  SPP_LAUNCH_CHECK();
}

void check_batch(const spp_cnn* N, int batch) {
  if (!N) throw Error(SPP_EINVAL, "null network");
  if (batch < 1 || batch > N->max_batch) throw Error(SPP_EINVAL, "batch must be in [1, max_batch]");
}

}  // namespace

namespace spp {
// Inference on Krylov vectors for the learned FGMRES stage: y = net(x) per
// sample (x, y complex128 [batch][n^2]); scale multiplies input and output
// (the network is positively homogeneous).
void cnn_apply(spp_cnn* N, const double2* x, double2* y, int batch, double in_scale, double out_scale,
               hipStream_t st) {
  check_batch(N, batch);
  const int64_t cnt = npix_of(N, batch);
  if (N->dtype == SPP_CNN_BF16) {
    to_channels_kernel<__bf16><<<ceil_div(cnt, 256), 256, 0, st>>>(x, static_cast<__bf16*>(N->act[0]), cnt, in_scale);
    SPP_LAUNCH_CHECK();
    forward_t<__bf16>(N, batch, st);
  } else {
    to_channels_kernel<float><<<ceil_div(cnt, 256), 256, 0, st>>>(x, static_cast<float*>(N->act[0]), cnt, in_scale);
    SPP_LAUNCH_CHECK();
    forward_t<float>(N, batch, st);
  }
  from_channels_kernel<<<ceil_div(cnt, 256), 256, 0, st>>>(N->yout, y, cnt, out_scale);
  SPP_LAUNCH_CHECK();
}
int cnn_grid(const spp_cnn* N) { return N->n; }
}  // namespace spp

extern "C" {

int spp_cnn_create(int32_t n, int32_t nlayers, const int32_t* channels, int32_t dtype, int32_t max_batch,
                   spp_cnn** out) {
  return cnn_guarded([&] {
    if (!out || !channels) throw Error(SPP_EINVAL, "null argument");
    *out = nullptr;
    if (n < 16 || n % 16 != 0) throw Error(SPP_EINVAL, "n must be a positive multiple of 16");
    if (nlayers < 1 || nlayers > 16) throw Error(SPP_EINVAL, "1 <= nlayers <= 16");
    if (dtype != SPP_CNN_BF16 && dtype != SPP_CNN_F32) throw Error(SPP_EINVAL, "unknown dtype");
    if (channels[0] != 2 || channels[nlayers] != 2) throw Error(SPP_EINVAL, "first and last channel counts must be 2");
    for (int l = 0; l <= nlayers; ++l)
      if (channels[l] < 1 || channels[l] > kMaxC) throw Error(SPP_EINVAL, "channel counts must be in [1, 32]");
    if (max_batch < 1) throw Error(SPP_EINVAL, "max_batch >= 1");
    auto N = std::make_unique<spp_cnn>();
    N->n = n; N->nlayers = nlayers; N->dtype = dtype; N->max_batch = max_batch;
    N->tsize = dtype == SPP_CNN_BF16 ? 2 : 4;
    N->ch.assign(channels, channels + nlayers + 1);
    for (int l = 0; l < nlayers; ++l) {
      N->woff.push_back(N->nweights);
      N->nweights += (int64_t)channels[l + 1] * channels[l] * kTaps;
    }
    N->w = N->dalloc<float>(N->nweights);
    N->g = N->dalloc<float>(N->nweights);
    N->m = N->dalloc<float>(N->nweights);
    N->v = N->dalloc<float>(N->nweights);
    SPP_HIP(hipMemset(N->w, 0, sizeof(float) * N->nweights));
    SPP_HIP(hipMemset(N->g, 0, sizeof(float) * N->nweights));
    SPP_HIP(hipMemset(N->m, 0, sizeof(float) * N->nweights));
    SPP_HIP(hipMemset(N->v, 0, sizeof(float) * N->nweights));
    const int64_t np = (int64_t)max_batch * n * n;
    for (int l = 0; l < nlayers; ++l) N->act.push_back(N->dalloc<char>((size_t)np * channels[l] * N->tsize));
    N->ga = N->dalloc<char>((size_t)np * kMaxC * N->tsize);
    N->gb = N->dalloc<char>((size_t)np * kMaxC * N->tsize);
    N->yout = N->dalloc<float>((size_t)np * 2);
    N->tgt = N->dalloc<float>((size_t)np * 2);
    N->part = N->dalloc<float>((size_t)600 * kTaps * kMaxC * kMaxC);
    N->lpart = N->dalloc<double>((size_t)max_batch * 64 * 2);
    N->lval = N->dalloc<double>(1);
    N->scale = N->dalloc<float>(max_batch);
    *out = N.release();
    return SPP_OK;
  });
}

int spp_cnn_weights(spp_cnn* net, const float* w_in, float* w_out, int64_t* count) {
  return cnn_guarded([&] {
    if (!net) throw Error(SPP_EINVAL, "null network");
    if (count) *count = net->nweights;
    if (w_in) {
      SPP_HIP(hipMemcpy(net->w, w_in, sizeof(float) * net->nweights, hipMemcpyHostToDevice));
      SPP_HIP(hipMemset(net->m, 0, sizeof(float) * net->nweights));
      SPP_HIP(hipMemset(net->v, 0, sizeof(float) * net->nweights));
      net->adam_t = 0;
    }
    if (w_out) SPP_HIP(hipMemcpy(w_out, net->w, sizeof(float) * net->nweights, hipMemcpyDeviceToHost));
    return SPP_OK;
  });
}

int spp_cnn_forward(spp_cnn* net, const void* x, int32_t batch, void* y, spp_stream_t stream) {
  return cnn_guarded([&] {
    check_batch(net, batch);
    if (!x || !y) throw Error(SPP_EINVAL, "null argument");
    cnn_apply(net, static_cast<const double2*>(x), static_cast<double2*>(y), batch, 1.0, 1.0,
              reinterpret_cast<hipStream_t>(stream));
    return SPP_OK;
  });
}

int spp_cnn_loss_grad(spp_cnn* net, const void* x, const void* t, int32_t batch, double* loss, float* grads,
                      spp_stream_t stream) {
  return cnn_guarded([&] {
    check_batch(net, batch);
    if (!x || !t) throw Error(SPP_EINVAL, "null argument");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t cnt = npix_of(net, batch);
    load_input(net, static_cast<const double2*>(x), batch, st);
    to_channels_f32_kernel<<<ceil_div(cnt, 256), 256, 0, st>>>(static_cast<const double2*>(t), net->tgt, cnt);
    SPP_LAUNCH_CHECK();
    if (net->dtype == SPP_CNN_BF16) forward_t<__bf16>(net, batch, st);
    else forward_t<float>(net, batch, st);
    const int64_t per = 2LL * net->n * net->n;
    const int nblk = 64;
    loss_partial_kernel<<<dim3(nblk, batch), 256, 0, st>>>(net->yout, net->tgt, per, net->lpart);
    SPP_LAUNCH_CHECK();
    loss_final_kernel<<<1, 256, 0, st>>>(net->lpart, nblk, batch, net->lval, net->scale);
    SPP_LAUNCH_CHECK();
    if (net->dtype == SPP_CNN_BF16) {
      loss_grad_kernel<__bf16><<<ceil_div(per * batch, 256), 256, 0, st>>>(net->yout, net->tgt, net->scale, per,
                                                                         per * batch, static_cast<__bf16*>(net->ga));
      SPP_LAUNCH_CHECK();
      backward_t<__bf16>(net, batch, st);
    } else {
      loss_grad_kernel<float><<<ceil_div(per * batch, 256), 256, 0, st>>>(net->yout, net->tgt, net->scale, per,
                                                                         per * batch, static_cast<float*>(net->ga));
      SPP_LAUNCH_CHECK();
      backward_t<float>(net, batch, st);
    }
    if (loss) {
      SPP_HIP(hipMemcpyAsync(loss, net->lval, sizeof(double), hipMemcpyDeviceToHost, st));
      SPP_HIP(hipStreamSynchronize(st));
    }
    if (grads) {
      SPP_HIP(hipMemcpyAsync(grads, net->g, sizeof(float) * net->nweights, hipMemcpyDeviceToHost, st));
      SPP_HIP(hipStreamSynchronize(st));
    }
    return SPP_OK;
  });
}

int spp_cnn_adam_step(spp_cnn* net, float lr, spp_stream_t stream) {
  return cnn_guarded([&] {
    if (!net) throw Error(SPP_EINVAL, "null network");
    if (!(lr > 0)) throw Error(SPP_EINVAL, "lr > 0");
    net->adam_t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)net->adam_t), c2 = 1.f - std::pow(b2, (float)net->adam_t);
    adam_kernel<<<ceil_div(net->nweights, 256), 256, 0, reinterpret_cast<hipStream_t>(stream)>>>(
        net->w, net->g, net->m, net->v, net->nweights, lr, b1, b2, 1e-8f, c1, c2);
    SPP_LAUNCH_CHECK();
    return SPP_OK;
  });
}

void spp_cnn_destroy(spp_cnn* net) {
  if (!net) return;
  (void)hipDeviceSynchronize();
  delete net;
}

const char* spp_cnn_last_error(void) { return g_cnn_error.c_str(); }

}  // extern "C"
