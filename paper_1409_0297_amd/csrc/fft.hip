// Complex FP64 FFT passes for the pseudospectral operator (Section 2.1, eq. G).
//
// One kernel transforms all grid lines along one axis of a [batch][outer][n][inner]
// array: each workgroup stages L lines in LDS (coalesced: along the line when
// inner == 1, across neighbouring lines otherwise), runs a mixed radix-4/2/3
// Stockham autosort FFT in LDS, and writes the lines back.  Optional fused
// pointwise work at the edges of the pass:
//   pre  : multiply the input by a real grid function (q in q .* z),
//   mid  : forward transform, multiply by a real array in Fourier order
//          (sigma_k / N), inverse transform -- the whole of G along the last
//          axis pass of a multi-axis transform,
//   add  : output = add + result (the "z +" of (I + G q) z).
// Forward and inverse transforms are unnormalised; the 1/N of the unitary
// pair F^{-1} (.) F is folded into the sigma array.
#include "common.hpp"
#include "kernels.hpp"

namespace spp {

namespace {

constexpr int kFftThreads = 256;
constexpr int kMaxStages = 12;

struct FftArgs {
  int n;
  int L;             // lines per workgroup
  int64_t outer, inner;
  int64_t N;         // grid size (batch stride)
  int nstages;
  int radix[kMaxStages];
};

__device__ inline double2 twiddle(const double2* tw, int m, int dir) {
  double2 w = tw[m];
  if (dir > 0) w.y = -w.y;
  return w;
}

// One Stockham stage of radix R over L lines of length n held in LDS.
template <int R>
__device__ void stockham_stage(const double2* __restrict__ x, double2* __restrict__ y, int n, int L,
                               int Ns, int dir, const double2* __restrict__ tw) {
  const int nb = n / R;              // butterflies per line
  const int stride_tw = n / (Ns * R);
  for (int t = threadIdx.x; t < L * nb; t += blockDim.x) {
    const int line = t / nb;
    const int j = t - line * nb;
    const double2* xl = x + line * n;
    double2* yl = y + line * n;
    const int k = j % Ns;
    double2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = xl[j + r * nb];
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], twiddle(tw, (r * k * stride_tw) % n, dir));
    double2 o[R];
    if constexpr (R == 2) {
      o[0] = cadd(v[0], v[1]);
      o[1] = csub(v[0], v[1]);
    } else if constexpr (R == 4) {
      // i^(dir) rotation: forward uses -i, inverse +i.
      double2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
      double2 c = cadd(v[1], v[3]), e = csub(v[1], v[3]);
      double2 ie = (dir < 0) ? cmake<double2>(e.y, -e.x) : cmake<double2>(-e.y, e.x);
      o[0] = cadd(a, c);
      o[1] = cadd(b, ie);
      o[2] = csub(a, c);
      o[3] = csub(b, ie);
    } else {  // R == 3
      const double c1 = -0.5;
      const double s1 = (dir < 0 ? -1.0 : 1.0) * 0.86602540378443864676;
      double2 sum = cadd(v[1], v[2]), dif = csub(v[1], v[2]);
      double2 m1 = cmake<double2>(v[0].x + c1 * sum.x, v[0].y + c1 * sum.y);
      double2 m2 = cmake<double2>(-s1 * dif.y, s1 * dif.x);   // i s1 (v1 - v2)
      o[0] = cadd(v[0], sum);
      o[1] = cadd(m1, m2);
      o[2] = csub(m1, m2);
    }
    const int base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) yl[base + r * Ns] = o[r];
  }
}

// Runs all stages; data starts in a, returns the buffer holding the result.
__device__ double2* fft_lines(double2* a, double2* b, const FftArgs& g, int dir, const double2* tw) {
  int Ns = 1;
  for (int s = 0; s < g.nstages; ++s) {
    const int R = g.radix[s];
    __syncthreads();
    if (R == 4) stockham_stage<4>(a, b, g.n, g.L, Ns, dir, tw);
    else if (R == 2) stockham_stage<2>(a, b, g.n, g.L, Ns, dir, tw);
    else stockham_stage<3>(a, b, g.n, g.L, Ns, dir, tw);
    Ns *= R;
    double2* t = a; a = b; b = t;
  }
  __syncthreads();
  return a;
}

__global__ void __launch_bounds__(kFftThreads)
fft_axis_kernel(const double2* in, double2* out, const double2* __restrict__ tw, FftArgs g,
                int dir, const double* __restrict__ pre, const double* __restrict__ mid,
                const double2* add, int per) {
  extern __shared__ double2 lds[];
  double2* A = lds;
  double2* B = lds + g.L * g.n;
  const int64_t lines_per_batch = g.outer * g.inner;
  const int64_t wg_per_batch = lines_per_batch / g.L;
  const int64_t batch = blockIdx.x / wg_per_batch;
  const int64_t line0 = (blockIdx.x - batch * wg_per_batch) * g.L;
  const int64_t bofs = batch * g.N;
  const int64_t aofs = (batch / per) * g.N;   // per-instance multiplier arrays
  const int total = g.L * g.n;

  auto addr = [&](int li, int k) -> int64_t {   // grid index (within one batch entry)
    const int64_t line = line0 + li;
    const int64_t o = line / g.inner, i = line - o * g.inner;
    return o * g.n * g.inner + (int64_t)k * g.inner + i;
  };
  auto unpack = [&](int t, int& li, int& k) {
    if (g.inner == 1) { li = t / g.n; k = t - li * g.n; }
    else { k = t / g.L; li = t - k * g.L; }
  };

  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    int li, k;
    unpack(t, li, k);
    const int64_t a = addr(li, k);
    double2 v = in[bofs + a];
    if (pre) { const double s = pre[aofs + a]; v.x *= s; v.y *= s; }
    A[li * g.n + k] = v;
  }
  double2* res = fft_lines(A, B, g, dir, tw);
  if (mid) {
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
      int li, k;
      unpack(t, li, k);
      const double s = mid[aofs + addr(li, k)];
      double2& v = res[li * g.n + k];
      v.x *= s; v.y *= s;
    }
    double2* other = (res == A) ? B : A;
    res = fft_lines(res, other, g, -dir, tw);
  }
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    int li, k;
    unpack(t, li, k);
    const int64_t a = addr(li, k);
    double2 v = res[li * g.n + k];
    if (add) v = cadd(v, add[bofs + a]);
    out[bofs + a] = v;
  }
}

// ------------------------------------------------------------------ radix-8
// Lengths n = 8^S (64, 512, 4096): a register Stockham FFT.  T = n / 8 lanes
// per line hold 8 points each; a stage is one radix-8 butterfly per lane in
// registers, with an LDS exchange between stages (S stages, S - 1 exchanges
// per transform).  A workgroup takes L lines: along the line (inner == 1,
// lane = position-major) or L neighbouring lines of a strided axis (lane =
// line-major, so a load of the L lines' entries at one position is one
// contiguous L x 16 B piece).  Same fused options as fft_axis_kernel.
__device__ inline double2 rot_i(double2 z, int dir) {   // dir * i * z
  return (dir < 0) ? cmake<double2>(z.y, -z.x) : cmake<double2>(-z.y, z.x);
}

__device__ inline void dft8(double2* v, int dir) {
  // Evens and odds by 4-point DFTs, then y_k = E_k + w^k O_k, y_{k+4} = E_k - w^k O_k.
  const double2 t0 = cadd(v[0], v[4]), t1 = csub(v[0], v[4]);
  const double2 t2 = cadd(v[2], v[6]), t3 = rot_i(csub(v[2], v[6]), dir);
  const double2 e0 = cadd(t0, t2), e2 = csub(t0, t2), e1 = cadd(t1, t3), e3 = csub(t1, t3);
  const double2 u0 = cadd(v[1], v[5]), u1 = csub(v[1], v[5]);
  const double2 u2 = cadd(v[3], v[7]), u3 = rot_i(csub(v[3], v[7]), dir);
  const double2 o0 = cadd(u0, u2), o2 = csub(u0, u2), o1 = cadd(u1, u3), o3 = csub(u1, u3);
  constexpr double h = 0.70710678118654752440;   // 1 / sqrt(2)
  // w = exp(dir 2 pi i / 8): w^1 = (1 + dir i) h, w^2 = dir i, w^3 = (-1 + dir i) h
  const double2 w1o1 = cmake<double2>(h * (o1.x - dir * o1.y), h * (o1.y + dir * o1.x));
  const double2 w2o2 = rot_i(o2, dir);
  const double2 w3o3 = cmake<double2>(h * (-o3.x - dir * o3.y), h * (-o3.y + dir * o3.x));
  v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
  v[1] = cadd(e1, w1o1); v[5] = csub(e1, w1o1);
  v[2] = cadd(e2, w2o2); v[6] = csub(e2, w2o2);
  v[3] = cadd(e3, w3o3); v[7] = csub(e3, w3o3);
}

// LDS index of line position i: one pad entry per 8 (the stage writes go 8
// or Ns apart per lane; the pad spreads them over the banks).
__device__ inline int pad8(int i) { return i + (i >> 3); }

// All S stages of one transform direction; on entry v[r] = x[t + T r], on
// exit v[r] = y[t + T r] (the last stage's outputs land in natural order).
// lds = this line's n + n / 8 entries.
template <int S>
__device__ inline void fft8_stages(double2* v, double2* lds, int t, int dir, const double2* __restrict__ tw) {
  constexpr int n = 1 << (3 * S), T = n / 8;
#pragma unroll
  for (int st = 0; st < S; ++st) {
    const int Ns = 1 << (3 * st);
    const int k = t & (Ns - 1);
    if (st > 0) {
      const int stride = n / (Ns * 8);
#pragma unroll
      for (int r = 1; r < 8; ++r) v[r] = cmul(v[r], twiddle(tw, (r * k * stride) & (n - 1), dir));
    }
    dft8(v, dir);
    if (st + 1 < S) {
      const int base = (t / Ns) * Ns * 8 + k;
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 8; ++r) lds[pad8(base + r * Ns)] = v[r];
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 8; ++r) v[r] = lds[pad8(t + T * r)];
    }
  }
}

template <int S, int L, bool STRIDED>
__global__ void __launch_bounds__((1 << (3 * S)) / 8 * L)
fft8_axis_kernel(const double2* in, double2* out, const double2* __restrict__ tw, int64_t outer, int64_t inner,
                 int64_t N, int dir, const double* __restrict__ pre, const double* __restrict__ mid,
                 const double2* add, int per) {
  constexpr int n = 1 << (3 * S), T = n / 8;
  extern __shared__ double2 lds8[];
  const int tid = threadIdx.x;
  const int li = STRIDED ? tid % L : tid / T;
  const int t = STRIDED ? tid / L : tid % T;
  const int64_t lines_per_batch = outer * inner;
  const int64_t wg_per_batch = lines_per_batch / L;
  const int64_t batch = blockIdx.x / wg_per_batch;
  const int64_t line = (blockIdx.x - batch * wg_per_batch) * L + li;
  const int64_t bofs = batch * N;
  const int64_t aofs = (batch / per) * N;
  const int64_t o = line / inner, i = line - o * inner;
  const int64_t lbase = o * n * inner + i;   // grid index of position 0 of this line
  double2* my = lds8 + li * (n + n / 8);
  double2 v[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int64_t a = lbase + (int64_t)(t + T * r) * inner;
    v[r] = in[bofs + a];
    if (pre) { const double q = pre[aofs + a]; v[r].x *= q; v[r].y *= q; }
  }
  fft8_stages<S>(v, my, t, dir, tw);
  if (mid) {
    // Fourier-side multiplier, then the inverse transform of the same lines
    // (the registers already hold the entries in the order it starts from).
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const double m = mid[aofs + lbase + (int64_t)(t + T * r) * inner];
      v[r].x *= m; v[r].y *= m;
    }
    fft8_stages<S>(v, my, t, -dir, tw);
  }
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int64_t a = lbase + (int64_t)(t + T * r) * inner;
    double2 y = v[r];
    if (add) y = cadd(y, add[bofs + a]);
    out[bofs + a] = y;
  }
}

__global__ void twiddle_kernel(double2* tw, int n) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < n) {
    double s, c;
    sincospi(2.0 * m / n, &s, &c);
    tw[m] = cmake<double2>(c, -s);   // exp(-2 pi i m / n)
  }
}

}  // namespace

void fft_make_twiddles(double2* tw, int n, hipStream_t st) {
  twiddle_kernel<<<ceil_div(n, 256), 256, 0, st>>>(tw, n);
  SPP_LAUNCH_CHECK();
}

bool fft_supported(int n) {
  while (n % 4 == 0) n /= 4;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

// Lines per workgroup: a power of two dividing the line count (and the
// inner stride), with two LDS buffers of L n complex values (<= 128 KB).
bool fft_lines_valid(int n, int64_t outer, int64_t inner, int L) {
  if (L < 1 || (L & (L - 1)) || (int64_t)L * n > 4096) return false;
  const int64_t lines = outer * inner;
  return lines % L == 0 && (inner == 1 || inner % L == 0);
}

// Default: fill about 2048 points of LDS per buffer.
int fft_lines_default(int n, int64_t outer, int64_t inner) {
  int L = 1;
  while (2 * L * n <= 2048) L *= 2;
  while (L > 1 && !fft_lines_valid(n, outer, inner, L)) L /= 2;
  return L;
}

std::string fft_tune_key(int n, int64_t outer, int64_t inner, int batch) {
  return tune_key("fft_lines", {n, outer, inner, batch});
}

void fft_axis(hipStream_t st, const double2* in, double2* out, const double2* tw, int n,
              int64_t outer, int64_t inner, int64_t N, int batch, int dir,
              const double* pre, const double* mid, const double2* add, int per) {
  FftArgs g{};
  g.n = n;
  g.outer = outer;
  g.inner = inner;
  g.N = N;
  int m = n, s = 0;
  while (m % 4 == 0) { g.radix[s++] = 4; m /= 4; }
  while (m % 2 == 0) { g.radix[s++] = 2; m /= 2; }
  while (m % 3 == 0) { g.radix[s++] = 3; m /= 3; }
  if (m != 1 || s > kMaxStages) throw Error(-7, "FFT length must be 2^a 3^b");
  g.nstages = s;
  const int64_t lines = outer * inner;
  // Algorithmic bytes: read and write every complex point once, plus the
  // fused real multipliers and the added vector.
  {
    const double pts = (double)N * batch;
    const double ninst = (double)((batch + per - 1) / per);
    const double bytes = pts * 32.0 + (pre ? 8.0 * N * ninst : 0.0) + (mid ? 8.0 * N * ninst : 0.0) +
                         (add ? 16.0 * pts : 0.0);
    const int perv = per > 0 ? per : batch;
    // Radix-8 lengths: L lines per workgroup from the same tuning table as
    // the general kernel (L in {1, 2, 4, 8} at n = 512, {8, 16, 32} at 64).
    if ((n == 512 || n == 64) && (inner == 1 || inner % 8 == 0)) {
      const bool strided = inner != 1;
      int L8 = tune_get(fft_tune_key(n, outer, inner, batch), n == 512 ? (strided ? 4 : 2) : 32);
      if (n == 512) L8 = std::min(std::max(L8, 1), 8);
      else L8 = std::min(std::max(L8, 8), 32);
      while (L8 > 1 && (lines % L8 != 0 || (strided && inner % L8 != 0))) L8 /= 2;
      const size_t row = sizeof(double2) * (n + n / 8);
      const unsigned blocks = (unsigned)(batch * (lines / L8));
      const unsigned threads = (unsigned)(n / 8 * L8);
      const void* kern = nullptr;
#define SPP_FFT8(S_, L_)                                                                   \
  if (n == (1 << (3 * S_)) && L8 == L_)                                                  \
    kern = strided ? (const void*)fft8_axis_kernel<S_, L_, true> : (const void*)fft8_axis_kernel<S_, L_, false>;
      SPP_FFT8(3, 1) SPP_FFT8(3, 2) SPP_FFT8(3, 4) SPP_FFT8(3, 8)
      SPP_FFT8(2, 8) SPP_FFT8(2, 16) SPP_FFT8(2, 32)
#undef SPP_FFT8
      if (kern && threads >= 64 && threads <= 1024) {
        int64_t outer_v = outer, inner_v = inner, N_v = N;
        int dir_v = dir, per_v = perv;
        void* args[] = {(void*)&in, (void*)&out, (void*)&tw, &outer_v, &inner_v, &N_v, &dir_v,
                        (void*)&pre, (void*)&mid, (void*)&add, &per_v};
        timer_begin(KC_FFT, st);
        SPP_HIP(hipLaunchKernel(kern, dim3(blocks), dim3(threads), args, L8 * row, st));
        timer_end(KC_FFT, st, bytes, 0.0);
        return;
      }
    }
  }
  int L = tune_get(fft_tune_key(n, outer, inner, batch), fft_lines_default(n, outer, inner));
  if (!fft_lines_valid(n, outer, inner, L)) L = fft_lines_default(n, outer, inner);
  g.L = L;
  const size_t lds = 2 * sizeof(double2) * L * n;
  const unsigned blocks = static_cast<unsigned>(batch * (lines / L));
  // Algorithmic bytes: read and write every complex point once, plus the
  // fused real multipliers and the added vector.
  const double pts = (double)N * batch;
  const double ninst = (double)((batch + per - 1) / per);
  const double bytes = pts * 32.0 + (pre ? 8.0 * N * ninst : 0.0) + (mid ? 8.0 * N * ninst : 0.0) + (add ? 16.0 * pts : 0.0);
  timer_begin(KC_FFT, st);
  fft_axis_kernel<<<blocks, kFftThreads, lds, st>>>(in, out, tw, g, dir, pre, mid, add, per > 0 ? per : batch);
  SPP_LAUNCH_CHECK();
  timer_end(KC_FFT, st, bytes, 0.0);
}

// (I + G q) z, G f, or plain transforms, over all d axes of [batch][n]^d.
void fft_multi(hipStream_t st, const double2* in, double2* out, double2* tmp, const double2* tw,
               int d, int n, int batch, const double* pre, const double* sigma, const double2* add, int per) {
  const int64_t N = (d == 2) ? (int64_t)n * n : (int64_t)n * n * n;
  if (d == 2) {
    fft_axis(st, in, tmp, tw, n, n, 1, N, batch, -1, pre, nullptr, nullptr, per);
    fft_axis(st, tmp, tmp, tw, n, 1, n, N, batch, -1, nullptr, sigma, nullptr, per);
    fft_axis(st, tmp, out, tw, n, n, 1, N, batch, +1, nullptr, nullptr, add, per);
  } else {
    fft_axis(st, in, tmp, tw, n, (int64_t)n * n, 1, N, batch, -1, pre, nullptr, nullptr, per);
    fft_axis(st, tmp, tmp, tw, n, n, n, N, batch, -1, nullptr, nullptr, nullptr, per);
    fft_axis(st, tmp, tmp, tw, n, 1, (int64_t)n * n, N, batch, -1, nullptr, sigma, nullptr, per);
    fft_axis(st, tmp, tmp, tw, n, n, n, N, batch, +1, nullptr, nullptr, nullptr, per);
    fft_axis(st, tmp, out, tw, n, (int64_t)n * n, 1, N, batch, +1, nullptr, nullptr, add, per);
  }
}

// Maxwell: w(k) = G(k) v(k) / N for the d components of each right-hand
// side at every wave vector, in place (G's symbol as in maxwell_symbol_kernel:
// first-derivative wave numbers with the Nyquist index dropped).
__global__ void vector_symbol_kernel(double2* __restrict__ v, int d, int n, int64_t N, int nrhs, double s) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= N * nrhs) return;
  const int64_t rhs = t / N, j = t - rhs * N;
  double kt[3] = {0, 0, 0};
  int64_t r = j;
  for (int a = d - 1; a >= 0; --a) {
    const int ra = (int)(r % n);
    r /= n;
    kt[a] = (ra == n / 2) ? 0.0 : (double)((ra > n / 2) ? ra - n : ra);
  }
  double k2 = 0;
  for (int a = 0; a < d; ++a) k2 += kt[a] * kt[a];
  const double pi = 3.14159265358979323846;
  const double trans = 1.0 / (4.0 * pi * pi * k2 - s) / (double)N, lon = 1.0 / (s * (double)N);
  double2* x = v + rhs * d * N + j;
  double2 in[3];
  for (int a = 0; a < d; ++a) in[a] = x[a * N];
  // G v = trans v - (trans + lon) kt (kt . v) / |kt|^2
  double2 dot = cmake<double2>(0, 0);
  for (int a = 0; a < d; ++a) dot = cmake<double2>(dot.x + kt[a] * in[a].x, dot.y + kt[a] * in[a].y);
  const double f = k2 > 0 ? (trans + lon) / k2 : 0.0;
  const double t0 = k2 > 0 ? trans : -lon;   // (kt = 0: G = -I / s)
  for (int a = 0; a < d; ++a)
    x[a * N] = cmake<double2>(t0 * in[a].x - f * kt[a] * dot.x, t0 * in[a].y - f * kt[a] * dot.y);
}

void fft_vector_green(hipStream_t st, const double2* in, double2* out, double2* tmp, const double2* tw, int d,
                      int n, int nrhs, double s, const double* pre, const double2* add) {
  const int64_t N = (d == 2) ? (int64_t)n * n : (int64_t)n * n * n;
  const int batch = nrhs * d;   // (pre: one array for every grid, per = batch)
  if (d == 2) {
    fft_axis(st, in, tmp, tw, n, n, 1, N, batch, -1, pre, nullptr, nullptr, batch);
    fft_axis(st, tmp, tmp, tw, n, 1, n, N, batch, -1, nullptr, nullptr, nullptr, batch);
  } else {
    fft_axis(st, in, tmp, tw, n, (int64_t)n * n, 1, N, batch, -1, pre, nullptr, nullptr, batch);
    fft_axis(st, tmp, tmp, tw, n, n, n, N, batch, -1, nullptr, nullptr, nullptr, batch);
    fft_axis(st, tmp, tmp, tw, n, 1, (int64_t)n * n, N, batch, -1, nullptr, nullptr, nullptr, batch);
  }
  timer_begin(KC_FFT, st);
  vector_symbol_kernel<<<(unsigned)ceil_div(N * nrhs, 256), 256, 0, st>>>(tmp, d, n, N, nrhs, s);
  SPP_LAUNCH_CHECK();
  timer_end(KC_FFT, st, 32.0 * N * batch, 0.0);
  if (d == 2) {
    fft_axis(st, tmp, tmp, tw, n, 1, n, N, batch, +1, nullptr, nullptr, nullptr, batch);
    fft_axis(st, tmp, out, tw, n, n, 1, N, batch, +1, nullptr, nullptr, add, batch);
  } else {
    fft_axis(st, tmp, tmp, tw, n, 1, (int64_t)n * n, N, batch, +1, nullptr, nullptr, nullptr, batch);
    fft_axis(st, tmp, tmp, tw, n, n, n, N, batch, +1, nullptr, nullptr, nullptr, batch);
    fft_axis(st, tmp, out, tw, n, (int64_t)n * n, 1, N, batch, +1, nullptr, nullptr, add, batch);
  }
}

// Unnormalised inverse transform over all axes (Green kernel construction).
void fft_inverse_all(hipStream_t st, const double2* in, double2* out, const double2* tw, int d, int n) {
  const int64_t N = (d == 2) ? (int64_t)n * n : (int64_t)n * n * n;
  if (d == 2) {
    fft_axis(st, in, out, tw, n, n, 1, N, 1, +1, nullptr, nullptr, nullptr, 1);
    fft_axis(st, out, out, tw, n, 1, n, N, 1, +1, nullptr, nullptr, nullptr, 1);
  } else {
    fft_axis(st, in, out, tw, n, (int64_t)n * n, 1, N, 1, +1, nullptr, nullptr, nullptr, 1);
    fft_axis(st, out, out, tw, n, n, n, N, 1, +1, nullptr, nullptr, nullptr, 1);
    fft_axis(st, out, out, tw, n, 1, (int64_t)n * n, N, 1, +1, nullptr, nullptr, nullptr, 1);
  }
}

}  // namespace spp
