// FP64 kernels of flexible GMRES (right preconditioning, Section 3 of the paper;
// Saad and Schultz) on (I + G q) u = G f, batched over right-hand sides.
//
// Arnoldi uses classical Gram-Schmidt applied twice (CGS2): the projections
// onto all previous basis vectors are one pass of block dot products
// (wavefront shuffles, then a cross-workgroup pass) and one fused update,
// instead of j dependent dot/axpy pairs.  The Hessenberg columns, Givens
// rotations and the small triangular solve live on the device as well; the
// host only reads back the residual estimates to decide when to stop.
#include "common.hpp"
#include "kernels.hpp"

namespace spp {

namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 2;
constexpr int kMaxVec = 512;

__device__ inline double2 wave_sum(double2 v) {
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_down(v.x, o, 64);
    v.y += __shfl_down(v.y, o, 64);
  }
  return v;
}
__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// partial[(rhs * nvec + i) * nslot + slot] = sum over the wave's chunk of conj(V_i) w
// (vector-major, so that the final pass reads each vector's partials contiguously).
// dj (optional): the iteration index j in device memory (graph replays);
// then nvec = j + 1 and every j-dependent pointer is base + j * jstride.
__global__ void __launch_bounds__(kThreads) dots_partial_kernel(const double2* __restrict__ V, int64_t vstride, int nvec,
                                                                const double2* __restrict__ w, int64_t N,
                                                                double2* __restrict__ partial, const int* dj) {
  if (dj) nvec = *dj + 1;
  const int rhs = blockIdx.y;
  const int nslot = gridDim.x * (kThreads / 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int slot = blockIdx.x * (kThreads / 64) + wave;
  // Each wave sums its own kPerThread * 64 entries and writes one partial
  // per vector (no LDS: many small blocks keep enough loads in flight).
  const int64_t e0 = (int64_t)slot * 64 * kPerThread + lane;
  const double2* wr = w + rhs * N;
  double2 wl[kPerThread];
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const int64_t e = e0 + (int64_t)k * 64;
    wl[k] = (e < N) ? wr[e] : cmake<double2>(0, 0);
  }
  // Four vectors per pass: their loads are all in flight before any sum,
  // and the next pass's loads are issued before this pass's wave sums.
  constexpr int kG = 4;
  double2 cur[kG][kPerThread];
  auto load = [&](double2 (&b)[kG][kPerThread], int i0) {
#pragma unroll
    for (int q = 0; q < kG; ++q) {
      const double2* vr = V + (int64_t)(i0 + q) * vstride + rhs * N;
#pragma unroll
      for (int k = 0; k < kPerThread; ++k) {
        const int64_t e = e0 + (int64_t)k * 64;
        b[q][k] = (i0 + q < nvec && e < N) ? vr[e] : cmake<double2>(0, 0);
      }
    }
  };
  load(cur, 0);
  for (int i0 = 0; i0 < nvec; i0 += kG) {
    double2 nxt[kG][kPerThread];
    load(nxt, i0 + kG);
    double2 s[kG];
#pragma unroll
    for (int q = 0; q < kG; ++q) {
      s[q] = cmake<double2>(0, 0);
#pragma unroll
      for (int k = 0; k < kPerThread; ++k) s[q] = cadd(s[q], cconjmul(cur[q][k], wl[k]));
    }
#pragma unroll
    for (int q = 0; q < kG; ++q) {
      if (i0 + q >= nvec) break;
      const double2 t = wave_sum(s[q]);
      if (lane == 0) partial[((int64_t)rhs * nvec + i0 + q) * nslot + slot] = t;
    }
#pragma unroll
    for (int q = 0; q < kG; ++q)
#pragma unroll
      for (int k = 0; k < kPerThread; ++k) cur[q][k] = nxt[q][k];
  }
}

// One wavefront per (vector, right-hand side) sums the per-block partials.
__global__ void dots_final_kernel(const double2* __restrict__ partial, int nblk, int nvec, double2* h, int hstride,
                                  int accumulate, double2* h_acc, int acc_stride, const int* dj, int64_t h_jstride,
                                  int64_t acc_jstride) {
  if (dj) {
    const int j = *dj;
    nvec = j + 1;
    h += j * h_jstride;
    if (h_acc) h_acc += j * acc_jstride;
  }
  const int rhs = blockIdx.y;
  const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= nvec) return;
  double2 s = cmake<double2>(0, 0);
  const double2* pr = partial + ((int64_t)rhs * nvec + i) * nblk;
#pragma unroll 8
  for (int b = lane; b < nblk; b += 64) s = cadd(s, pr[b]);
  s = wave_sum(s);
  if (lane != 0) return;
  double2* hr = h + (int64_t)rhs * hstride;
  hr[i] = accumulate ? cadd(hr[i], s) : s;
  if (h_acc) {
    double2* ha = h_acc + (int64_t)rhs * acc_stride;
    ha[i] = cadd(ha[i], s);
  }
}

// w -= sum_i V_i h_i
__global__ void __launch_bounds__(kThreads) update_kernel(const double2* __restrict__ V, int64_t vstride, int nvec,
                                                          double2* __restrict__ w, int64_t N,
                                                          const double2* __restrict__ h, int hstride, const int* dj,
                                                          int64_t h_jstride) {
  if (dj) {
    nvec = *dj + 1;
    h += *dj * h_jstride;
  }
  const int rhs = blockIdx.y;
  __shared__ double2 hs[kMaxVec];
  for (int i = threadIdx.x; i < nvec; i += kThreads) hs[i] = h[(int64_t)rhs * hstride + i];
  __syncthreads();
  const int64_t e = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (e >= N) return;
  double2 acc = w[rhs * N + e];
#pragma unroll 8
  for (int i = 0; i < nvec; ++i) cfms(acc, V[(int64_t)i * vstride + rhs * N + e], hs[i]);
  w[rhs * N + e] = acc;
}

// CGS2 fused passes (eager iterations): w -= V h, then the partial dot
// products of the updated w with every V_i in the layout of
// dots_partial_kernel (each wave its own kPerThread * 64 entries: the wave
// updates exactly the entries it then projects, so no other workgroup's
// writes are involved).  The second sweep over V re-reads what the first
// just read.
__global__ void __launch_bounds__(kThreads) update_dots_kernel(const double2* __restrict__ V, int64_t vstride, int nvec,
                                                               double2* __restrict__ w, int64_t N,
                                                               const double2* __restrict__ h, int hstride,
                                                               double2* __restrict__ partial) {
  const int rhs = blockIdx.y;
  __shared__ double2 hs[kMaxVec];
  for (int i = threadIdx.x; i < nvec; i += kThreads) hs[i] = h[(int64_t)rhs * hstride + i];
  __syncthreads();
  const int nslot = gridDim.x * (kThreads / 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int slot = blockIdx.x * (kThreads / 64) + wave;
  const int64_t e0 = (int64_t)slot * 64 * kPerThread + lane;
  double2* wr = w + rhs * N;
  double2 wl[kPerThread];
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const int64_t e = e0 + (int64_t)k * 64;
    wl[k] = (e < N) ? wr[e] : cmake<double2>(0, 0);
  }
#pragma unroll 4
  for (int i = 0; i < nvec; ++i) {
    const double2* vr = V + (int64_t)i * vstride + rhs * N;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      const int64_t e = e0 + (int64_t)k * 64;
      if (e < N) cfms(wl[k], vr[e], hs[i]);
    }
  }
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const int64_t e = e0 + (int64_t)k * 64;
    if (e < N) wr[e] = wl[k];
  }
  for (int i = 0; i < nvec; ++i) {
    const double2* vr = V + (int64_t)i * vstride + rhs * N;
    double2 s = cmake<double2>(0, 0);
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      const int64_t e = e0 + (int64_t)k * 64;
      if (e < N) s = cadd(s, cconjmul(vr[e], wl[k]));
    }
    s = wave_sum(s);
    if (lane == 0) partial[((int64_t)rhs * nvec + i) * nslot + slot] = s;
  }
}

// w -= V h, and the partial sums of |w|^2 for the normalisation (grid
// (kNormBlocks, nrhs), the layout sumsq_partial_kernel writes).
constexpr int kNormBlocks = 256;
__global__ void __launch_bounds__(kThreads) update_sumsq_kernel(const double2* __restrict__ V, int64_t vstride,
                                                                int nvec, double2* __restrict__ w, int64_t N,
                                                                const double2* __restrict__ h, int hstride,
                                                                double* __restrict__ partial) {
  const int rhs = blockIdx.y;
  __shared__ double2 hs[kMaxVec];
  for (int i = threadIdx.x; i < nvec; i += kThreads) hs[i] = h[(int64_t)rhs * hstride + i];
  __syncthreads();
  double s = 0;
  for (int64_t e = blockIdx.x * (int64_t)kThreads + threadIdx.x; e < N; e += (int64_t)gridDim.x * kThreads) {
    double2 acc = w[rhs * N + e];
#pragma unroll 8
    for (int i = 0; i < nvec; ++i) cfms(acc, V[(int64_t)i * vstride + rhs * N + e], hs[i]);
    w[rhs * N + e] = acc;
    s += cabs2(acc);
  }
  s = wave_sum(s);
  __shared__ double sh[kThreads / 64];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int q = 0; q < kThreads / 64; ++q) t += sh[q];
    partial[(int64_t)rhs * gridDim.x + blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(kThreads) sumsq_partial_kernel(const double2* __restrict__ w, int64_t N,
                                                                 double* __restrict__ partial) {
  const int rhs = blockIdx.y;
  double s = 0;
  for (int64_t e = blockIdx.x * (int64_t)kThreads + threadIdx.x; e < N; e += (int64_t)gridDim.x * kThreads)
    s += cabs2(w[rhs * N + e]);
  s = wave_sum(s);
  __shared__ double sh[kThreads / 64];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int q = 0; q < kThreads / 64; ++q) t += sh[q];
    partial[(int64_t)rhs * gridDim.x + blockIdx.x] = t;
  }
}

// norms[rhs] = sqrt(sum of partials); optionally H entry = norm.  One
// wavefront (blockIdx.x) per right-hand side.
__global__ void __launch_bounds__(64) sumsq_final_kernel(const double* __restrict__ partial, int nblk, int nrhs,
                                                         double* norms, double2* h_sub, int hstride, const int* dj,
                                                         int64_t h_jstride) {
  if (dj && h_sub) h_sub += *dj * h_jstride;
  const int rhs = blockIdx.x;
  if (rhs >= nrhs) return;
  double s = 0;
  for (int b = threadIdx.x; b < nblk; b += 64) s += partial[(int64_t)rhs * nblk + b];
  s = wave_sum(s);
  if (threadIdx.x != 0) return;
  const double nrm = sqrt(s);
  norms[rhs] = nrm;
  if (h_sub) h_sub[(int64_t)rhs * hstride] = cmake<double2>(nrm, 0.0);
}

__device__ inline void givens_column(double2* H, int hcol, int hrhs, double* cs, double2* sn, double2* g, int j,
                                     int ldg, double* resid, int col, double* resid_host = nullptr);

// v = w / ||w||, the norm summed from the nblk partials by every workgroup
// (the same sum in the same order everywhere); workgroup 0 also stores the
// norm and the Hessenberg entry and, with gv.H set, makes the column's
// Givens rotation (column gv.c0 + right-hand side).
__global__ void __launch_bounds__(kThreads) norm_scale_kernel(const double2* __restrict__ w, double2* __restrict__ v,
                                                              const double* __restrict__ partial, int nblk,
                                                              double* norms, double2* h_sub, int hstride, int64_t N,
                                                              const int* dj, int64_t v_jstride, int64_t h_jstride,
                                                              KrGivens gv) {
  if (dj) {
    v += *dj * v_jstride;
    if (h_sub) h_sub += *dj * h_jstride;
    gv.j = *dj;
  }
  const int rhs = blockIdx.y;
  __shared__ double nrm_s;
  if (threadIdx.x < 64) {
    double s = 0;
    for (int b = threadIdx.x; b < nblk; b += 64) s += partial[(int64_t)rhs * nblk + b];
    s = wave_sum(s);
    if (threadIdx.x == 0) {
      const double nrm = sqrt(s);
      nrm_s = nrm;
      if (blockIdx.x == 0) {
        norms[rhs] = nrm;
        if (h_sub) h_sub[(int64_t)rhs * hstride] = cmake<double2>(nrm, 0.0);
        if (gv.H)
          givens_column(gv.H, gv.hcol, gv.hrhs, gv.cs, gv.sn, gv.g, gv.j, gv.ldg, gv.resid, gv.c0 + rhs,
                        gv.resid_host);
      }
    }
  }
  __syncthreads();
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= N) return;
  const double nrm = nrm_s;
  const double inv = nrm > 0 ? 1.0 / nrm : 0.0;
  v[rhs * N + e] = cscale(w[rhs * N + e], inv);
}

__global__ void scale_kernel(const double2* __restrict__ w, double2* __restrict__ v, const double* __restrict__ norms,
                             int64_t N, const int* dj, int64_t v_jstride) {
  if (dj) v += *dj * v_jstride;
  const int rhs = blockIdx.y;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= N) return;
  const double nrm = norms[rhs];
  const double inv = nrm > 0 ? 1.0 / nrm : 0.0;
  v[rhs * N + e] = cscale(w[rhs * N + e], inv);
}

// Complex Givens rotation G = [[c, s], [-conj(s), c]] with c real that maps
// (a, b) to (r, 0): c = |a| / t, s = (a/|a|) conj(b) / t, r = (a/|a|) t.
__device__ inline void make_givens(double2 a, double2 b, double& c, double2& s, double2& r) {
  const double aa = sqrt(cabs2(a)), bb = sqrt(cabs2(b));
  if (bb == 0) { c = 1; s = cmake<double2>(0, 0); r = a; return; }
  if (aa == 0) { c = 0; s = cmake<double2>(b.x / bb, -b.y / bb); r = cmake<double2>(bb, 0); return; }
  const double t = hypot(aa, bb);
  const double2 ph = cmake<double2>(a.x / aa, a.y / aa);
  c = aa / t;
  s = cscale(cmul(ph, cmake<double2>(b.x, -b.y)), 1.0 / t);
  r = cscale(ph, t);
}

// Column `col` of the Hessenberg matrix: apply the earlier rotations, make
// the new one, update g and the residual estimate |g_{j+1}|.
__device__ inline void givens_column(double2* H, int hcol, int hrhs, double* cs, double2* sn, double2* g, int j,
                                     int ldg, double* resid, int col, double* resid_host) {
  double2* h = H + (int64_t)col * hrhs + (int64_t)j * hcol;
  double* c = cs + (int64_t)col * ldg;
  double2* s = sn + (int64_t)col * ldg;
  double2* gg = g + (int64_t)col * ldg;
  for (int i = 0; i < j; ++i) {
    const double2 hi = h[i], hi1 = h[i + 1];
    const double2 t = cadd(cscale(hi, c[i]), cmul(s[i], hi1));
    h[i + 1] = csub(cscale(hi1, c[i]), cconjmul(s[i], hi));
    h[i] = t;
  }
  double cj;
  double2 sj, r;
  make_givens(h[j], h[j + 1], cj, sj, r);
  c[j] = cj;
  s[j] = sj;
  h[j] = r;
  h[j + 1] = cmake<double2>(0, 0);
  const double2 gj = gg[j];
  gg[j + 1] = cscale(cconjmul(sj, gj), -1.0);
  gg[j] = cscale(gj, cj);
  const double rj = sqrt(cabs2(gg[j + 1]));
  resid[col] = rj;
  if (resid_host) resid_host[col] = rj;   // read by the host after the launch's event
}

__global__ void givens_kernel(double2* H, int hcol, int hrhs, double* cs, double2* sn, double2* g, int j,
                              int nrhs, int ldg, double* resid, const int* active, const int* dj) {
  if (dj) j = *dj;
  const int rhs = blockIdx.x * blockDim.x + threadIdx.x;
  if (rhs >= nrhs) return;
  if (active && !active[rhs]) return;
  givens_column(H, hcol, hrhs, cs, sn, g, j, ldg, resid, rhs);
}

__global__ void backsolve_kernel(const double2* H, int hcol, int hrhs, const double2* g, int ldg, double2* y,
                                 int k, int nrhs, const int* kvec) {
  const int rhs = blockIdx.x * blockDim.x + threadIdx.x;
  if (rhs >= nrhs) return;
  const int kk = kvec ? kvec[rhs] : k;
  const double2* h = H + (int64_t)rhs * hrhs;
  const double2* gg = g + (int64_t)rhs * ldg;
  double2* yy = y + (int64_t)rhs * ldg;
  for (int i = kk - 1; i >= 0; --i) {
    double2 s = gg[i];
    for (int l = i + 1; l < kk; ++l) cfms(s, h[(int64_t)l * hcol + i], yy[l]);
    yy[i] = cdiv(s, h[(int64_t)i * hcol + i]);
  }
  for (int i = kk; i < ldg; ++i) yy[i] = cmake<double2>(0, 0);
}

// u = Z y, or u += Z y with accumulate (a restarted cycle adds its correction).
__global__ void combine_kernel(const double2* __restrict__ Z, int64_t zstride, int nvec, const double2* __restrict__ y,
                               int ldy, double2* __restrict__ u, int64_t N, const int* kvec, int accumulate) {
  const int rhs = blockIdx.y;
  __shared__ double2 ys[kMaxVec];
  const int kk = kvec ? kvec[rhs] : nvec;
  for (int i = threadIdx.x; i < kk; i += blockDim.x) ys[i] = y[(int64_t)rhs * ldy + i];
  __syncthreads();
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= N) return;
  double2 acc = cmake<double2>(0, 0);
  for (int i = 0; i < kk; ++i) cfma(acc, Z[(int64_t)i * zstride + rhs * N + e], ys[i]);
  u[rhs * N + e] = accumulate ? cadd(u[rhs * N + e], acc) : acc;
}

__global__ void sub_kernel(const double2* a, const double2* b, double2* out, int64_t count) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < count) out[e] = csub(a[e], b[e]);
}

__global__ void init_g_kernel(const double* norms, int nrhs, double2* gvec, int ldg) {
  const int rhs = blockIdx.x * blockDim.x + threadIdx.x;
  if (rhs >= nrhs) return;
  for (int i = 0; i < ldg; ++i) gvec[(int64_t)rhs * ldg + i] = cmake<double2>(0, 0);
  gvec[(int64_t)rhs * ldg] = cmake<double2>(norms[rhs], 0.0);
}

// dst + j * dst_jstride = src + j * src_jstride (count complex values), j = *dj.
__global__ void copy_j_kernel(const double2* __restrict__ src, int64_t src_jstride, double2* __restrict__ dst,
                              int64_t dst_jstride, int64_t count, const int* dj) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= count) return;
  const int j = *dj;
  dst[j * dst_jstride + e] = src[j * src_jstride + e];
}

__global__ void set_counter_kernel(int* c, int value, int add) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c = add ? *c + value : value;
}

int dot_blocks(int64_t N) { return (int)ceil_div(N, (int64_t)kThreads * kPerThread); }

}  // namespace

int64_t kr_dot_slots(int64_t N) { return (int64_t)dot_blocks(N) * (kThreads / 64); }

void kr_dots(hipStream_t st, const double2* V, int64_t vstride, int nvec, const double2* w, int nrhs, int64_t N,
             double2* partial, double2* h_out, int hstride, int accumulate, double2* h_acc, int acc_stride,
             const int* dj, int64_t h_jstride, int64_t acc_jstride) {
  if (nvec > kMaxVec) throw Error(-7, "Krylov dimension exceeds the kernel limit");
  const int nblk = dot_blocks(N);
  dots_partial_kernel<<<dim3(nblk, nrhs), kThreads, 0, st>>>(V, vstride, nvec, w, N, partial, dj);
  SPP_LAUNCH_CHECK();
  const int nslot = (int)kr_dot_slots(N);
  dots_final_kernel<<<dim3(ceil_div(nvec, 4), nrhs), 256, 0, st>>>(partial, nslot, nvec, h_out, hstride, accumulate,
                                                                       h_acc, acc_stride, dj, h_jstride, acc_jstride);
  SPP_LAUNCH_CHECK();
}

void kr_update(hipStream_t st, const double2* V, int64_t vstride, int nvec, double2* w, int nrhs, int64_t N,
               const double2* h, int hstride, const int* dj, int64_t h_jstride) {
  update_kernel<<<dim3(ceil_div(N, kThreads), nrhs), kThreads, 0, st>>>(V, vstride, nvec, w, N, h, hstride, dj,
                                                                         h_jstride);
  SPP_LAUNCH_CHECK();
}

void kr_cgs2_second(hipStream_t st, const double2* V, int64_t vstride, int nvec, double2* w, int nrhs, int64_t N,
                    const double2* h1, int h1stride, double2* dpart, double2* h2, int h2stride, double2* h_acc,
                    int acc_stride, double* npart) {
  if (nvec > kMaxVec) throw Error(-7, "Krylov dimension exceeds the kernel limit");
  const int nblk = dot_blocks(N);
  update_dots_kernel<<<dim3(nblk, nrhs), kThreads, 0, st>>>(V, vstride, nvec, w, N, h1, h1stride, dpart);
  SPP_LAUNCH_CHECK();
  const int nslot = (int)kr_dot_slots(N);
  dots_final_kernel<<<dim3(ceil_div(nvec, 4), nrhs), 256, 0, st>>>(dpart, nslot, nvec, h2, h2stride, 0, h_acc,
                                                                       acc_stride, nullptr, 0, 0);
  SPP_LAUNCH_CHECK();
  update_sumsq_kernel<<<dim3(kNormBlocks, nrhs), kThreads, 0, st>>>(V, vstride, nvec, w, N, h2, h2stride, npart);
  SPP_LAUNCH_CHECK();
}

void kr_normalize(hipStream_t st, const double2* w, double2* v, int nrhs, int64_t N, double* partial,
                  double2* h_sub, int hstride, const KrGivens& gv) {
  double* norms = partial + (int64_t)kNormBlocks * nrhs;
  norm_scale_kernel<<<dim3(ceil_div(N, kThreads), nrhs), kThreads, 0, st>>>(w, v, partial, kNormBlocks, norms, h_sub,
                                                                             hstride, N, nullptr, 0, 0, gv);
  SPP_LAUNCH_CHECK();
}

void kr_norms(hipStream_t st, const double2* v, int nrhs, int64_t N, double* partial, double* out) {
  const int nblk = 256;
  sumsq_partial_kernel<<<dim3(nblk, nrhs), kThreads, 0, st>>>(v, N, partial);
  SPP_LAUNCH_CHECK();
  sumsq_final_kernel<<<nrhs, 64, 0, st>>>(partial, nblk, nrhs, out, nullptr, 0, nullptr, 0);
  SPP_LAUNCH_CHECK();
}

// v = w / ||w|| and h_sub = ||w|| per right-hand side; norms kept in partial[0..nrhs).
void kr_norm_scale(hipStream_t st, const double2* w, double2* v, int nrhs, int64_t N, double* partial,
                   double2* h_sub, int hstride, const int* dj, int64_t v_jstride, int64_t h_jstride,
                   const KrGivens& gv) {
  const int nblk = kNormBlocks;
  double* norms = partial + (int64_t)nblk * nrhs;
  sumsq_partial_kernel<<<dim3(nblk, nrhs), kThreads, 0, st>>>(w, N, partial);
  SPP_LAUNCH_CHECK();
  norm_scale_kernel<<<dim3(ceil_div(N, kThreads), nrhs), kThreads, 0, st>>>(w, v, partial, nblk, norms, h_sub, hstride,
                                                                             N, dj, v_jstride, h_jstride, gv);
  SPP_LAUNCH_CHECK();
}

void kr_givens(hipStream_t st, double2* H, int hcol, int hrhs, double* cs, double2* sn, double2* g, int j, int nrhs,
               int ldg, double* resid, const int* active, const int* dj) {
  givens_kernel<<<ceil_div(nrhs, 64), 64, 0, st>>>(H, hcol, hrhs, cs, sn, g, j, nrhs, ldg, resid, active, dj);
  SPP_LAUNCH_CHECK();
}

void kr_backsolve(hipStream_t st, const double2* H, int hcol, int hrhs, const double2* g, int ldg, double2* y, int k,
                  int nrhs, const int* kvec) {
  backsolve_kernel<<<ceil_div(nrhs, 64), 64, 0, st>>>(H, hcol, hrhs, g, ldg, y, k, nrhs, kvec);
  SPP_LAUNCH_CHECK();
}

void kr_combine(hipStream_t st, const double2* Z, int64_t zstride, int nvec, const double2* y, int ldy, double2* u,
                int nrhs, int64_t N, const int* kvec, bool accumulate) {
  if (nvec > kMaxVec) throw Error(-7, "Krylov dimension exceeds the kernel limit");
  combine_kernel<<<dim3(ceil_div(N, kThreads), nrhs), kThreads, 0, st>>>(Z, zstride, nvec, y, ldy, u, N, kvec,
                                                                         accumulate ? 1 : 0);
  SPP_LAUNCH_CHECK();
}

void kr_sub(hipStream_t st, const double2* a, const double2* b, double2* out, int64_t count) {
  sub_kernel<<<ceil_div(count, kThreads), kThreads, 0, st>>>(a, b, out, count);
  SPP_LAUNCH_CHECK();
}

void kr_scale_init(hipStream_t st, const double2* g, double2* v0, const double* norms, int nrhs, int64_t N,
                   double2* gvec, int ldg) {
  scale_kernel<<<dim3(ceil_div(N, kThreads), nrhs), kThreads, 0, st>>>(g, v0, norms, N, nullptr, 0);
  SPP_LAUNCH_CHECK();
  init_g_kernel<<<ceil_div(nrhs, 64), 64, 0, st>>>(norms, nrhs, gvec, ldg);
  SPP_LAUNCH_CHECK();
}

void kr_copy_j(hipStream_t st, const double2* src, int64_t src_jstride, double2* dst, int64_t dst_jstride,
               int64_t count, const int* dj) {
  copy_j_kernel<<<ceil_div(count, kThreads), kThreads, 0, st>>>(src, src_jstride, dst, dst_jstride, count, dj);
  SPP_LAUNCH_CHECK();
}

void kr_set_counter(hipStream_t st, int* c, int value, bool add) {
  set_counter_kernel<<<1, 64, 0, st>>>(c, value, add ? 1 : 0);
  SPP_LAUNCH_CHECK();
}

}  // namespace spp
