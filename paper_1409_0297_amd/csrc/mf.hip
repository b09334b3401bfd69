// Multifrontal factorisation and substitution of P = Q + C q (Sections 2.2-2.3).
//
// Fronts are dense F x F column-major matrices in one arena, ordered pivots
// first.  Per nested-dissection level:
//   assemble   P(S, gamma(S)) = [I  -T_S] + C_S diag(q_gamma(S)) generated
//              on the fly from the per-type stencils, scattered into fronts;
//   extend-add the children's Schur complements, one child slot per launch
//              so that no two workgroups add into the same entry;
//   partial LU right-looking blocked LU of the first p columns with partial
//              pivoting restricted to the p fully-summed rows: panel kernel,
//              row-block triangular solve, and a complex trailing update on
//              MFMA (FP64 16x16x4 for complex128 fronts, FP32 16x16x4 for
//              complex64 fronts) that also forms the Schur complement;
//   inverses   L11^{-1} and U11^{-1} by blocked substitution on the identity
//              (same kernels), stored over the LU of the pivot block so that
//              every substitution step is a bandwidth-bound matrix-vector
//              product.
// The solve runs forward elimination leaves -> root (children's update
// vectors pulled by the parent) and back substitution root -> leaves.
#include "common.hpp"
#include "kernels.hpp"

namespace spp {

namespace {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename R> struct Acc;
template <> struct Acc<double> { using type = d4v; };
template <> struct Acc<float> { using type = f4v; };

__device__ inline d4v mfma16(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4v mfma16(float a, float b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// Row of the 16x16 output tile held by lane l in accumulator register r.
__device__ inline int mfma_row(double, int lane, int r) { return (lane >> 4) + 4 * r; }
__device__ inline int mfma_row(float, int lane, int r) { return 4 * (lane >> 4) + r; }

__device__ inline int anchor_point(const MfDev& mf, int anchor, const int* off) {
  int ac[3];
  int a = anchor;
  for (int i = mf.d - 1; i >= 0; --i) { ac[i] = a % mf.m; a /= mf.m; }
  int g = 0;
  for (int i = 0; i < mf.d; ++i) g = g * mf.n + (((ac[i] * mf.b + off[i]) % mf.n) + mf.n) % mf.n;
  return g;
}

// ------------------------------------------------------------------ assembly
template <typename R>
__global__ void assemble_kernel(MfDev mf, cplx_t<R>* __restrict__ arena, int blk0) {
  using C = cplx_t<R>;
  const AsmBlockDev B = mf.blocks[blk0 + blockIdx.x];
  const FrontDev f = mf.fronts[B.front];
  const TypeDev T = mf.types[B.type];
  C* A = arena + f.off;
  const int total = T.nS * T.nG;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int i = t / T.nG, j = t - i * T.nG;
    const int rp = mf.pos[B.rowpos + i];
    const int cp = mf.pos[B.colpos + j];
    if (rp < 0 || cp < 0) continue;
    const int g = anchor_point(mf, B.anchor, T.off + j * mf.d);
    double2 v = cscale(T.C[i * T.nG + j], mf.q[g]);
    if (j < T.nS) {
      if (j == i) v.x += 1.0;
    } else {
      v = csub(v, T.T[i * T.nB + (j - T.nS)]);
    }
    C& dst = A[(int64_t)cp * f.F + rp];
    dst = cadd(dst, cconvert<C>(v));
  }
}

// ------------------------------------------------------------------ extend-add
template <typename R>
__global__ void extend_add_kernel(MfDev mf, cplx_t<R>* __restrict__ arena, int f0, int slot, int cols_per_wg) {
  using C = cplx_t<R>;
  const FrontDev par = mf.fronts[f0 + blockIdx.y];
  if (slot >= par.nchild) return;
  const FrontDev ch = mf.fronts[par.child[slot]];
  const int K = ch.F - ch.p;
  const int* map = mf.map + ch.map;
  const C* S = arena + ch.off;
  C* A = arena + par.off;
  const int j0 = blockIdx.x * cols_per_wg;
  for (int jj = 0; jj < cols_per_wg; ++jj) {
    const int j = j0 + jj;
    if (j >= K) return;
    const int64_t pc = (int64_t)map[j] * par.F;
    const C* src = S + (int64_t)(ch.p + j) * ch.F + ch.p;
    for (int i = threadIdx.x; i < K; i += blockDim.x) {
      C& d = A[pc + map[i]];
      d = cadd(d, src[i]);
    }
  }
}

// ------------------------------------------------------------------ panel LU
template <typename R>
__global__ void __launch_bounds__(256) panel_kernel(MfDev mf, cplx_t<R>* __restrict__ arena, int* __restrict__ ipiv,
                                                     int f0, int k0, int nb, int front_base) {
  using C = cplx_t<R>;
  const int fi = f0 + blockIdx.x;
  const FrontDev f = mf.fronts[fi];
  if (k0 >= f.p) return;
  const int kb = min(nb, f.p - k0);
  const int F = f.F;
  C* A = arena + f.off;
  __shared__ R sval[256];
  __shared__ int sidx[256];
  for (int j = k0; j < k0 + kb; ++j) {
    R best = -1;
    int bi = j;
    for (int r = j + threadIdx.x; r < f.p; r += blockDim.x) {
      const R v = cabs2(A[(int64_t)j * F + r]);
      if (v > best) { best = v; bi = r; }
    }
    sval[threadIdx.x] = best;
    sidx[threadIdx.x] = bi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) {
        const R o = sval[threadIdx.x + s];
        const int oi = sidx[threadIdx.x + s];
        if (o > sval[threadIdx.x] || (o == sval[threadIdx.x] && oi < sidx[threadIdx.x])) {
          sval[threadIdx.x] = o;
          sidx[threadIdx.x] = oi;
        }
      }
      __syncthreads();
    }
    const int piv = sidx[0];
    const bool ok = sval[0] > R(0) && isfinite(sval[0]);
    if (threadIdx.x == 0) {
      ipiv[f.perm + j] = piv;
      if (!ok) atomicCAS(mf.info, 0, front_base + fi + 1);
    }
    if (piv != j) {
      for (int c = threadIdx.x; c < F; c += blockDim.x) {
        C a = A[(int64_t)c * F + j];
        A[(int64_t)c * F + j] = A[(int64_t)c * F + piv];
        A[(int64_t)c * F + piv] = a;
      }
    }
    __syncthreads();
    const C inv = ok ? crecip(A[(int64_t)j * F + j]) : cmake<C>(0, 0);
    for (int r = j + 1 + threadIdx.x; r < F; r += blockDim.x)
      A[(int64_t)j * F + r] = cmul(A[(int64_t)j * F + r], inv);
    __syncthreads();
    const int rows = F - j - 1, cols = k0 + kb - j - 1;
    for (int t = threadIdx.x; t < rows * cols; t += blockDim.x) {
      const int r = j + 1 + t % rows, c = j + 1 + t / rows;
      cfms(A[(int64_t)c * F + r], A[(int64_t)j * F + r], A[(int64_t)c * F + j]);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ row-block TRSM
// mode 0: LU row block  front[k0:k0+kb, k0+kb:F] = L_kk^{-1} (.)
// mode 1: L inverse     XL[k0:k0+kb, 0:k0+kb]    = L_kk^{-1} (.)
// mode 2: U inverse     XU[k0:k0+kb, k0:p]       = U_kk^{-1} (.)   (k0 counted from the last block)
constexpr int kTrsmMaxB = 32;

template <typename R>
__device__ inline bool step_range(const FrontDev& f, int mode, int step, int nb, int& k0, int& kb) {
  if (mode == 2) {
    const int nblk = (f.p + nb - 1) / nb;
    const int blk = nblk - 1 - step;
    if (blk < 0) return false;
    k0 = blk * nb;
  } else {
    k0 = step * nb;
    if (k0 >= f.p) return false;
  }
  kb = min(nb, f.p - k0);
  return true;
}

template <typename R>
__global__ void __launch_bounds__(256) trsm_kernel(MfDev mf, cplx_t<R>* __restrict__ arena, cplx_t<R>* __restrict__ xwork,
                                                   int f0, int step, int nb, int mode) {
  using C = cplx_t<R>;
  const FrontDev f = mf.fronts[f0 + blockIdx.y];
  int k0, kb;
  if (!step_range<R>(f, mode, step, nb, k0, kb)) return;
  const int F = f.F, p = f.p;
  const C* A = arena + f.off;
  C* X;
  int ld, c0, c1;
  if (mode == 0) { X = arena + f.off; ld = F; c0 = k0 + kb; c1 = F; }
  else if (mode == 1) { X = xwork + f.xoff; ld = p; c0 = 0; c1 = k0 + kb; }
  else { X = xwork + f.xoff + (int64_t)p * p; ld = p; c0 = k0; c1 = p; }
  __shared__ C Tb[kTrsmMaxB * kTrsmMaxB];
  for (int t = threadIdx.x; t < kb * kb; t += blockDim.x) {
    const int i = t % kb, j = t / kb;
    Tb[i * kTrsmMaxB + j] = A[(int64_t)(k0 + j) * F + (k0 + i)];
  }
  __syncthreads();
  const int col = c0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= c1) return;
  C x[kTrsmMaxB];
  C* xc = X + (int64_t)col * ld + k0;
#pragma unroll
  for (int i = 0; i < kTrsmMaxB; ++i) x[i] = (i < kb) ? xc[i] : cmake<C>(0, 0);
  if (mode != 2) {
#pragma unroll
    for (int i = 1; i < kTrsmMaxB; ++i) {
      if (i < kb) {
        C s = x[i];
#pragma unroll
        for (int j = 0; j < kTrsmMaxB; ++j)
          if (j < i) cfms(s, Tb[i * kTrsmMaxB + j], x[j]);
        x[i] = s;
      }
    }
  } else {
#pragma unroll
    for (int i = kTrsmMaxB - 1; i >= 0; --i) {
      if (i < kb) {
        C s = x[i];
#pragma unroll
        for (int j = 0; j < kTrsmMaxB; ++j)
          if (j > i && j < kb) cfms(s, Tb[i * kTrsmMaxB + j], x[j]);
        const C dd = Tb[i * kTrsmMaxB + i];
        x[i] = (cabs2(dd) > R(0)) ? cdiv(s, dd) : cmake<C>(0, 0);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kTrsmMaxB; ++i)
    if (i < kb) xc[i] = x[i];
}

// ------------------------------------------------------------------ MFMA GEMM
// C -= A B for one 64 x 64 tile per workgroup; complex operands, column-major.
// mode 0: LU trailing update / Schur complement
// mode 1: L inverse update   XL[k0+kb:p, 0:k0+kb] -= L[k0+kb:p, k0:k0+kb] XL[k0:k0+kb, 0:k0+kb]
// mode 2: U inverse update   XU[0:k0, k0:p]       -= U[0:k0, k0:k0+kb]    XU[k0:k0+kb, k0:p]
constexpr int kBM = 64, kBN = 64, kBK = 16;

template <typename R>
__global__ void __launch_bounds__(256) gemm_kernel(MfDev mf, cplx_t<R>* __restrict__ arena, cplx_t<R>* __restrict__ xwork,
                                                   int f0, int step, int nb, int mode, int tiles_m) {
  using C = cplx_t<R>;
  using V = typename Acc<R>::type;
  const FrontDev f = mf.fronts[f0 + blockIdx.y];
  int k0, kb;
  if (!step_range<R>(f, mode, step, nb, k0, kb)) return;
  const int F = f.F, p = f.p;
  C* base = arena + f.off;
  const C *Ap, *Bp;
  C* Cp;
  int m, n, k, lda, ldb, ldc;
  if (mode == 0) {
    m = n = F - k0 - kb; k = kb;
    Ap = base + (int64_t)k0 * F + (k0 + kb); lda = F;
    Bp = base + (int64_t)(k0 + kb) * F + k0; ldb = F;
    Cp = base + (int64_t)(k0 + kb) * F + (k0 + kb); ldc = F;
  } else if (mode == 1) {
    C* XL = xwork + f.xoff;
    m = p - k0 - kb; n = k0 + kb; k = kb;
    Ap = base + (int64_t)k0 * F + (k0 + kb); lda = F;
    Bp = XL + k0; ldb = p;
    Cp = XL + (k0 + kb); ldc = p;
  } else {
    C* XU = xwork + f.xoff + (int64_t)p * p;
    m = k0; n = p - k0; k = kb;
    Ap = base + (int64_t)k0 * F; lda = F;
    Bp = XU + (int64_t)k0 * p + k0; ldb = p;
    Cp = XU + (int64_t)k0 * p; ldc = p;
  }
  const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
  const int m0 = tm * kBM, n0 = tn * kBN;
  if (m <= 0 || n <= 0 || k <= 0 || m0 >= m || n0 >= n) return;

  __shared__ C As[kBK][kBM + 1];
  __shared__ C Bs[kBK][kBN + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  V rr[2][2], ii[2][2], ri[2][2], ir[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) { rr[a][b] = V{}; ii[a][b] = V{}; ri[a][b] = V{}; ir[a][b] = V{}; }

  for (int kk0 = 0; kk0 < k; kk0 += kBK) {
    for (int e = threadIdx.x; e < kBM * kBK; e += 256) {
      const int row = e % kBM, kk = e / kBM;
      const int gr = m0 + row, gk = kk0 + kk;
      As[kk][row] = (gr < m && gk < k) ? Ap[(int64_t)gk * lda + gr] : cmake<C>(0, 0);
    }
    for (int e = threadIdx.x; e < kBK * kBN; e += 256) {
      const int kk = e % kBK, col = e / kBK;
      const int gk = kk0 + kk, gc = n0 + col;
      Bs[kk][col] = (gk < k && gc < n) ? Bp[(int64_t)gc * ldb + gk] : cmake<C>(0, 0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 4) {
      C av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[kk + (lane >> 4)][wm + 16 * a + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Bs[kk + (lane >> 4)][wn + 16 * b + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          rr[a][b] = mfma16(av[a].x, bv[b].x, rr[a][b]);
          ii[a][b] = mfma16(av[a].y, bv[b].y, ii[a][b]);
          ri[a][b] = mfma16(av[a].x, bv[b].y, ri[a][b]);
          ir[a][b] = mfma16(av[a].y, bv[b].x, ir[a][b]);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + 16 * a + mfma_row(R(0), lane, r);
        const int col = n0 + wn + 16 * b + (lane & 15);
        if (row < m && col < n) {
          C& c = Cp[(int64_t)col * ldc + row];
          c.x -= rr[a][b][r] - ii[a][b][r];
          c.y -= ri[a][b][r] + ir[a][b][r];
        }
      }
}

// ------------------------------------------------------------------ inverse helpers
template <typename R>
__global__ void identity_kernel(MfDev mf, cplx_t<R>* __restrict__ xwork, int f0) {
  using C = cplx_t<R>;
  const FrontDev f = mf.fronts[f0 + blockIdx.y];
  const int64_t pp = (int64_t)f.p * f.p;
  C* X = xwork + f.xoff;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < pp; t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % f.p), j = (int)(t / f.p);
    const C v = cmake<C>(i == j ? 1 : 0, 0);
    X[t] = v;
    X[pp + t] = v;
  }
}

template <typename R>
__global__ void merge_inverse_kernel(MfDev mf, cplx_t<R>* __restrict__ arena, const cplx_t<R>* __restrict__ xwork, int f0) {
  using C = cplx_t<R>;
  const FrontDev f = mf.fronts[f0 + blockIdx.y];
  const int64_t pp = (int64_t)f.p * f.p;
  const C* X = xwork + f.xoff;
  C* A = arena + f.off;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < pp; t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % f.p), j = (int)(t / f.p);
    A[(int64_t)j * f.F + i] = (i > j) ? X[t] : X[pp + t];
  }
}

__global__ void perm_kernel(MfDev mf, const int* __restrict__ ipiv, int f0, int f1) {
  const int fi = f0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (fi >= f1) return;
  const FrontDev f = mf.fronts[fi];
  int* perm = mf.perm + f.perm;
  for (int i = 0; i < f.p; ++i) perm[i] = i;
  for (int j = 0; j < f.p; ++j) {
    const int r = ipiv[f.perm + j];
    const int t = perm[j]; perm[j] = perm[r]; perm[r] = t;
  }
}

// ------------------------------------------------------------------ Q apply
// (Q r)_S = r_S - T_S r_beta(S) for every set instance (Section 2.3).
__global__ void q_apply_kernel(MfDev mf, const double2* __restrict__ r, double2* __restrict__ y, int nrhs, int type) {
  const TypeDev T = mf.types[type];
  const int anchor = blockIdx.x;
  const int rhs = blockIdx.y;
  const double2* rr = r + (int64_t)rhs * mf.N;
  double2* yy = y + (int64_t)rhs * mf.N;
  extern __shared__ double2 rb[];
  for (int j = threadIdx.x; j < T.nB; j += blockDim.x)
    rb[j] = rr[anchor_point(mf, anchor, T.off + (T.nS + j) * mf.d)];
  __syncthreads();
  for (int i = threadIdx.x; i < T.nS; i += blockDim.x) {
    const int g = anchor_point(mf, anchor, T.off + i * mf.d);
    double2 s = rr[g];
    for (int j = 0; j < T.nB; ++j) cfms(s, T.Tt[(int64_t)j * T.nS + i], rb[j]);
    yy[g] = s;
  }
}

// ------------------------------------------------------------------ solve
// Vectors per front: w and z arenas, position-major, nrhs consecutive values.
template <typename R>
__global__ void fwd_gather_kernel(MfDev mf, cplx_t<R>* __restrict__ W, const cplx_t<R>* __restrict__ x, int nrhs, int f0) {
  using C = cplx_t<R>;
  const FrontDev f = mf.fronts[f0 + blockIdx.x];
  C* w = W + f.voff * nrhs;
  const int* idx = mf.idx + f.idx;
  for (int t = threadIdx.x; t < f.F * nrhs; t += blockDim.x) {
    const int i = t / nrhs, r = t - i * nrhs;
    w[t] = (i < f.p) ? x[(int64_t)r * mf.N + idx[i]] : cmake<C>(0, 0);
  }
  __syncthreads();
  for (int c = 0; c < f.nchild; ++c) {
    const FrontDev ch = mf.fronts[f.child[c]];
    const int K = ch.F - ch.p;
    const int* map = mf.map + ch.map;
    const C* wc = W + (ch.voff + ch.p) * nrhs;
    for (int t = threadIdx.x; t < K * nrhs; t += blockDim.x) {
      const int i = t / nrhs, r = t - i * nrhs;
      C& d = w[map[i] * nrhs + r];
      d = cadd(d, wc[t]);
    }
    __syncthreads();
  }
}

// Row-tiled complex GEMV for the four substitution products.
//  mode 0: z = Linv (P w_piv)            rows [0,p),  cols j < row (+ unit diagonal)
//  mode 1: w_bnd -= L21 z                rows [0,F-p), cols [0,p)
//  mode 2: z -= U12 x(bnd)               rows [0,p),  cols [0,F-p)
//  mode 3: x(piv) = Uinv z               rows [0,p),  cols j >= row
template <typename R, int NR>
__global__ void __launch_bounds__(256) gemv_kernel(MfDev mf, const cplx_t<R>* __restrict__ arena, cplx_t<R>* __restrict__ W,
                                                   cplx_t<R>* __restrict__ Z, cplx_t<R>* __restrict__ xout, int nrhs,
                                                   int r0, int f0, int mode) {
  using C = cplx_t<R>;
  const FrontDev f = mf.fronts[f0 + blockIdx.y];
  const int F = f.F, p = f.p;
  const int nrows = (mode == 1) ? F - p : p;
  const int row0 = blockIdx.x * 64;
  if (row0 >= nrows) return;
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int row = row0 + lane;
  const C* A = arena + f.off;
  const int* idx = mf.idx + f.idx;
  const int* perm = mf.perm + f.perm;
  C* w = W + f.voff * nrhs;
  C* z = Z + f.voff * nrhs;
  int jlo, jhi;
  if (mode == 0) { jlo = 0; jhi = min(p, row0 + 64); }
  else if (mode == 1) { jlo = 0; jhi = p; }
  else if (mode == 2) { jlo = 0; jhi = F - p; }
  else { jlo = row0; jhi = p; }
  C acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = cmake<C>(0, 0);
  const bool live = row < nrows;
  for (int j = jlo + grp; j < jhi; j += 4) {
    C a;
    bool use;
    if (mode == 0) { use = live && j < row; a = use ? A[(int64_t)j * F + row] : cmake<C>(0, 0); }
    else if (mode == 1) { use = live; a = use ? A[(int64_t)j * F + p + row] : cmake<C>(0, 0); }
    else if (mode == 2) { use = live; a = use ? A[(int64_t)(p + j) * F + row] : cmake<C>(0, 0); }
    else { use = live && j >= row; a = use ? A[(int64_t)j * F + row] : cmake<C>(0, 0); }
    if (!use) continue;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (r0 + r >= nrhs) break;
      C v;
      if (mode == 0) v = w[perm[j] * nrhs + r0 + r];
      else if (mode == 1) v = z[j * nrhs + r0 + r];
      else if (mode == 2) v = xout[(int64_t)(r0 + r) * mf.N + idx[p + j]];
      else v = z[j * nrhs + r0 + r];
      cfma(acc[r], a, v);
    }
  }
  __shared__ C red[4][64][NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) red[grp][lane][r] = acc[r];
  __syncthreads();
  if (grp != 0 || !live) return;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r0 + r >= nrhs) break;
    C s = cadd(cadd(red[0][lane][r], red[1][lane][r]), cadd(red[2][lane][r], red[3][lane][r]));
    const int rr = r0 + r;
    if (mode == 0) {
      z[row * nrhs + rr] = cadd(s, w[perm[row] * nrhs + rr]);
    } else if (mode == 1) {
      C& d = w[(p + row) * nrhs + rr];
      d = csub(d, s);
    } else if (mode == 2) {
      C& d = z[row * nrhs + rr];
      d = csub(d, s);
    } else {
      xout[(int64_t)rr * mf.N + idx[row]] = s;
    }
  }
}

template <typename R>
__global__ void cast_kernel(const void* in, void* out, int64_t count, int to_double) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= count) return;
  if (to_double) static_cast<double2*>(out)[t] = cconvert<double2>(static_cast<const cplx_t<R>*>(in)[t]);
  else static_cast<cplx_t<R>*>(out)[t] = cconvert<cplx_t<R>>(static_cast<const double2*>(in)[t]);
}

constexpr int kNB = 32;

}  // namespace

template <typename R>
void mf_factor_level(hipStream_t st, const MfDev& mf, void* arena_v, void* xwork_v, int f0, int f1, int maxF,
                     int maxP, int blk0, int blk1, int max_children, int prev_f0) {
  using C = cplx_t<R>;
  (void)prev_f0;
  C* arena = static_cast<C*>(arena_v);
  C* xwork = static_cast<C*>(xwork_v);
  const int nf = f1 - f0;
  if (blk1 > blk0) {
    assemble_kernel<R><<<blk1 - blk0, 256, 0, st>>>(mf, arena, blk0);
    SPP_LAUNCH_CHECK();
  }
  for (int s = 0; s < max_children; ++s) {
    const int cols = 4;
    dim3 grid(ceil_div(maxF, cols), nf);
    extend_add_kernel<R><<<grid, 256, 0, st>>>(mf, arena, f0, s, cols);
    SPP_LAUNCH_CHECK();
  }
  const int steps = (maxP + kNB - 1) / kNB;
  const int tiles = (int)ceil_div(maxF, kBM);
  for (int s = 0; s < steps; ++s) {
    panel_kernel<R><<<nf, 256, 0, st>>>(mf, arena, mf.ipiv, f0, s * kNB, kNB, 0);
    SPP_LAUNCH_CHECK();
    trsm_kernel<R><<<dim3(ceil_div(maxF, 256), nf), 256, 0, st>>>(mf, arena, xwork, f0, s, kNB, 0);
    SPP_LAUNCH_CHECK();
    gemm_kernel<R><<<dim3(tiles * tiles, nf), 256, 0, st>>>(mf, arena, xwork, f0, s, kNB, 0, tiles);
    SPP_LAUNCH_CHECK();
  }
  (void)maxP;
  perm_kernel<<<ceil_div(nf, 64), 64, 0, st>>>(mf, mf.ipiv, f0, f1);
  SPP_LAUNCH_CHECK();
  // Inverses of L11 and U11.
  const int ptiles = (int)ceil_div(maxP, kBM);
  identity_kernel<R><<<dim3(ceil_div((int64_t)maxP * maxP, 256 * 4), nf), 256, 0, st>>>(mf, xwork, f0);
  SPP_LAUNCH_CHECK();
  for (int s = 0; s < steps; ++s) {
    trsm_kernel<R><<<dim3(ceil_div(maxP, 256), nf), 256, 0, st>>>(mf, arena, xwork, f0, s, kNB, 1);
    SPP_LAUNCH_CHECK();
    gemm_kernel<R><<<dim3(ptiles * ptiles, nf), 256, 0, st>>>(mf, arena, xwork, f0, s, kNB, 1, ptiles);
    SPP_LAUNCH_CHECK();
  }
  for (int s = 0; s < steps; ++s) {
    trsm_kernel<R><<<dim3(ceil_div(maxP, 256), nf), 256, 0, st>>>(mf, arena, xwork, f0, s, kNB, 2);
    SPP_LAUNCH_CHECK();
    gemm_kernel<R><<<dim3(ptiles * ptiles, nf), 256, 0, st>>>(mf, arena, xwork, f0, s, kNB, 2, ptiles);
    SPP_LAUNCH_CHECK();
  }
  merge_inverse_kernel<R><<<dim3(ceil_div((int64_t)maxP * maxP, 256 * 4), nf), 256, 0, st>>>(mf, arena, xwork, f0);
  SPP_LAUNCH_CHECK();
}

void q_apply(hipStream_t st, const MfDev& mf, const double2* r, double2* y, int nrhs) {
  const int ntypes = 1 << mf.d;
  const int anchors = (int)(mf.N / ((int64_t)mf.b * (mf.d == 3 ? (int64_t)mf.b * mf.b : mf.b)));
  for (int t = 0; t < ntypes; ++t) {
    q_apply_kernel<<<dim3(anchors, nrhs), 256, sizeof(double2) * mf.types[t].nB, st>>>(mf, r, y, nrhs, t);
    SPP_LAUNCH_CHECK();
  }
}

template <typename R>
void mf_solve(hipStream_t st, const MfDev& mf, const void* arena_v, void* w_v, void* z_v, const void* x_in,
              void* x_out, int nrhs, const int* level_begin, const int* level_maxF, const int* level_maxP,
              int nlevels) {
  using C = cplx_t<R>;
  const C* arena = static_cast<const C*>(arena_v);
  C* W = static_cast<C*>(w_v);
  C* Z = static_cast<C*>(z_v);
  const C* xin = static_cast<const C*>(x_in);
  C* xout = static_cast<C*>(x_out);
  auto gemv = [&](int f0, int nf, int rows, int mode) {
    dim3 grid(ceil_div(rows, 64), nf);
    int r0 = 0;
    while (r0 < nrhs) {
      if (nrhs - r0 >= 4) {
        gemv_kernel<R, 4><<<grid, 256, 0, st>>>(mf, arena, W, Z, xout, nrhs, r0, f0, mode);
        r0 += 4;
      } else {
        gemv_kernel<R, 1><<<grid, 256, 0, st>>>(mf, arena, W, Z, xout, nrhs, r0, f0, mode);
        r0 += 1;
      }
      SPP_LAUNCH_CHECK();
    }
  };
  for (int l = 0; l < nlevels; ++l) {
    const int f0 = level_begin[l], nf = level_begin[l + 1] - f0;
    fwd_gather_kernel<R><<<nf, 256, 0, st>>>(mf, W, xin, nrhs, f0);
    SPP_LAUNCH_CHECK();
    gemv(f0, nf, level_maxP[l], 0);
    gemv(f0, nf, level_maxF[l], 1);
  }
  for (int l = nlevels - 1; l >= 0; --l) {
    const int f0 = level_begin[l], nf = level_begin[l + 1] - f0;
    gemv(f0, nf, level_maxP[l], 2);
    gemv(f0, nf, level_maxP[l], 3);
  }
}

template <typename R>
void cast_vectors(hipStream_t st, const void* in, void* out, int64_t count, int to_double) {
  cast_kernel<R><<<ceil_div(count, 256), 256, 0, st>>>(in, out, count, to_double);
  SPP_LAUNCH_CHECK();
}

template void mf_factor_level<double>(hipStream_t, const MfDev&, void*, void*, int, int, int, int, int, int, int, int);
template void mf_factor_level<float>(hipStream_t, const MfDev&, void*, void*, int, int, int, int, int, int, int, int);
template void mf_solve<double>(hipStream_t, const MfDev&, const void*, void*, void*, const void*, void*, int,
                               const int*, const int*, const int*, int);
template void mf_solve<float>(hipStream_t, const MfDev&, const void*, void*, void*, const void*, void*, int,
                              const int*, const int*, const int*, int);
template void cast_vectors<double>(hipStream_t, const void*, void*, int64_t, int);
template void cast_vectors<float>(hipStream_t, const void*, void*, int64_t, int);

}  // namespace spp
