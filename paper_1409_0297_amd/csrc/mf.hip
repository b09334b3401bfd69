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
#include <algorithm>
#include <limits>
#include <type_traits>
#include <utility>

#include <hip/hip_cooperative_groups.h>

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

// Grid index of offset `off` from the corner of leaf box `anchor` of instance I.
__device__ inline int anchor_point(const InstDev& I, int anchor, const int* off) {
  int ac[3];
  int a = anchor;
  for (int i = I.d - 1; i >= 0; --i) { ac[i] = a % I.m; a /= I.m; }
  int g = 0;
  for (int i = 0; i < I.d; ++i) g = g * I.n + (((ac[i] * I.b + off[i]) % I.n) + I.n) % I.n;
  return g;
}

// ------------------------------------------------------------------ assembly
// with_norm (levels without children, where assembly writes every nonzero
// of a front exactly once): the largest |entry| written also goes to
// mf.fnorm, as front_norm_kernel would find it, so that pass is skipped.
template <typename R>
__global__ void __launch_bounds__(256) assemble_kernel(MfDev mf, cplx_t<R>* __restrict__ arena, int blk0,
                                                       int with_norm) {
  using C = cplx_t<R>;
  const AsmBlockDev B = mf.blocks[blk0 + blockIdx.x];
  const FrontDev f = mf.fronts[B.front];
  const InstDev& I = mf.inst[f.inst];
  const TypeDev& T = I.types[B.type];
  C* A = arena + f.off;
  // Column data of this block once per workgroup: front position and q at
  // every unknown of gamma(S) (q of its point: nc unknowns per point).
  __shared__ int cpos[1024];
  __shared__ double qg[1024];
  __shared__ int rpos[1024];
  for (int j = threadIdx.x; j < T.nG; j += blockDim.x) {
    cpos[j] = mf.pos[B.colpos + j];
    qg[j] = I.q[anchor_point(I, B.anchor, T.off + (j / I.nc) * I.d)];
  }
  for (int i = threadIdx.x; i < T.nS; i += blockDim.x) rpos[i] = mf.pos[B.rowpos + i];
  __syncthreads();
  // Consecutive threads take consecutive rows of one column: coalesced reads
  // of the transposed stencils and coalesced writes into the column-major front.
  const int total = T.nS * T.nG;
  R m2 = 0;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int j = t / T.nS, i = t - j * T.nS;
    const int rp = rpos[i], cp = cpos[j];
    if (rp < 0 || cp < 0) continue;
    double2 v = cscale(T.Ct[(int64_t)j * T.nS + i], qg[j]);
    if (j < T.nS) {
      if (j == i) v.x += 1.0;
    } else {
      v = csub(v, T.Tt[(int64_t)(j - T.nS) * T.nS + i]);
    }
    // Every row of P belongs to one set instance and every (row, column)
    // pair of a block is distinct, so each front entry is written by at most
    // one thread: a plain store (no read of the zeroed arena).
    const C c = cconvert<C>(v);
    A[(int64_t)cp * f.F + rp] = c;
    m2 = fmax(m2, cabs2(c));
  }
  if (!with_norm) return;
  float m = (float)sqrt((double)m2);
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  __shared__ float wmax[4];
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    atomicMax(mf.fnorm + B.front, __float_as_uint(fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]))));
}

// ------------------------------------------------------------------ extend-add
template <typename R>
__global__ void extend_add_kernel(MfDev mf, cplx_t<R>* __restrict__ arena, int f0, int slot, int cols_per_wg) {
  using C = cplx_t<R>;
  const FrontDev& par = mf.fronts[f0 + blockIdx.y];   // by reference: child[] indexed at run time
  if (slot >= par.nchild) return;
  const FrontDev& ch = mf.fronts[par.child[slot]];
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

// ------------------------------------------------------------------ front norm
// Largest |entry| of every front of a level as assembled (after the
// extend-add), as float bits in mf.fnorm (entries are >= 0, so the bit
// patterns order like the values).
template <typename R>
__global__ void __launch_bounds__(256) front_norm_kernel(MfDev mf, const cplx_t<R>* __restrict__ arena, int f0,
                                                         int64_t chunk) {
  // Workgroup (x, y): entries [x chunk, (x + 1) chunk) of front f0 + y, read
  // as one flat array (the front is F x F contiguous); four loads in flight
  // per thread, squared magnitudes compared, one atomic per workgroup.
  const int fi = f0 + blockIdx.y;
  const FrontDev& f = mf.fronts[fi];
  const int64_t n = (int64_t)f.F * f.F;
  const int64_t e0 = (int64_t)blockIdx.x * chunk;
  if (e0 >= n) return;
  const int64_t e1 = min(n, e0 + chunk);
  const cplx_t<R>* A = arena + f.off;
  R m0 = 0, m1 = 0, m2 = 0, m3 = 0;
  int64_t e = e0 + threadIdx.x;
  for (; e + 768 < e1; e += 1024) {
    const cplx_t<R> a = A[e], b = A[e + 256], c = A[e + 512], d = A[e + 768];
    m0 = fmax(m0, cabs2(a));
    m1 = fmax(m1, cabs2(b));
    m2 = fmax(m2, cabs2(c));
    m3 = fmax(m3, cabs2(d));
  }
  for (; e < e1; e += 256) m0 = fmax(m0, cabs2(A[e]));
  float m = (float)sqrt((double)fmax(fmax(m0, m1), fmax(m2, m3)));
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  __shared__ float wmax[4];
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    atomicMax(mf.fnorm + fi, __float_as_uint(fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]))));
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

// ------------------------------------------------------------------ register panel LU
// Factors the panel columns [k0, k0 + kb) over rows [k0, F) of one front per
// workgroup.  The panel is processed in sub-panels of 8 columns held in
// registers (thread t owns rows c0 + t + i NT); per column: argmax over the
// fully-summed rows by wave shuffles and one LDS round, the pivot row swap
// through LDS, then scaling and the rank-1 update entirely in registers (two
// barriers per column).  Interchanges are applied here only to the panel's own
// columns; laswp_kernel applies them to the rest of the front.  After each
// sub-panel the remaining panel columns receive its U rows and rank-8 update.
constexpr int kSW = 8;

template <typename R, int NT, int RPT>
__global__ void __launch_bounds__(NT) panel2_kernel(MfDev mf, cplx_t<R>* __restrict__ arena, int* __restrict__ ipiv,
                                                    int f0, int k0, int nb) {
  using C = cplx_t<R>;
  constexpr int NW = NT / 64;
  const int fi = f0 + blockIdx.x;
  const FrontDev f = mf.fronts[fi];
  if (k0 >= f.p) return;
  const int kb = min(nb, f.p - k0);
  const int F = f.F, p = f.p;
  C* A = arena + f.off;
  __shared__ R red_v[NW];
  __shared__ int red_i[NW];
  __shared__ C prow[kSW], jrow[kSW];
  __shared__ C Ub[kSW][64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  C a[RPT][kSW];
  for (int c0 = k0; c0 < k0 + kb; c0 += kSW) {
    const int sw = min(kSW, k0 + kb - c0);
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = c0 + tid + i * NT;
#pragma unroll
      for (int jj = 0; jj < kSW; ++jj)
        a[i][jj] = (r < F && jj < sw) ? A[(int64_t)(c0 + jj) * F + r] : cmake<C>(0, 0);
    }
#pragma unroll
    for (int jj = 0; jj < kSW; ++jj) {
      if (jj >= sw) break;   // sw is uniform over the workgroup
      const int j = c0 + jj;
      R best = -1;
      int bi = 0x7fffffff;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = c0 + tid + i * NT;
        if (r >= j && r < p) {
          const R v = cabs2(a[i][jj]);
          if (v > best) { best = v; bi = r; }
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const R ov = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
      }
      if (lane == 0) { red_v[wave] = best; red_i[wave] = bi; }
      __syncthreads();
      best = red_v[0];
      bi = red_i[0];
#pragma unroll
      for (int w = 1; w < NW; ++w) {
        const R ov = red_v[w];
        const int oi = red_i[w];
        if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
      }
      const bool ok = best > R(0) && isfinite(best);
      const int piv = ok ? bi : j;
      const int tp = (piv - c0) % NT, ip = (piv - c0) / NT;
      const int tj = (j - c0) % NT, ij = (j - c0) / NT;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        if (tid == tp && i == ip)
#pragma unroll
          for (int x = 0; x < kSW; ++x) prow[x] = a[i][x];
        if (tid == tj && i == ij)
#pragma unroll
          for (int x = 0; x < kSW; ++x) jrow[x] = a[i][x];
      }
      if (piv != j) {
        // Other columns of this outer panel (outside the register sub-panel).
        for (int c = tid; c < kb - sw; c += NT) {
          const int col = (c < c0 - k0) ? k0 + c : c0 + sw + (c - (c0 - k0));
          C* cp = A + (int64_t)col * F;
          const C t = cp[j]; cp[j] = cp[piv]; cp[piv] = t;
        }
      }
      if (tid == 0) {
        ipiv[f.perm + j] = piv;
        if (!ok) atomicCAS(mf.info, 0, fi + 1);
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        if (tid == tj && i == ij)
#pragma unroll
          for (int x = 0; x < kSW; ++x) a[i][x] = prow[x];
        if (piv != j && tid == tp && i == ip)
#pragma unroll
          for (int x = 0; x < kSW; ++x) a[i][x] = jrow[x];
      }
      const C inv = ok ? crecip(prow[jj]) : cmake<C>(0, 0);
      C pr[kSW];
#pragma unroll
      for (int x = 0; x < kSW; ++x) pr[x] = prow[x];
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = c0 + tid + i * NT;
        if (r > j && r < F) {
          C l;
#pragma unroll
          for (int x = 0; x < kSW; ++x) {
            if (x == jj) { l = cmul(a[i][x], inv); a[i][x] = l; }
          }
#pragma unroll
          for (int x = 0; x < kSW; ++x)
            if (x > jj && x < sw) cfms(a[i][x], l, pr[x]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = c0 + tid + i * NT;
      if (r < F)
#pragma unroll
        for (int jj = 0; jj < kSW; ++jj)
          if (jj < sw) A[(int64_t)(c0 + jj) * F + r] = a[i][jj];
    }
    __syncthreads();
    const int rw = k0 + kb - (c0 + sw);
    if (rw > 0) {
      // U rows of this sub-panel for the remaining panel columns.
      for (int c = tid; c < rw; c += NT) {
        C* cp = A + (int64_t)(c0 + sw + c) * F + c0;
        C x[kSW];
#pragma unroll
        for (int jj = 0; jj < kSW; ++jj) x[jj] = (jj < sw) ? cp[jj] : cmake<C>(0, 0);
#pragma unroll
        for (int jj = 1; jj < kSW; ++jj)
#pragma unroll
          for (int l = 0; l < kSW; ++l)
            if (l < jj && jj < sw) cfms(x[jj], A[(int64_t)(c0 + l) * F + c0 + jj], x[l]);
#pragma unroll
        for (int jj = 0; jj < kSW; ++jj)
          if (jj < sw) { cp[jj] = x[jj]; Ub[jj][c] = x[jj]; }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = c0 + tid + i * NT;
        if (r >= c0 + sw && r < F) {
          for (int c = 0; c < rw; ++c) {
            C& d = A[(int64_t)(c0 + sw + c) * F + r];
            C s = d;
#pragma unroll
            for (int jj = 0; jj < kSW; ++jj)
              if (jj < sw) cfms(s, a[i][jj], Ub[jj][c]);
            d = s;
          }
        }
      }
      __syncthreads();
    }
  }
}

// Applies the interchanges of panel [k0, k0 + kb) to the columns outside it:
// the net permutation of the touched rows is built once per workgroup, then
// every column gathers its touched rows and scatters them back.
template <typename R>
__global__ void __launch_bounds__(64) laswp_kernel(MfDev mf, cplx_t<R>* __restrict__ arena, const int* __restrict__ ipiv,
                                                   int f0, int k0, int nb) {
  using C = cplx_t<R>;
  const FrontDev f = mf.fronts[f0 + blockIdx.y];
  if (k0 >= f.p) return;
  const int kb = min(nb, f.p - k0);
  __shared__ int rows[128], lab[128], cnt;
  __shared__ C tmp[64][65];
  if (threadIdx.x == 0) {
    int n = 0;
    for (int j = k0; j < k0 + kb; ++j) {
      const int pv = ipiv[f.perm + j];
      if (pv == j) continue;
      int a = -1, b = -1;
      for (int x = 0; x < n; ++x) { if (rows[x] == j) a = x; if (rows[x] == pv) b = x; }
      if (a < 0) { rows[n] = j; lab[n] = j; a = n++; }
      if (b < 0) { rows[n] = pv; lab[n] = pv; b = n++; }
      const int t = lab[a]; lab[a] = lab[b]; lab[b] = t;
    }
    int m = 0;
    for (int x = 0; x < n; ++x)
      if (lab[x] != rows[x]) { rows[m] = rows[x]; lab[m] = lab[x]; ++m; }
    cnt = m;
  }
  __syncthreads();
  const int n = cnt;   // at most 2 kb <= 64 touched rows (nb <= 32)
  if (n == 0 || n > 64) return;
  const int col = blockIdx.x * 64 + threadIdx.x;
  if (col >= f.F || (col >= k0 && col < k0 + kb)) return;
  C* cp = arena + f.off + (int64_t)col * f.F;
  for (int x = 0; x < n; ++x) tmp[threadIdx.x][x] = cp[lab[x]];
  for (int x = 0; x < n; ++x) cp[rows[x]] = tmp[threadIdx.x][x];
}

// ------------------------------------------------------------------ block-local pivoting LU
// Default factorisation step (block-local pivoting): the pivot of column j is
// the largest-modulus entry among the rows of the current kb x kb diagonal
// block (kb <= 32), so the pivot search and elimination of a step stay in one
// workgroup.  The block's L and U are written back, their inverses
// Linv_kk, Uinv_kk (kb x kb, column-major) go to dinv, and the other two
// products of the step become dense, dependency-free MFMA multiplications:
// L21 = A21 Uinv_kk and U12 = Linv_kk P A12 (gemm_kernel mode 7).
constexpr int kDB = 32;

template <typename R>
struct DiagLds {
  cplx_t<R> D[kDB][kDB + 1];    // the block to factor
  cplx_t<R> Lm[kDB][kDB + 1];   // the previous step's L part (rows of this block)
  cplx_t<R> X[kDB][kDB + 1];    // the LU in pivot order
  int rsel[kDB];                // pivot row of each step
  int kofr[kDB];                // pivot index of each row of the previous block
};

// Lane exchanges of one wave: the value of a uniform lane (a scalar read),
// and rotation by N lanes inside each row of 16 lanes (DPP).
__device__ inline float lane_read(float x, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), src));
}
__device__ inline double lane_read(double x, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), src);
  return __hiloint2double(hi, lo);
}
template <int N> __device__ inline double row_ror(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x120 + N, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x120 + N, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// c ? x : y on the components (a select of whole vector structs goes through
// their addresses and keeps register arrays in memory).
template <typename C> __device__ inline C csel(bool c, C x, C y) {
  return cmake<C>(c ? x.x : y.x, c ? x.y : y.y);
}
template <typename C> __device__ inline C lane_read(C x, int src) {
  return cmake<C>(lane_read(x.x, src), lane_read(x.y, src));
}

// Bitwise equality of two values (true for two NaNs with the same bits).
__device__ __forceinline__ bool memcmp_eq(float a, float b) { return __float_as_int(a) == __float_as_int(b); }
__device__ __forceinline__ bool memcmp_eq(double a, double b) {
  return __double_as_longlong(a) == __double_as_longlong(b);
}

// a -= m * b as four fused multiply-adds (the negations are operand modifiers).
template <typename C> __device__ __forceinline__ void cfms4(C& a, C m, C b) {
  a.x = fma(-m.x, b.x, a.x);
  a.x = fma(m.y, b.y, a.x);
  a.y = fma(-m.x, b.y, a.y);
  a.y = fma(-m.y, b.x, a.y);
}
// 1 / x for x > 0, else 0 (the single-precision reciprocal instruction is
// accurate to 1 ulp, enough for a pivot's reciprocal).
__device__ __forceinline__ float pos_recip(float x) { return x > 0.f ? __builtin_amdgcn_rcpf(x) : 0.f; }
__device__ __forceinline__ double pos_recip(double x) { return x > 0.0 ? 1.0 / x : 0.0; }

// Largest |d|^2 over the 32 rows of the wave (lanes r and r + 32 hold row r;
// rows already used as pivots carry -1).  In single precision the bit
// patterns are compared as integers: they order like the values for x >= 0,
// -1 is below all of them, and a NaN is above every number, so a NaN entry
// is the one chosen (and then reported).
// (B = 32: the same over lanes 32 .. 63.)
template <int B = 0>
__device__ __forceinline__ float rows_max(float v) {
  int m = __float_as_int(v);
  m = max(m, __builtin_amdgcn_update_dpp(0, m, 0x121, 0xF, 0xF, false));
  m = max(m, __builtin_amdgcn_update_dpp(0, m, 0x122, 0xF, 0xF, false));
  m = max(m, __builtin_amdgcn_update_dpp(0, m, 0x124, 0xF, 0xF, false));
  m = max(m, __builtin_amdgcn_update_dpp(0, m, 0x128, 0xF, 0xF, false));
  return __int_as_float(max(__builtin_amdgcn_readlane(m, B), __builtin_amdgcn_readlane(m, B + 16)));
}
template <int B = 0>
__device__ __forceinline__ double rows_max(double v) {
  auto mx = [](double a, double b) { return (a > b || a != a) ? a : b; };
  v = mx(v, row_ror<1>(v));
  v = mx(v, row_ror<2>(v));
  v = mx(v, row_ror<4>(v));
  v = mx(v, row_ror<8>(v));
  return mx(lane_read(v, B), lane_read(v, B + 16));
}

// Value of lane src for each lane (src may differ between lanes; through
// the LDS crossbar, no LDS memory).
__device__ inline float lane_gather(float x, int src) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(x)));
}
__device__ inline double lane_gather(double x, int src) {
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, __double2loint(x));
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, __double2hiint(x));
  return __hiloint2double(hi, lo);
}
template <typename C> __device__ inline C lane_gather(C x, int src) {
  return cmake<C>(lane_gather(x.x, src), lane_gather(x.y, src));
}

// One wave factors the 32 x 32 block (wave_lu32): lane r holds columns
// 0, 2, .. 30 of row r and lane r + 32 columns 1, 3, .. 31 of the same row,
// slot q of a lane being column 2 q + h (h = lane / 32).
//
// Slot Q of step J: a_Q -= l * (pivot row)_Q on the columns right of J.  The
// slot of column J + 1, which the next pivot search waits for, reads the
// pivot row's entries by scalar reads; the others by lane gathers, all of
// a step's gathers issued before the first of its products (wave_lu_fetch),
// so that their latencies overlap.
template <typename R, int J, int Q>
__device__ __forceinline__ void wave_lu_fetch(cplx_t<R> (&g)[kDB / 2], const cplx_t<R> (&a)[kDB / 2], int src) {
  if constexpr (2 * Q + 1 > J && Q != (J + 1) / 2) g[Q] = lane_gather(a[Q], src);
}
template <typename R, int J, int Q>
__device__ __forceinline__ void wave_lu_slot(cplx_t<R> (&a)[kDB / 2], const cplx_t<R> (&g)[kDB / 2], cplx_t<R> l,
                                             int rp, bool hi) {
  using C = cplx_t<R>;
  if constexpr (2 * Q + 1 > J) {
    C pv;
    if constexpr (Q == (J + 1) / 2) {
      if constexpr (2 * Q == J) pv = lane_read(a[Q], rp + 32);   // (only column 2 Q + 1 = J + 1 moves)
      else pv = csel(hi, lane_read(a[Q], rp + 32), lane_read(a[Q], rp));
    } else {
      pv = g[Q];
    }
    C t = a[Q];
    cfms4(t, l, pv);
    a[Q] = (2 * Q == J) ? csel(hi, t, a[Q]) : t;
  }
}

// Step J: the remaining row of largest |d_rJ|^2 becomes the pivot (exact
// ties to the lowest row, a NaN maximum matches itself); every other
// remaining row keeps its multiplier in column J and eliminates column J
// from its columns right of J.  Column J sits in the half H = J % 2; the
// other half takes each row's d_rJ by a lane gather (during the search) and
// forms the same multiplier.
template <typename R, int J, int... Q>
__device__ __forceinline__ void wave_lu_step(std::integer_sequence<int, Q...>, cplx_t<R> (&a)[kDB / 2], int r,
                                             bool hi, int kb, bool& done, bool& bad, int& mystep) {
  using C = cplx_t<R>;
  constexpr int H = J & 1, QJ = J >> 1;
  const bool mine = hi == (H == 1);
  const C dj = a[QJ];
  const C drj = lane_gather(dj, r + 32 * H);   // d_rJ in both halves
  const R v2 = (done || !mine) ? R(-1) : cabs2(dj);
  const R m = rows_max<32 * H>(v2);
  const unsigned hit = (unsigned)(__builtin_amdgcn_ballot_w64(mine && !done && memcmp_eq(v2, m)) >> (32 * H));
  const unsigned live = (unsigned)(__builtin_amdgcn_ballot_w64(mine && !done) >> (32 * H));
  const int rp = __builtin_ctz(hit ? hit : live);
  bad = bad | ((J < kb) & !(m > R(0) && m <= std::numeric_limits<R>::max()));
  const C pv = lane_read(dj, rp + 32 * H);
  const R inv = pos_recip(cabs2(pv));
  const bool upd = !done && r != rp;
  const C l = cmul(drj, cmake<C>(pv.x * inv, -pv.y * inv));
  const C le = csel(upd, l, cmake<C>(0, 0));
  if (mine) a[QJ] = csel(upd, l, a[QJ]);
  mystep = r == rp ? J : mystep;
  done = done || r == rp;
  C g[kDB / 2];
  (wave_lu_fetch<R, J, Q>(g, a, rp + (hi ? 32 : 0)), ...);
  (wave_lu_slot<R, J, Q>(a, g, le, rp, hi), ...);
}

template <typename R, int... J>
__device__ __forceinline__ void wave_lu_steps(std::integer_sequence<int, J...>, cplx_t<R> (&a)[kDB / 2], int r,
                                              bool hi, int kb, bool& done, bool& bad, int& mystep) {
  (wave_lu_step<R, J>(std::make_integer_sequence<int, kDB / 2>{}, a, r, hi, kb, done, bad, mystep), ...);
}

// LU with row pivoting of the 32 x 32 block S.D by the first wave of the
// workgroup alone (no barrier between steps).  Step j takes as pivot the
// remaining row of largest |d_rj|^2 and eliminates column j from the other
// remaining rows; each row keeps its multipliers in place, so the row chosen
// at step k ends as row k of the LU in pivot order: L left of column k, U
// from column k on.  Writes that LU to S.X and the chosen rows to S.rsel
// (the other waves go straight to the caller's barrier, after which both
// may be read); returns true in the first wave if a pivot among the first
// kb was zero or not finite.
template <typename R>
__device__ __forceinline__ bool wave_lu32(DiagLds<R>& S, int kb) {
  using C = cplx_t<R>;
  if (threadIdx.x >= 64) return false;
  const int lane = threadIdx.x, r = lane & 31;
  const bool hi = lane >= 32;
  C a[kDB / 2];
#pragma unroll
  for (int q = 0; q < kDB / 2; ++q) a[q] = S.D[r][2 * q + (hi ? 1 : 0)];
  bool done = false, bad = false;
  int mystep = 0;   // the step at which row r became the pivot
  wave_lu_steps<R>(std::make_integer_sequence<int, kDB>{}, a, r, hi, kb, done, bad, mystep);
#pragma unroll
  for (int q = 0; q < kDB / 2; ++q) S.X[mystep][2 * q + (hi ? 1 : 0)] = a[q];
  if (!hi) S.rsel[mystep] = r;   // (every row is the pivot of exactly one step)
  return bad;
}

// Inverses of the triangles of a 32 x 32 LU (X, pivot order) by column
// sweeps over the identity, two waves per triangle.  Lane (i, g) holds row i
// of the inverse at the columns 4 t + g (t < 8); the row needed at sweep step
// j is row j of the lane's own group, read from lane j or j + 32 of the wave.
//   L^{-1}: for j = 0 .. 30, rows i > j: z_i -= l_ij z_j  (z_j is final by then);
//   U^{-1}: for j = 31 .. 1, rows i < j: z_i -= (u_ij / u_jj) z_j, and every
//           row is divided by its own u_ii at the end.
// Only the columns where row j can be nonzero are swept (c <= j for L^{-1},
// c >= j for U^{-1}); rows outside a step's range take a zero multiplier.
template <typename R, bool LOWER, int J, int T>
__device__ __forceinline__ void tri_inv_slot(cplx_t<R> (&z)[kDB / 4], cplx_t<R> m, bool hi) {
  if constexpr (LOWER ? T <= J / 4 : T >= J / 4)
    cfms4(z[T], m, csel(hi, lane_read(z[T], J + 32), lane_read(z[T], J)));
}
template <typename R, int J, int... T>
__device__ __forceinline__ void lower_inv_step(std::integer_sequence<int, T...>, cplx_t<R> (&z)[kDB / 4],
                                               cplx_t<R> (*X)[kDB + 1], int i, bool hi) {
  using C = cplx_t<R>;
  const C l = csel(i > J, X[i][J], cmake<C>(0, 0));
  (tri_inv_slot<R, true, J, T>(z, l, hi), ...);
}
template <typename R, int J, int... T>
__device__ __forceinline__ void upper_inv_step(std::integer_sequence<int, T...>, cplx_t<R> (&z)[kDB / 4],
                                               cplx_t<R> (*X)[kDB + 1], int i, bool hi) {
  using C = cplx_t<R>;
  const C d = X[J][J];
  const R inv = pos_recip(cabs2(d));
  const C u = csel(i < J, cmul(X[i][J], cmake<C>(d.x * inv, -d.y * inv)), cmake<C>(0, 0));
  (tri_inv_slot<R, false, J, T>(z, u, hi), ...);
}
template <typename R, int... Q>
__device__ __forceinline__ void tri_inv_sweeps(std::integer_sequence<int, Q...>, cplx_t<R> (&z)[kDB / 4],
                                               cplx_t<R> (*X)[kDB + 1], int i, bool hi, bool lower) {
  constexpr auto slots = std::make_integer_sequence<int, kDB / 4>{};
  if (lower) (lower_inv_step<R, Q>(slots, z, X, i, hi), ...);
  else (upper_inv_step<R, kDB - 1 - Q>(slots, z, X, i, hi), ...);
}

// Workgroup part: waves 0-1 invert L, waves 2-3 U; column-major results.
template <typename R>
__device__ __forceinline__ void tri_inv32(cplx_t<R> (*X)[kDB + 1], cplx_t<R>* __restrict__ Li,
                                          cplx_t<R>* __restrict__ Ui, int kb) {
  using C = cplx_t<R>;
  const int w = threadIdx.x >> 6, gh = (threadIdx.x >> 5) & 1, i = threadIdx.x & 31;
  const bool lower = w < 2;
  const int g = 2 * (w & 1) + gh;
  C z[kDB / 4];
#pragma unroll
  for (int t = 0; t < kDB / 4; ++t) z[t] = cmake<C>(4 * t + g == i ? 1 : 0, 0);
  tri_inv_sweeps<R>(std::make_integer_sequence<int, kDB - 1>{}, z, X, i, gh == 1, lower);
  C* out = lower ? Li : Ui;
  C s = cmake<C>(1, 0);
  if (!lower) {
    const C d = X[i][i];
    const R inv = pos_recip(cabs2(d));
    s = cmake<C>(d.x * inv, -d.y * inv);
  }
#pragma unroll
  for (int t = 0; t < kDB / 4; ++t) {
    const int c = 4 * t + g;
    if (i < kb && c < kb) out[c * kDB + i] = cmul(z[t], s);
  }
}

// One 16 x 16 block of a complex product on MFMA, k over [0, kmax) in steps
// of 4: acc += A(16 rows) B(16 columns), operands fetched per lane through
// a(row, k) and b(k, col) (row, col in 0..15); accumulator entry r of a lane
// is output (lane & 15, mfma_row(lane, r)), as in gemm_tile_core.
template <typename R, typename FA, typename FB>
__device__ __forceinline__ void mfma_block16(typename Acc<R>::type& re, typename Acc<R>::type& im, int kmax, FA&& a,
                                             FB&& b) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int kk = 0; kk < kmax; kk += 4) {
    const cplx_t<R> av = a(lane & 15, kk + (lane >> 4));
    const cplx_t<R> bv = b(kk + (lane >> 4), lane & 15);
    re = mfma16(bv.x, av.x, re);
    re = mfma16(-bv.y, av.y, re);
    im = mfma16(bv.y, av.x, im);
    im = mfma16(bv.x, av.y, im);
  }
}

// The diagonal-block LU of block [k0, k0 + kb) of front fi by one workgroup
// of 256 threads.  With kprev >= 0 the block first takes the trailing update
// of the previous step (full block at kprev): A_kk -= L(k, prev) U(prev, k),
// read from the L21 and U12 that step wrote, or (fused) formed here from the
// previous block's strips as they stand and its triangle inverses:
// L(k, prev) = A(k, prev) U_prev^{-1}, U(prev, k) = L_prev^{-1} P A(prev, k).
template <typename R>
__device__ __forceinline__ void diag_lu_block(const MfDev& mf, cplx_t<R>* __restrict__ arena, cplx_t<R>* __restrict__ dinv, int fi,
                              int k0, int nb, int kprev, DiagLds<R>& S, bool fused = false) {
  using C = cplx_t<R>;
  const FrontDev& f = mf.fronts[fi];
  const int p = f.p;
  if (k0 >= p) return;
  const int kb = min(nb, p - k0);
  const int F = f.F;
  C* A = arena + f.off + (int64_t)k0 * F + k0;   // block origin, leading dimension F
  auto& D = S.D;
  auto& Lm = S.Lm;
  auto& X = S.X;
  auto& rsel = S.rsel;
  const int tid = threadIdx.x;
  const float fn = __uint_as_float(mf.fnorm[fi]);   // (read here, used after the LU)
  if (kprev >= 0 && !fused) {
    const C* base = arena + f.off;
    for (int t = tid; t < kDB * kDB; t += 256) {
      const int c = t / kDB, i = t - c * kDB;
      Lm[i][c] = (i < kb) ? base[(int64_t)(kprev + c) * F + k0 + i] : cmake<C>(0, 0);
      X[i][c] = (c < kb) ? base[(int64_t)(k0 + c) * F + kprev + i] : cmake<C>(0, 0);
    }
    __syncthreads();
  } else if (kprev >= 0) {
    // (the previous block is a full 32 x 32 one: kprev + 32 = k0 < p)
    const C* base = arena + f.off;
    const C* Lp = dinv + (int64_t)2 * kDB * kDB * (f.dblk + kprev / kDB);   // column-major
    const C* Up = Lp + kDB * kDB;
    const int* pr = mf.prow + f.perm + kprev;                               // front rows, pivot order
    // (U_prev^{-1} is loaded with the rest and kept in registers until D is
    // free again, so the second product does not wait on memory; the block's
    // own entries come in with them, each lane taking those of its place in
    // the last product's output)
    // ((P A)(prev, k) comes as the previous block's rows in their stored
    // order, each landing at its pivot index, so those loads need not wait
    // for pr)
    const int i32 = tid & (kDB - 1);
    const int pri = pr[i32];
    using V = typename Acc<R>::type;
    const int w = tid >> 6, lane = tid & 63, ba = 16 * (w % 2), bb = 16 * (w / 2);
    C akk[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = ba + (lane & 15), col = bb + mfma_row(R(0), lane, r);
      akk[r] = (row < kb && col < kb) ? A[(int64_t)col * F + row] : cmake<C>(row == col ? 1 : 0, 0);
    }
    constexpr int kPer = kDB * kDB / 256;
    C up[kPer], xr[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int t = tid + 256 * u, c = t / kDB, i = t - c * kDB;   // (i = i32)
      Lm[i][c] = (i < kb) ? base[(int64_t)(kprev + c) * F + k0 + i] : cmake<C>(0, 0);   // A(k, prev)
      xr[u] = (c < kb) ? base[(int64_t)(k0 + c) * F + kprev + i] : cmake<C>(0, 0);      // A(prev, k), stored order
      D[i][c] = Lp[c * kDB + i];
      up[u] = Up[c * kDB + i];
    }
    if (tid < kDB) S.kofr[pri - kprev] = tid;
    __syncthreads();
    {
      const int u_ = S.kofr[i32];
#pragma unroll
      for (int u = 0; u < kPer; ++u) X[u_][(tid + 256 * u) / kDB] = xr[u];   // (P A)(prev, k)
    }
    __syncthreads();
    // U(prev, k) = L_prev^{-1} X and L(k, prev) = A(k, prev) U_prev^{-1}: wave
    // w forms the 16 x 16 block (w % 2, w / 2) of each on MFMA.
    V ure = {}, uim = {}, lre = {}, lim = {};
    mfma_block16<R>(ure, uim, kDB, [&](int r, int k) { return D[ba + r][k]; },
                    [&](int k, int c) { return X[k][bb + c]; });
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int t = tid + 256 * u, c = t / kDB, i = t - c * kDB;
      D[i][c] = up[u];
    }
    __syncthreads();
    mfma_block16<R>(lre, lim, kDB, [&](int r, int k) { return Lm[ba + r][k]; },
                    [&](int k, int c) { return D[k][bb + c]; });
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = ba + (lane & 15), col = bb + mfma_row(R(0), lane, r);
      X[row][col] = cmake<C>(ure[r], uim[r]);
      Lm[row][col] = cmake<C>(lre[r], lim[r]);
    }
    __syncthreads();
    // A_kk - L(k, prev) U(prev, k), block (w % 2, w / 2) of wave w on MFMA
    // (rows and columns past kb keep the identity: L and U are zero there).
    V dre = {}, dim = {};
    mfma_block16<R>(dre, dim, kDB, [&](int r, int k) { return Lm[ba + r][k]; },
                    [&](int k, int c) { return X[k][bb + c]; });
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = ba + (lane & 15), col = bb + mfma_row(R(0), lane, r);
      D[row][col] = cmake<C>(akk[r].x - dre[r], akk[r].y - dim[r]);
    }
    __syncthreads();
  }
  // The block is padded to 32 x 32 with the identity so that every step is
  // uniform.  Rows stay where they are (physical order); the pivot chosen at
  // step j is recorded in rsel[j] and the LU is written back in pivot order.
  if (!(kprev >= 0 && fused)) {
    for (int t = tid; t < kDB * kDB; t += 256) {
      const int c = t / kDB, i = t - c * kDB;
      C v = cmake<C>(i == c ? 1 : 0, 0);
      if (i < kb && c < kb) {
        v = A[(int64_t)c * F + i];
        if (kprev >= 0)
          for (int u = 0; u < kDB; ++u) cfms(v, Lm[i][u], X[u][c]);
      }
      D[i][c] = v;
    }
    __syncthreads();
  }
  if (wave_lu32<R>(S, kb) && tid == 0) atomicCAS(mf.info, 0, fi + 1);
  __syncthreads();
  // Block-local pivoting keeps every interchange inside the block, so the
  // row order is also the block's part of the front's final permutation.
  if (tid < kb) {
    mf.prow[f.perm + k0 + tid] = k0 + rsel[tid];
    mf.perm[f.perm + k0 + tid] = k0 + rsel[tid];
  }
  // Pivot statistics against the largest entry of the front as assembled:
  // a pivot below piv_tol (1e3 FP64 eps) times it is a breakdown (info[0] =
  // front + 1, info[10] = 1); one below piv_warn (1e3 eps of the front
  // precision) is counted in info[9]; the block's largest entry before and
  // after its LU feeds the growth statistic.
  float gmax = 0.f;
  for (int t = tid; t < kDB * kDB; t += 256) {
    const int c = t / kDB, i = t - c * kDB;
    if (i < kb && c < kb) {
      A[(int64_t)c * F + i] = X[i][c];
      gmax = fmaxf(gmax, (float)sqrt(fmax(cabs2(X[i][c]), cabs2(D[i][c]))));
    }
  }
  if (fn > 0.f) {
    // (reduced in the workgroup first: one atomic per statistic and block,
    // not one per pivot and wave, as a launch over many fronts would send
    // thousands of atomics to the same two words)
    float rmin = 3.0e38f;
    if (tid < kb) {
      const float u = (float)sqrt(cabs2(X[tid][tid]));
      const float ratio = u / fn;
      if (!(ratio >= mf.piv_tol)) {
        atomicCAS(mf.info, 0, fi + 1);
        atomicExch(mf.info + 10, 1);
      }
      if (!(ratio >= mf.piv_warn)) atomicAdd(mf.info + 9, 1);
      if (ratio >= 0.f) rmin = ratio;
    }
    for (int o = 32; o > 0; o >>= 1) {   // (the kb <= 32 pivots are in wave 0)
      rmin = fminf(rmin, __shfl_xor(rmin, o));
      gmax = fmaxf(gmax, __shfl_xor(gmax, o));
    }
    __shared__ float gwave[4];
    if ((tid & 63) == 0) gwave[tid >> 6] = gmax;
    __syncthreads();
    if (tid == 0) {
      if (rmin < 3.0e38f) atomicMin(mf.pstat + 1, __float_as_uint(rmin));
      atomicMax(mf.pstat, __float_as_uint(fmaxf(fmaxf(gwave[0], gwave[1]), fmaxf(gwave[2], gwave[3])) / fn));
    }
  }
  C* Li = dinv + (int64_t)2 * kDB * kDB * (f.dblk + k0 / kDB);
  tri_inv32<R>(X, Li, Li + kDB * kDB, kb);
}

template <typename R>
__global__ void __launch_bounds__(256) diag_lu_kernel(MfDev mf, cplx_t<R>* __restrict__ arena,
                                                      cplx_t<R>* __restrict__ dinv, int f0, int k0, int nb) {
  __shared__ DiagLds<R> S;
  diag_lu_block<R>(mf, arena, dinv, f0 + blockIdx.x, k0, nb, -1, S);
}

// ------------------------------------------------------------------ tournament pivoting
// Pivot rows of a block [c, c + kb) of a large front chosen over all its
// remaining fully-summed rows [c, p) by a tournament (communication-avoiding
// LU): every chunk of 256 rows names kb candidates by LU with partial
// pivoting of its copy of the block's columns, groups of 8 candidate sets
// (256 rows) are reduced the same way until one set is left, and those kb
// rows are swapped to the top of the block; the diagonal-block LU and the
// L21 / U12 products then run on them as on any block.
constexpr int kTpRows = 256, kTpFan = 8;

// LU with partial pivoting of the rows `row` (one per thread, -1: none; at
// most 256) restricted to the columns [c, c + kb) of the front at A (leading
// dimension F); the positions of the kb pivot rows in pivot order go to
// out[0 .. kb) (-1 where fewer rows remain).  Largest modulus first, ties to
// the lowest position (the moduli compared in single precision).
template <typename R>
__device__ __forceinline__ void tp_pick(const cplx_t<R>* __restrict__ A, int F, int c, int kb, int row, int* out) {
  using C = cplx_t<R>;
  __shared__ unsigned long long key;
  __shared__ C prow[kDB];
  C a[kDB];
#pragma unroll
  for (int j = 0; j < kDB; ++j) a[j] = (row >= 0 && j < kb) ? A[(int64_t)(c + j) * F + row] : cmake<C>(0, 0);
  bool live = row >= 0;
#pragma unroll
  for (int j = 0; j < kDB; ++j) {
    if (j < kb) {
      if (threadIdx.x == 0) key = 0;
      __syncthreads();
      unsigned long long k = 0;
      if (live) {
        const float v = (float)sqrt(cabs2(a[j]));
        k = ((unsigned long long)__float_as_uint(v) << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)row);
      }
      for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long t = __shfl_xor(k, o);
        k = t > k ? t : k;
      }
      if ((threadIdx.x & 63) == 0 && k) atomicMax(&key, k);
      __syncthreads();
      const unsigned long long kk = key;
      const int pr = kk ? (int)(0xFFFFFFFFu - (unsigned)(kk & 0xFFFFFFFFull)) : -1;
      if (threadIdx.x == 0) out[j] = pr;
      if (live && row == pr) {
#pragma unroll
        for (int t = 0; t < kDB; ++t) prow[t] = a[t];
        live = false;
      }
      __syncthreads();
      if (live && pr >= 0) {
        const C d = prow[j];
        const C l = cabs2(d) > R(0) ? cdiv(a[j], d) : cmake<C>(0, 0);
#pragma unroll
        for (int t = j + 1; t < kDB; ++t) cfms(a[t], l, prow[t]);
      }
    } else if (threadIdx.x == 0) {
      out[j] = -1;
    }
  }
}

// Sets of level 0: chunk blockIdx.x of the rows [c, p) of front f0 +
// blockIdx.y; cand[(front * maxsets + set) * 32 + j].
template <typename R>
__global__ void __launch_bounds__(256) tp_select_kernel(MfDev mf, const cplx_t<R>* __restrict__ arena,
                                                        int* __restrict__ cand, int f0, int c, int maxsets) {
  const FrontDev& f = mf.fronts[f0 + blockIdx.y];
  if (c >= f.p) return;
  const int r0 = c + blockIdx.x * kTpRows;
  if (r0 >= f.p) return;
  const int kb = min(kDB, f.p - c);
  const int row = (r0 + (int)threadIdx.x < f.p) ? r0 + threadIdx.x : -1;
  __shared__ int out[kDB];
  tp_pick<R>(arena + f.off, f.F, c, kb, row, out);
  __syncthreads();
  if (threadIdx.x < kDB) cand[((int64_t)blockIdx.y * maxsets + blockIdx.x) * kDB + threadIdx.x] = out[threadIdx.x];
}

// Level lev >= 1: set blockIdx.x merges the sets [8 x, 8 x + 8) of level
// lev - 1 (read from cin, written to cout); a front's set count at level
// lev is its chunk count divided by 8 lev times, rounded up.
template <typename R>
__global__ void __launch_bounds__(256) tp_reduce_kernel(MfDev mf, const cplx_t<R>* __restrict__ arena,
                                                        const int* __restrict__ cin, int* __restrict__ cout, int f0,
                                                        int c, int lev, int maxsets) {
  const FrontDev& f = mf.fronts[f0 + blockIdx.y];
  if (c >= f.p) return;
  int nin = (f.p - c + kTpRows - 1) / kTpRows;
  for (int l = 1; l < lev; ++l) nin = (nin + kTpFan - 1) / kTpFan;
  const int s0 = blockIdx.x * kTpFan;
  if (s0 >= nin) return;
  const int kb = min(kDB, f.p - c);
  const int set = s0 + threadIdx.x / kDB, j = threadIdx.x % kDB;
  const int row = set < nin ? cin[((int64_t)blockIdx.y * maxsets + set) * kDB + j] : -1;
  __shared__ int out[kDB];
  tp_pick<R>(arena + f.off, f.F, c, kb, row, out);
  __syncthreads();
  if (threadIdx.x < kDB) cout[((int64_t)blockIdx.y * maxsets + blockIdx.x) * kDB + threadIdx.x] = out[threadIdx.x];
}

// Swaps the winners win[front * maxsets * 32 + j] (positions >= c) to the
// rows c + j of the whole front, as a sequence of interchanges recorded
// LAPACK-style in ipiv (ipiv[c + j] = the row swapped with row c + j at step
// j).  Every workgroup derives the same net permutation of the touched rows
// (at most 64) and applies it to its 64 columns; blockIdx.y = front.
template <typename R>
__global__ void __launch_bounds__(64) tp_swap_kernel(MfDev mf, cplx_t<R>* __restrict__ arena, const int* __restrict__ win,
                                                     int* __restrict__ ipiv, int f0, int c, int maxsets) {
  using C = cplx_t<R>;
  const FrontDev& f = mf.fronts[f0 + blockIdx.y];
  if (c >= f.p) return;
  const int kb = min(kDB, f.p - c);
  __shared__ int pos[2 * kDB], content[2 * kDB], cnt;
  __shared__ C tmp[64][2 * kDB + 1];
  if (threadIdx.x == 0) {
    int n = 0;
    const int* w = win + (int64_t)blockIdx.y * maxsets * kDB;
    for (int j = 0; j < kb; ++j) {
      const int a = c + j;
      int wj = w[j];
      if (wj < c || wj >= f.p) wj = a;   // (no candidate: keep the row)
      // current position of the original row wj, and the slot of row a
      int xw = -1, xa = -1;
      for (int x = 0; x < n; ++x) {
        if (content[x] == wj) xw = x;
        if (pos[x] == a) xa = x;
      }
      if (xw < 0) {   // untouched: still at its own position
        for (int x = 0; x < n; ++x)
          if (pos[x] == wj) xw = x;
        if (xw < 0) { pos[n] = wj; content[n] = wj; xw = n++; }
      }
      if (xa < 0) { pos[n] = a; content[n] = a; xa = n++; }
      if (blockIdx.x == 0) ipiv[f.perm + a] = pos[xw];
      const int t = content[xa]; content[xa] = content[xw]; content[xw] = t;
    }
    cnt = n;
  }
  __syncthreads();
  const int n = cnt;
  const int col = blockIdx.x * 64 + threadIdx.x;
  if (col >= f.F) return;
  C* cp = arena + f.off + (int64_t)col * f.F;
  for (int x = 0; x < n; ++x) tmp[threadIdx.x][x] = cp[content[x]];
  for (int x = 0; x < n; ++x) cp[pos[x]] = tmp[threadIdx.x][x];
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
// Minimum waves per SIMD asked of the GEMM kernels: 4 in FP32 (fits without
// spills); none in FP64, whose accumulators and prefetch registers need more.
template <typename R> constexpr int kGemmWaves = sizeof(R) == 4 ? 4 : 1;

// One 64 x 64 tile (rows m0.., columns n0..) of C = from_c ? C + sgn A B : sgn A B,
// complex column-major operands, k restricted to [kbeg, kend).  brow (optional)
// maps row gk of B to row brow[gk] - brow_off (a row permutation of B).
// Tile shapes BM x BN of the four waves (each wave 32 x 32): 64 x 64 by
// default, 128 x 32 and 32 x 128 for products with one side of at most 32
// (L21 / U12 of a step, the second block's column and row of a pair).
template <typename R, int BM = kBM, int BN = kBN>
struct GemmLds {
  cplx_t<R> As[kBK][BM + 1];
  cplx_t<R> Bs[kBK][BN + 1];
};

// skip > 0: entries with row < skip and column < skip are not stored (a
// block another workgroup of the same launch owns).
template <typename R, int BM = kBM, int BN = kBN>
__device__ inline void gemm_tile_core(GemmLds<R, BM, BN>& L, const cplx_t<R>* __restrict__ Ap, int lda,
                                      const cplx_t<R>* __restrict__ Bp, int ldb, cplx_t<R>* __restrict__ Cp, int ldc,
                                      int m, int n, int k, int m0, int n0, bool from_c, R sgn, int kbeg, int kend,
                                      const int* brow, int brow_off, int skip) {
  using C = cplx_t<R>;
  using V = typename Acc<R>::type;
  auto& As = L.As;
  auto& Bs = L.Bs;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  static_assert((BM / 32) * (BN / 32) == 4, "four waves of 32 x 32");
  const int wm = (wave % (BM / 32)) * 32, wn = (wave / (BM / 32)) * 32;
  // Two real accumulators per 16 x 16 complex block: re = sum (ar br - ai bi),
  // im = sum (ar bi + ai br).  Updates start from C and take A scaled by sgn
  // when it is staged in LDS, so C -= A B needs no extra pass.  The products
  // are formed as (B^T A^T)^T: B takes the MFMA's first operand, so that the
  // 16 lanes holding one output column hold 16 consecutive rows of C, and
  // loads and stores of the column-major C tile are contiguous.
  // Addresses are a tile base (uniform) plus 32-bit offsets inside the tile.
  C* __restrict__ Ct = Cp + (int64_t)n0 * ldc + m0;
  const int mt = m - m0, nt = n - n0;
  kend = min(kend, k);
  // (the first stage's row index of B goes out before the C tile: the memory
  // counter waits in issue order, and the first B loads wait on it)
  const int bkk = threadIdx.x % kBK;   // this thread's k row in every stage
  const int brow0 = (brow && kbeg < kend) ? brow[bkk < kend - kbeg ? kbeg + bkk : 0] - brow_off : 0;
  V re[2][2], im[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wm + 16 * a + (lane & 15);
        const int col = wn + 16 * b + mfma_row(R(0), lane, r);
        C c0 = cmake<C>(0, 0);
        if (from_c && row < mt && col < nt) c0 = Ct[col * ldc + row];
        re[a][b][r] = c0.x;
        im[a][b][r] = c0.y;
      }
  // Register prefetch: the next stage's operands are loaded while the
  // current stage runs on MFMA (one LDS buffer, two barriers per stage).
  constexpr int kPerA = BM * kBK / 256, kPerB = BN * kBK / 256;
  C ra[kPerA], rb[kPerB];
  const C* __restrict__ Bt = Bp + (int64_t)n0 * ldb;
  auto load_stage = [&](int kk0) {
    const C* __restrict__ At = Ap + (int64_t)kk0 * lda + m0;
    const int kt = kend - kk0;
#pragma unroll
    for (int u = 0; u < kPerA; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int row = e % BM, kk = e / BM;
      ra[u] = (row < mt && kk < kt) ? At[kk * lda + row] : cmake<C>(0, 0);
    }
#pragma unroll
    for (int u = 0; u < kPerB; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int kk = e % kBK, col = e / kBK;   // (kk = bkk)
      const int br = brow ? (kk0 == kbeg ? brow0 : brow[kk < kt ? kk0 + kk : 0] - brow_off) : kk0 + kk;
      rb[u] = (kk < kt && col < nt) ? Bt[col * ldb + br] : cmake<C>(0, 0);
    }
  };
  if (kbeg < kend) load_stage(kbeg);
  for (int kk0 = kbeg; kk0 < kend; kk0 += kBK) {
#pragma unroll
    for (int u = 0; u < kPerA; ++u) {
      const int e = threadIdx.x + 256 * u;
      As[e / BM][e % BM] = cmake<C>(sgn * ra[u].x, sgn * ra[u].y);
    }
#pragma unroll
    for (int u = 0; u < kPerB; ++u) {
      const int e = threadIdx.x + 256 * u;
      Bs[e % kBK][e / kBK] = rb[u];
    }
    __syncthreads();
    if (kk0 + kBK < kend) load_stage(kk0 + kBK);
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
          re[a][b] = mfma16(bv[b].x, av[a].x, re[a][b]);
          re[a][b] = mfma16(-bv[b].y, av[a].y, re[a][b]);
          im[a][b] = mfma16(bv[b].y, av[a].x, im[a][b]);
          im[a][b] = mfma16(bv[b].x, av[a].y, im[a][b]);
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
        const int row = wm + 16 * a + (lane & 15);
        const int col = wn + 16 * b + mfma_row(R(0), lane, r);
        if (row < mt && col < nt && !(m0 + row < skip && n0 + col < skip))
          Ct[col * ldc + row] = cmake<C>(re[a][b][r], im[a][b][r]);
      }
}

template <typename R>
__device__ inline void gemm_tile(const cplx_t<R>* __restrict__ Ap, int lda, const cplx_t<R>* __restrict__ Bp, int ldb,
                                 cplx_t<R>* __restrict__ Cp, int ldc, int m, int n, int k, int m0, int n0, bool from_c,
                                 R sgn, int kbeg, int kend, const int* brow = nullptr, int brow_off = 0) {
  __shared__ GemmLds<R> L;
  gemm_tile_core<R>(L, Ap, lda, Bp, ldb, Cp, ldc, m, n, k, m0, n0, from_c, sgn, kbeg, kend, brow, brow_off, 0);
}

// Front GEMMs of one elimination step (k0 = step block, kb <= 32 columns):
//   mode 0: trailing update  A22 -= L21 U12
//   mode 1: L inverse update XL[k0+kb:p, 0:k0+kb] -= L[k0+kb:p, k0:k0+kb] XL[k0:k0+kb, 0:k0+kb]
//   mode 2: U inverse update XU[0:k0, k0:p]       -= U[0:k0, k0:k0+kb]    XU[k0:k0+kb, k0:p]
//   mode 7: L21 = A21 Uinv_kk (first tiles_m workgroups) and U12 = Linv_kk P A12
//           (the rest), P the step's row order from the diagonal-block LU,
//           applied while loading A12.  Both overwrite their input block;
//           every workgroup reads all of its own block before writing it.
//   mode 6: as mode 7 on 64 x 64 tiles
//   mode 3: the next block's column and row take this step's update (a pair
//           of steps whose trailing update then goes as one rank-2kb product)
// NEXT (mode 0 only): a workgroup with bx < 0 factors the next diagonal
// block of front by, taking this step's update of that block itself; the
// tile holding the block skips it.
// (bx, by) = (tile, front) of the workgroup.
//   mode 8: column strip of block k0 (rows [k0, F), its kb columns) takes
//           the updates of the steps [kf, k0) of an outer block
//   mode 9: row strip of block k0 (its kb rows, columns [k0 + kb, F)) takes
//           the same updates (left-looking inside an outer block whose
//           trailing update then goes as one rank-(k0 - kf) product)
// LDS bytes gemm_body<R, NEXT, mode> needs (the kernels that call it hold it).
template <typename R, bool NEXT, int mode>
constexpr size_t gemm_body_lds() {
  constexpr bool kNarrow = mode == 3 || mode == 7 || mode == 8 || mode == 9;
  constexpr size_t kGemm = kNarrow ? sizeof(GemmLds<R, 128, 32>) : sizeof(GemmLds<R>);
  return NEXT ? (sizeof(DiagLds<R>) > kGemm ? sizeof(DiagLds<R>) : kGemm) : kGemm;
}

template <typename R, bool NEXT, int mode>
__device__ inline void gemm_body(const MfDev& mf, cplx_t<R>* __restrict__ arena, cplx_t<R>* __restrict__ xwork,
                                 cplx_t<R>* __restrict__ dinv, int f0, int step, int nb, int tiles_m, int bx, int by,
                                 unsigned char* __restrict__ lds, int kf = 0) {
  using C = cplx_t<R>;
  // Modes 3 and 7: products with one side of at most 32 take the 128 x 32
  // (tall) or 32 x 128 (wide) tile; tiles_m then counts 128-row tiles.
  // Mode 6 is mode 7 on 64 x 64 tiles (twice the workgroups, each with half
  // its waves idle): shorter launches for levels of few fronts, where the
  // step's latency rather than its throughput counts.
  constexpr bool kNarrow = mode == 3 || mode == 7 || mode == 8 || mode == 9;
  const FrontDev f = mf.fronts[f0 + by];
  int k0, kb;
  if (!step_range<R>(f, mode == 2 ? 2 : 0, step, nb, k0, kb)) return;
  int skip = 0;
  if (NEXT) {
    const int k1 = k0 + kb;
    if (bx < 0) {
      if (k1 < f.p) diag_lu_block<R>(mf, arena, dinv, f0 + by, k1, nb, k0, *reinterpret_cast<DiagLds<R>*>(lds));
      return;
    }
    if (k1 < f.p) skip = min(nb, f.p - k1);
  }
  const int F = f.F, p = f.p;
  C* base = arena + f.off;
  const C *Ap, *Bp;
  C* Cp;
  int m, n, k, lda, ldb, ldc;
  int tm, tn;
  const int* brow = nullptr;
  bool assign = false;
  if constexpr (mode == 8 || mode == 9) {
    // Strips of block k0 against the outer block's earlier steps [kf, k0);
    // mode 8 uses the tall tiles (bx < tiles_m), mode 9 the wide ones.
    k = k0 - kf;
    Ap = base + (int64_t)kf * F + k0; lda = F;
    if constexpr (mode == 8) {
      if (bx >= tiles_m) return;
      tm = bx; tn = 0;
      m = F - k0; n = kb;
      Bp = base + (int64_t)k0 * F + kf; ldb = F;
      Cp = base + (int64_t)k0 * F + k0; ldc = F;
    } else {
      if (bx < tiles_m) return;
      tm = 0; tn = bx - tiles_m;
      m = kb; n = F - k0 - kb;
      Bp = base + (int64_t)(k0 + kb) * F + kf; ldb = F;
      Cp = base + (int64_t)(k0 + kb) * F + k0; ldc = F;
    }
  } else if constexpr (mode == 3) {
    // The next block (kb2 columns / rows after this one) of a pair of
    // steps: its column below this block (first tiles_m workgroups) and its
    // row right of it (the rest) take this step's update.
    const int kb2 = min(nb, p - k0 - kb);
    if (kb2 <= 0) return;
    Ap = base + (int64_t)k0 * F + (k0 + kb); lda = F;
    k = kb;
    if (bx < tiles_m) {
      tm = bx; tn = 0;
      m = F - k0 - kb; n = kb2;
      Bp = base + (int64_t)(k0 + kb) * F + k0; ldb = F;
      Cp = base + (int64_t)(k0 + kb) * F + (k0 + kb); ldc = F;
    } else {
      tm = 0; tn = bx - tiles_m;
      m = kb2; n = F - k0 - kb - kb2;
      Bp = base + (int64_t)(k0 + kb + kb2) * F + k0; ldb = F;
      Cp = base + (int64_t)(k0 + kb + kb2) * F + (k0 + kb); ldc = F;
    }
  } else if constexpr (mode == 7 || mode == 6) {
    const C* Li = dinv + (int64_t)2 * kDB * kDB * (f.dblk + k0 / kDB);
    const C* Ui = Li + kDB * kDB;
    assign = true;
    if (bx < tiles_m) {                // L21 = A21 Uinv_kk
      tm = bx; tn = 0;
      m = F - k0 - kb; n = kb; k = kb;
      Ap = base + (int64_t)k0 * F + (k0 + kb); lda = F;
      Bp = Ui; ldb = kDB;
      Cp = base + (int64_t)k0 * F + (k0 + kb); ldc = F;
    } else {                           // U12 = Linv_kk (P A12)
      tm = 0; tn = bx - tiles_m;
      m = kb; n = F - k0 - kb; k = kb;
      Ap = Li; lda = kDB;
      Bp = base + (int64_t)(k0 + kb) * F; ldb = F;
      Cp = base + (int64_t)(k0 + kb) * F + k0; ldc = F;
      brow = mf.prow + f.perm + k0;
    }
  } else {
    tm = bx % tiles_m;
    tn = bx / tiles_m;
    if constexpr (mode == 0) {
      m = n = F - k0 - kb; k = kb;
      Ap = base + (int64_t)k0 * F + (k0 + kb); lda = F;
      Bp = base + (int64_t)(k0 + kb) * F + k0; ldb = F;
      Cp = base + (int64_t)(k0 + kb) * F + (k0 + kb); ldc = F;
    } else if constexpr (mode == 1) {
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
  }
  if constexpr (kNarrow) {
    if (bx < tiles_m) {   // n <= 32: 128-row tiles
      const int m0 = tm * 128;
      if (m <= 0 || n <= 0 || k <= 0 || m0 >= m) return;
      gemm_tile_core<R, 128, 32>(*reinterpret_cast<GemmLds<R, 128, 32>*>(lds), Ap, lda, Bp, ldb, Cp, ldc, m, n, k,
                                 m0, 0, !assign, assign ? R(1) : R(-1), 0, k, brow, 0, 0);
    } else {              // m <= 32: 128-column tiles
      const int n0 = tn * 128;
      if (m <= 0 || n <= 0 || k <= 0 || n0 >= n) return;
      gemm_tile_core<R, 32, 128>(*reinterpret_cast<GemmLds<R, 32, 128>*>(lds), Ap, lda, Bp, ldb, Cp, ldc, m, n, k,
                                 0, n0, !assign, assign ? R(1) : R(-1), 0, k, brow, 0, 0);
    }
  } else {
    const int m0 = tm * kBM, n0 = tn * kBN;
    if (m <= 0 || n <= 0 || k <= 0 || m0 >= m || n0 >= n) return;
    gemm_tile_core<R>(*reinterpret_cast<GemmLds<R>*>(lds), Ap, lda, Bp, ldb, Cp, ldc, m, n, k, m0, n0, !assign,
                      assign ? R(1) : R(-1), 0, k, brow, 0, skip);
  }
}

template <typename R, int MODE>
__global__ void __launch_bounds__(256, kGemmWaves<R>) gemm_kernel(MfDev mf, cplx_t<R>* __restrict__ arena, cplx_t<R>* __restrict__ xwork,
                                                   cplx_t<R>* __restrict__ dinv, int f0, int step, int nb,
                                                   int tiles_m, int kf = 0) {
  __shared__ __align__(16) unsigned char lds[gemm_body_lds<R, false, MODE>()];
  gemm_body<R, false, MODE>(mf, arena, xwork, dinv, f0, step, nb, tiles_m, blockIdx.x, blockIdx.y, lds, kf);
}

// Trailing update with the next diagonal block (mode 0, NEXT above); asks
// for 4 waves per SIMD so that the block's registers do not halve the tiles'
// occupancy.  Grid (tiles + 1, fronts): the first nf workgroups in launch
// order factor the diagonal blocks (so that they start first and overlap the
// tiles instead of waiting for free slots), the rest are the fronts' tiles.
template <typename R>
__global__ void __launch_bounds__(256, 4) gemm_next_kernel(MfDev mf, cplx_t<R>* __restrict__ arena,
                                                           cplx_t<R>* __restrict__ xwork, cplx_t<R>* __restrict__ dinv,
                                                           int f0, int step, int nb, int tiles_m) {
  const int nf = gridDim.y, per = gridDim.x - 1;
  const int lin = blockIdx.x + gridDim.x * blockIdx.y;
  int bx = -1, by = lin;
  if (lin >= nf) {
    by = (lin - nf) / per;
    bx = lin - nf - by * per;
  }
  __shared__ __align__(16) unsigned char lds[gemm_body_lds<R, true, 0>()];
  gemm_body<R, true, 0>(mf, arena, xwork, dinv, f0, step, nb, tiles_m, bx, by, lds);
}

// ------------------------------------------------------------------ fused single steps
// One launch per elimination step (levels of single steps, block-local
// pivoting) instead of an L21 / U12 launch and a trailing-update launch:
//  (a) one workgroup per front updates and factors the next diagonal block,
//      forming its share of L21 / U12 itself (diag_lu_block, fused form);
//  (b) each 64 x 64 trailing tile forms its own rows of L21 = A21 U_kk^{-1}
//      and columns of U12 = L_kk^{-1} P A12 from the strips as they stand,
//      then takes C -= L21 U12 on MFMA (the tile holding the next diagonal
//      block skips it, as in the NEXT form);
//  (c) the previous step's L21 / U12 are written into the front (gemm_body
//      mode 6 of step - 1).  Nothing else in the launch reads or writes the
//      strips of step - 1: the tiles and (a) read the strips of this step,
//      and (b) writes only the trailing block.
// After the last step one mode-6 (or 7) launch writes that step's L21 / U12.
template <typename R>
struct FusedLds {
  cplx_t<R> Lt[kDB][kBM + 1];   // L21 rows of the tile by k (negated once formed)
  cplx_t<R> Ut[kDB][kBN + 1];   // U12 columns of the tile by k
  int kofr[kDB];                // pivot index of each row of the block
};

template <typename R>
__device__ inline void fused_tile(const MfDev& mf, cplx_t<R>* __restrict__ arena, const cplx_t<R>* __restrict__ dinv,
                                  const FrontDev& f, int k0, int kb, int skip, int tm, int tn, FusedLds<R>& L) {
  using C = cplx_t<R>;
  using V = typename Acc<R>::type;
  const int F = f.F, k1 = k0 + kb;
  const int m = F - k1;                     // trailing rows = columns
  const int m0 = tm * kBM, n0 = tn * kBN;
  if (m <= 0 || m0 >= m || n0 >= m) return;
  const int mt = m - m0, nt = m - n0;
  C* base = arena + f.off;
  const C* Li = dinv + (int64_t)2 * kDB * kDB * (f.dblk + k0 / kDB);   // column-major, valid for < kb
  const C* Ui = Li + kDB * kDB;
  const int* pr = mf.prow + f.perm + k0;                               // front rows, pivot order
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  auto& Lt = L.Lt;
  auto& Ut = L.Ut;
  // Loads in the order their waits come (the memory counter waits in issue
  // order): each thread's pivot row of the P A12 strip, the strips, the
  // inverse entries; the trailing tile C right after the products (before
  // their write-back and barrier).
  // On MFMA, wave w: L21 rows 16 w .. 16 w + 15 (all 32 columns u, two
  // blocks) = A21 Uinv, and U12 columns 16 w .. 16 w + 15 (all 32 rows u) =
  // Linv (P A12).  The inverses' entries come from global memory (a few KB);
  // outside [0, kb) they are not written by the block LU, so the operands
  // are masked there (A21 and P A12 are zero beyond kb).
  // A21 by rows of a column; P A12 as the block's rows k0 + i of a column
  // in their stored order (the pivot rows pr[u] are a permutation of them),
  // each landing in LDS at its pivot index: the loads need not wait for pr.
  // (i = tid % 32 in every pass)
  const int i32 = tid & (kDB - 1);
  const int pru = i32 < kb ? pr[i32] : 0;
  constexpr int kUp = kDB * kBN / 256;
  C uraw[kUp];
#pragma unroll
  for (int q = 0; q < kUp; ++q) {
    const int t = tid + 256 * q, c = t / kDB;
    uraw[q] = (i32 < kb && c < nt) ? base[(int64_t)(k1 + n0 + c) * F + k0 + i32] : cmake<C>(0, 0);
  }
  for (int t = tid; t < kDB * kBM; t += 256) {
    const int v = t / kBM, r = t - v * kBM;
    Lt[v][r] = (v < kb && r < mt) ? base[(int64_t)(k0 + v) * F + k1 + m0 + r] : cmake<C>(0, 0);   // A21
  }
  const int li = lane & 15, lk = lane >> 4;
  C uv[2][kDB / 4], lv[2][kDB / 4];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int u = 16 * b + li;
#pragma unroll
    for (int t = 0; t < kDB / 4; ++t) {
      const int k = 4 * t + lk;
      uv[b][t] = (k < kb && u < kb) ? Ui[u * kDB + k] : cmake<C>(0, 0);   // Uinv(k, u)
      lv[b][t] = (k < kb && u < kb) ? Li[k * kDB + u] : cmake<C>(0, 0);   // Linv(u, k)
    }
  }
  if (tid < kb) L.kofr[pru - k0] = tid;
  __syncthreads();
  {
    // (rows past kb, of a ragged last block, stay zero at their own index)
    const int u = i32 < kb ? L.kofr[i32] : i32;
#pragma unroll
    for (int q = 0; q < kUp; ++q) Ut[u][(tid + 256 * q) / kDB] = uraw[q];   // P A12
  }
  __syncthreads();
  using Vt = typename Acc<R>::type;
  Vt lre[2] = {}, lim[2] = {}, ure[2] = {}, uim[2] = {};
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    mfma_block16<R>(lre[b], lim[b], kDB, [&](int r, int k) { return Lt[k][16 * w + r]; },
                    [&](int k, int) { return uv[b][k >> 2]; });
    mfma_block16<R>(ure[b], uim[b], kDB, [&](int, int k) { return lv[b][k >> 2]; },
                    [&](int k, int c) { return Ut[k][16 * w + c]; });
  }
  const int wm = (w % 2) * 32, wn = (w / 2) * 32;
  C* __restrict__ Ct = base + (int64_t)(k1 + n0) * F + k1 + m0;
  V re[2][2], im[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wm + 16 * a + (lane & 15);
        const int col = wn + 16 * b + mfma_row(R(0), lane, r);
        C c0 = cmake<C>(0, 0);
        if (row < mt && col < nt) c0 = Ct[(int64_t)col * F + row];
        re[a][b][r] = c0.x;
        im[a][b][r] = c0.y;
      }
  // (wave w has read and now writes only the columns 16 w .. 16 w + 15 of
  // Lt and Ut, so no barrier is needed before these stores)
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = lane & 15, j = mfma_row(R(0), lane, r);
      Lt[16 * b + j][16 * w + i] = cmake<C>(-lre[b][r], -lim[b][r]);   // L21(16 w + i, 16 b + j), negated
      Ut[16 * b + i][16 * w + j] = cmake<C>(ure[b][r], uim[b][r]);     // U12(16 b + i, 16 w + j)
    }
  __syncthreads();
  // C -= L21 U12 over k < 32 (entries past kb are 0), waves of 32 x 32 as in
  // gemm_tile_core: B takes the MFMA's first operand, lanes of one output
  // column hold 16 consecutive rows.
#pragma unroll
  for (int kk = 0; kk < kDB; kk += 4) {
    C av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) av[a] = Lt[kk + (lane >> 4)][wm + 16 * a + (lane & 15)];
#pragma unroll
    for (int b = 0; b < 2; ++b) bv[b] = Ut[kk + (lane >> 4)][wn + 16 * b + (lane & 15)];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        re[a][b] = mfma16(bv[b].x, av[a].x, re[a][b]);
        re[a][b] = mfma16(-bv[b].y, av[a].y, re[a][b]);
        im[a][b] = mfma16(bv[b].y, av[a].x, im[a][b]);
        im[a][b] = mfma16(bv[b].x, av[a].y, im[a][b]);
      }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wm + 16 * a + (lane & 15);
        const int col = wn + 16 * b + mfma_row(R(0), lane, r);
        if (row < mt && col < nt && !(m0 + row < skip && n0 + col < skip))
          Ct[(int64_t)col * F + row] = cmake<C>(re[a][b][r], im[a][b][r]);
      }
}

template <typename R>
constexpr size_t fused_lds() {
  constexpr size_t a = sizeof(DiagLds<R>), b = sizeof(FusedLds<R>), c = gemm_body_lds<R, false, 6>();
  return a > b ? (a > c ? a : c) : (b > c ? b : c);
}

// Grid (ndiag + nwb + tiles^2, fronts), taken in linear order: the ndiag nf
// diagonal-block workgroups first (they start first and overlap the tiles),
// then the nwb nf write-back workgroups of step - 1, then the tiles.
template <typename R>
__global__ void __launch_bounds__(256, kGemmWaves<R>) gemm_fused_kernel(MfDev mf, cplx_t<R>* __restrict__ arena,
                                                                        cplx_t<R>* __restrict__ xwork,
                                                                        cplx_t<R>* __restrict__ dinv, int f0,
                                                                        int step, int nb, int tiles, int ndiag,
                                                                        int nwb) {
  __shared__ __align__(16) unsigned char lds[fused_lds<R>()];
  const int nf = gridDim.y;
  int rest = blockIdx.x + gridDim.x * blockIdx.y;
  if (rest < ndiag * nf) {
    const int fi = f0 + rest;
    const FrontDev& f = mf.fronts[fi];
    int k0, kb;
    if (!step_range<R>(f, 0, step, nb, k0, kb)) return;
    if (k0 + kb < f.p)
      diag_lu_block<R>(mf, arena, dinv, fi, k0 + kb, nb, k0, *reinterpret_cast<DiagLds<R>*>(lds), true);
    return;
  }
  rest -= ndiag * nf;
  if (rest < nwb * nf) {
    const int by = rest / nwb, bx = rest - by * nwb;
    gemm_body<R, false, 6>(mf, arena, xwork, dinv, f0, step - 1, nb, tiles, bx, by, lds);
    return;
  }
  rest -= nwb * nf;
  const int per = tiles * tiles;
  const int by = rest / per, bx = rest - by * per;
  const FrontDev f = mf.fronts[f0 + by];
  int k0, kb;
  if (!step_range<R>(f, 0, step, nb, k0, kb)) return;
  const int k1 = k0 + kb;
  const int skip = (ndiag && k1 < f.p) ? min(nb, f.p - k1) : 0;
  fused_tile<R>(mf, arena, dinv, f, k0, kb, skip, bx % tiles, bx / tiles, *reinterpret_cast<FusedLds<R>*>(lds));
}

// Row interchanges of every 32-row diagonal block of a level's fronts applied
// to the columns left of the block (the L part written by earlier steps),
// once after all steps: rows [k0, k0 + kb) of columns [0, k0) take the order
// prow.  blockIdx.x = (block, 64-column chunk), blockIdx.y = front; each
// workgroup reads its 32 x 64 piece whole before writing it back.
template <typename R>
__global__ void __launch_bounds__(256) leftswap_kernel(MfDev mf, cplx_t<R>* __restrict__ arena, int f0, int cchunks) {
  using C = cplx_t<R>;
  const FrontDev& f = mf.fronts[f0 + blockIdx.y];
  const int k0 = (blockIdx.x / cchunks) * kDB, c0 = (blockIdx.x % cchunks) * 64;
  if (k0 >= f.p || k0 == 0 || c0 >= k0) return;
  const int kb = min(kDB, f.p - k0);
  const int r = threadIdx.x & 31, cl = threadIdx.x >> 5;
  const int src = (r < kb) ? mf.prow[f.perm + k0 + r] : 0;
  C* A = arena + f.off;
  C v[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int c = c0 + cl + 8 * u;
    v[u] = (r < kb && c < k0) ? A[(int64_t)c * f.F + src] : cmake<C>(0, 0);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int c = c0 + cl + 8 * u;
    if (r < kb && c < k0) A[(int64_t)c * f.F + k0 + r] = v[u];
  }
}

// Triangular inverses of a front's pivot block by recursive doubling over
// its 32-column diagonal blocks (whose inverses the diagonal-block LU left in
// dinv).  For the pair of diagonal blocks A = [o, o + h), B = [o + h, o + h + nb):
//   phase 0:  TL = L(B, A) XL(A, A)        TU = U(A, B) XU(B, B)
//   phase 1:  XL(B, A) = -XL(B, B) TL      XU(A, B) = -XU(A, A) TU
// XL / XU are the lower / upper inverses (p x p, column-major, in xwork), TL
// and TU sit at the same positions of the p x p temporary tbuf.  blockIdx.z =
// 2 pair + (0: L, 1: U); k is cut to where the triangular factor is nonzero.
template <typename R>
__global__ void __launch_bounds__(256, kGemmWaves<R>) inv_gemm_kernel(MfDev mf, const cplx_t<R>* __restrict__ arena,
                                                       cplx_t<R>* __restrict__ xwork, cplx_t<R>* __restrict__ tbuf,
                                                       int f0, int h, int phase, int tiles_m) {
  using C = cplx_t<R>;
  const FrontDev& f = mf.fronts[f0 + blockIdx.y];
  const int p = f.p, F = f.F;
  const int pair = blockIdx.z >> 1, upper = blockIdx.z & 1;
  const int o = 2 * h * pair;
  if (o + h >= p) return;
  const int nb = min(h, p - o - h);
  const C* LU = arena + f.off;
  C* XL = xwork + f.xoff;
  C* XU = XL + (int64_t)p * p;
  C* T = tbuf + f.xoff / 2;
  const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
  const int m0 = tm * kBM, n0 = tn * kBN;
  const int64_t oA = o, oB = o + h;
  if (!upper) {
    if (phase == 0) {   // TL (nb x h) = L(B, A) (nb x h) XL(A, A) (h x h, lower)
      if (m0 >= nb || n0 >= h) return;
      gemm_tile<R>(LU + oA * F + oB, F, XL + oA * p + oA, p, T + oA * p + oB, p, nb, h, h, m0, n0, false, R(1), n0, h);
    } else {            // XL(B, A) (nb x h) = -XL(B, B) (nb x nb, lower) TL (nb x h)
      if (m0 >= nb || n0 >= h) return;
      gemm_tile<R>(XL + oB * p + oB, p, T + oA * p + oB, p, XL + oA * p + oB, p, nb, h, nb, m0, n0, false, R(-1), 0,
                   m0 + kBM);
    }
  } else {
    if (phase == 0) {   // TU (h x nb) = U(A, B) (h x nb) XU(B, B) (nb x nb, upper)
      if (m0 >= h || n0 >= nb) return;
      gemm_tile<R>(LU + oB * F + oA, F, XU + oB * p + oB, p, T + oB * p + oA, p, h, nb, nb, m0, n0, false, R(1), 0,
                   n0 + kBN);
    } else {            // XU(A, B) (h x nb) = -XU(A, A) (h x h, upper) TU (h x nb)
      if (m0 >= h || n0 >= nb) return;
      gemm_tile<R>(XU + oA * p + oA, p, T + oB * p + oA, p, XU + oB * p + oA, p, h, nb, h, m0, n0, false, R(-1), m0, h);
    }
  }
}

// XL, XU of every front of a level: zero, with the diagonal 32 x 32 blocks
// taken from dinv.
template <typename R>
__global__ void inv_init_kernel(MfDev mf, cplx_t<R>* __restrict__ xwork, const cplx_t<R>* __restrict__ dinv, int f0) {
  using C = cplx_t<R>;
  const FrontDev& f = mf.fronts[f0 + blockIdx.y];
  const int p = f.p;
  const int64_t pp = (int64_t)p * p;
  C* X = xwork + f.xoff;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < pp; t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % p), j = (int)(t / p);
    C l = cmake<C>(0, 0), u = cmake<C>(0, 0);
    if (i / kDB == j / kDB) {
      const C* Li = dinv + (int64_t)2 * kDB * kDB * (f.dblk + j / kDB);
      const int bi = i % kDB, bj = j % kDB;
      l = Li[bj * kDB + bi];
      u = Li[kDB * kDB + bj * kDB + bi];
    }
    X[t] = l;
    X[pp + t] = u;
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

// Side blocks of the product form of the substitution, after XL = L11^{-1}
// (unit lower) and XU = U11^{-1} (upper):
//   Lt = L21 XL  ((F - p) x p, column-major, ld F - p)    blockIdx.z = 0
//   Ut = XU U12  (p x (F - p), column-major, ld p)        blockIdx.z = 1
// in the front's work slot after XL and XU; k is cut to the triangle.
template <typename R>
__global__ void __launch_bounds__(256, kGemmWaves<R>) inv_side_kernel(MfDev mf, const cplx_t<R>* __restrict__ arena,
                                                       cplx_t<R>* __restrict__ xwork, int f0, int tiles_m) {
  using C = cplx_t<R>;
  const FrontDev& f = mf.fronts[f0 + blockIdx.y];
  const int p = f.p, F = f.F, K = F - p;
  if (K <= 0 || p <= 0) return;
  const C* LU = arena + f.off;
  const C* XL = xwork + f.xoff;
  const C* XU = XL + (int64_t)p * p;
  C* Lt = xwork + f.xoff + 2 * (int64_t)p * p;
  C* Ut = Lt + (int64_t)K * p;
  const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
  const int m0 = tm * kBM, n0 = tn * kBN;
  if (blockIdx.z == 0) {
    if (m0 >= K || n0 >= p) return;
    gemm_tile<R>(LU + p, F, XL, p, Lt, K, K, p, p, m0, n0, false, R(1), n0, p);
  } else {
    if (m0 >= p || n0 >= K) return;
    gemm_tile<R>(XU, p, LU + (int64_t)p * F, F, Ut, p, p, K, p, m0, n0, false, R(1), m0, p);
  }
}

// Writes XL (strictly lower) and XU (upper) over the front's pivot block and,
// with side = true, Lt and Ut over L21 and U12.
template <typename R>
__global__ void merge_inverse_kernel(MfDev mf, cplx_t<R>* __restrict__ arena, const cplx_t<R>* __restrict__ xwork, int f0,
                                     bool side) {
  using C = cplx_t<R>;
  const FrontDev f = mf.fronts[f0 + blockIdx.y];
  const int p = f.p, F = f.F, K = F - p;
  const int64_t pp = (int64_t)p * p;
  const C* X = xwork + f.xoff;
  C* A = arena + f.off;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < pp; t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % p), j = (int)(t / p);
    A[(int64_t)j * F + i] = (i > j) ? X[t] : X[pp + t];
  }
  if (!side || K <= 0) return;
  const int64_t kp = (int64_t)K * p;
  const C* Lt = X + 2 * pp;
  const C* Ut = Lt + kp;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < kp; t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % K), j = (int)(t / K);
    A[(int64_t)j * F + p + i] = Lt[t];
    const int i2 = (int)(t % p), j2 = (int)(t / p);
    A[(int64_t)(p + j2) * F + i2] = Ut[t];
  }
}

// Final row permutation of each front's pivot block from the interchange
// record: one workgroup per front, the bookkeeping done in LDS.
// lds: the record and the permutation fit in LDS (2 p ints); else the
// interchanges are replayed in place in the global permutation array.
// compose: the interchanges moved whole rows to the tops of the 32-row
// blocks, and the diagonal-block LU then ordered each block's rows (prow);
// the final permutation is the replayed one read through prow (the ipiv
// record, no longer needed, holds the intermediate).
__global__ void perm_kernel(MfDev mf, int* __restrict__ ipiv, int f0, int lds, int compose) {
  const FrontDev f = mf.fronts[f0 + blockIdx.x];
  if (!lds) {
    int* perm = mf.perm + f.perm;
    for (int i = threadIdx.x; i < f.p; i += blockDim.x) perm[i] = i;
    __syncthreads();
    if (threadIdx.x == 0)
      for (int j = 0; j < f.p; ++j) {
        const int r = ipiv[f.perm + j];
        const int t = perm[j]; perm[j] = perm[r]; perm[r] = t;
      }
    __syncthreads();
    if (compose) {
      for (int i = threadIdx.x; i < f.p; i += blockDim.x) ipiv[f.perm + i] = perm[mf.prow[f.perm + i]];
      __syncthreads();
      for (int i = threadIdx.x; i < f.p; i += blockDim.x) perm[i] = ipiv[f.perm + i];
    }
    return;
  }
  extern __shared__ int sp[];
  int* perm = sp;
  int* piv = sp + f.p;
  for (int i = threadIdx.x; i < f.p; i += blockDim.x) { perm[i] = i; piv[i] = ipiv[f.perm + i]; }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int j = 0; j < f.p; ++j) {
      const int r = piv[j];
      const int t = perm[j]; perm[j] = perm[r]; perm[r] = t;
    }
  __syncthreads();
  for (int i = threadIdx.x; i < f.p; i += blockDim.x)
    mf.perm[f.perm + i] = compose ? perm[mf.prow[f.perm + i]] : perm[i];
}

// Inverses of the 32 x 32 diagonal blocks of a factored pivot block (L unit
// lower, U upper, rows in final pivot order) into their dinv slots, for the
// blocked substitution of levels factored with full partial pivoting (the
// block-local form writes them during the factorisation).  blockIdx.x =
// diagonal block, blockIdx.y = front.
template <typename R>
__global__ void __launch_bounds__(256) diag_inv_kernel(MfDev mf, const cplx_t<R>* __restrict__ arena,
                                                       cplx_t<R>* __restrict__ dinv, int f0) {
  using C = cplx_t<R>;
  const FrontDev& f = mf.fronts[f0 + blockIdx.y];
  const int k0 = blockIdx.x * kDB;
  if (k0 >= f.p) return;
  const int kb = min(kDB, f.p - k0);
  __shared__ DiagLds<R> S;
  const C* A = arena + f.off + (int64_t)k0 * f.F + k0;
  for (int t = threadIdx.x; t < kDB * kDB; t += 256) {
    const int c = t / kDB, i = t - c * kDB;
    S.X[i][c] = (i < kb && c < kb) ? A[(int64_t)c * f.F + i] : cmake<C>(i == c ? 1 : 0, 0);
  }
  __syncthreads();
  C* Li = dinv + (int64_t)2 * kDB * kDB * (f.dblk + k0 / kDB);
  tri_inv32<R>(S.X, Li, Li + kDB * kDB, kb);
}

// ------------------------------------------------------------------ Q apply
// (Q r)_S = r_S - T_S r_beta(S) for every set instance (Section 2.3).
// blockIdx = (instance of the set type, right-hand side x set type, problem);
// the set types cover disjoint points, so all of them go in one launch.
template <typename O>   // output: double2, or float2 for complex64 fronts
__global__ void q_apply_kernel(MfDev mf, const double2* __restrict__ r, O* __restrict__ y, int nrhs) {
  const InstDev& I = mf.inst[blockIdx.z];
  int anchors = 1;
  for (int i = 0; i < I.d; ++i) anchors *= I.m;
  const int anchor = blockIdx.x;
  if (anchor >= anchors) return;
  const int ntypes = 1 << I.d;
  const int type = blockIdx.y % ntypes, rhs = blockIdx.y / ntypes;
  const TypeDev& T = I.types[type];
  const int64_t base = I.Noff * nrhs + (int64_t)rhs * I.N;
  const double2* rr = r + base;
  O* yy = y + base;
  // Unknown u of a set list (point-major, nc per point) is component u % nc
  // of point u / nc: vector entry (u % nc) npts + point.
  const int nc = I.nc;
  auto at = [&](int u) {
    return (int64_t)(u % nc) * I.npts + anchor_point(I, anchor, T.off + (u / nc) * I.d);
  };
  extern __shared__ double2 rb[];
  for (int j = threadIdx.x; j < T.nB; j += blockDim.x) rb[j] = rr[at(T.nS + j)];
  __syncthreads();
  for (int i = threadIdx.x; i < T.nS; i += blockDim.x) {
    const int64_t g = at(i);
    double2 s = rr[g];
    if (std::is_same<O, float2>::value && T.Tt32) {   // (accumulated in FP64 all the same)
      for (int j = 0; j < T.nB; ++j) {
        const float2 a = T.Tt32[(int64_t)j * T.nS + i];
        cfms(s, make_double2(a.x, a.y), rb[j]);
      }
    } else {
      for (int j = 0; j < T.nB; ++j) cfms(s, T.Tt[(int64_t)j * T.nS + i], rb[j]);
    }
    yy[g].x = s.x;
    yy[g].y = s.y;
  }
}

// ------------------------------------------------------------------ solve
// Vectors per front: w and z arenas, position-major, nrhs consecutive values.
// w of every front of a level: x at the pivots, zero elsewhere, plus the
// children's boundary updates.  blockIdx.x = range of kGatherRows front
// positions (each workgroup applies the children's updates that land in its
// range, children in order, so the sums are deterministic), blockIdx.y = front.
constexpr int kGatherRows = 256;

template <typename R>
__global__ void fwd_gather_kernel(MfDev mf, cplx_t<R>* __restrict__ W, const cplx_t<R>* __restrict__ x, int nrhs, int f0) {
  using C = cplx_t<R>;
  const FrontDev f = mf.fronts[f0 + blockIdx.y];
  const int lo = blockIdx.x * kGatherRows, hi = min(f.F, lo + kGatherRows);
  if (lo >= hi) return;
  C* w = W + f.voff * nrhs;
  const int* idx = mf.idx + f.idx;
  const InstDev& I = mf.inst[f.inst];
  const C* xi = x + I.Noff * nrhs;
  for (int t = threadIdx.x; t < (hi - lo) * nrhs; t += blockDim.x) {
    const int i = lo + t / nrhs, r = t % nrhs;
    w[i * nrhs + r] = (i < f.p) ? xi[(int64_t)r * I.N + idx[i]] : cmake<C>(0, 0);
  }
  __syncthreads();
  const int* children = mf.fronts[f0 + blockIdx.y].child;   // global, indexed at run time
  for (int c = 0; c < f.nchild; ++c) {
    const FrontDev& ch = mf.fronts[children[c]];
    const int K = ch.F - ch.p;
    const int* map = mf.map + ch.map;
    const C* wc = W + (ch.voff + ch.p) * nrhs;
    for (int t = threadIdx.x; t < K * nrhs; t += blockDim.x) {
      const int i = t / nrhs, r = t - i * nrhs;
      const int pos = map[i];
      if (pos < lo || pos >= hi) continue;
      C& d = w[pos * nrhs + r];
      d = cadd(d, wc[t]);
    }
    __syncthreads();
  }
}

// Entry i of a front's vector before its own products: the right-hand side
// at a pivot position plus the boundary updates its children left for that
// position, added in child order (as fwd_gather_kernel adds them).
template <typename R>
__device__ inline cplx_t<R> gathered(const MfDev& mf, const FrontDev& f, const cplx_t<R>* __restrict__ W,
                                     const cplx_t<R>* __restrict__ xi, int64_t NI, int nrhs, int rr, int i) {
  using C = cplx_t<R>;
  C v = (i < f.p) ? xi[(int64_t)rr * NI + mf.idx[f.idx + i]] : cmake<C>(0, 0);
  const int b = mf.gptr[f.gptr + i], e = mf.gptr[f.gptr + i + 1];
  for (int t = b; t < e; ++t) v = cadd(v, W[mf.gsrc[t] * nrhs + rr]);
  return v;
}

// Row-tiled complex GEMV for the substitution products.
//  mode 0: z = Linv (P w_piv)            rows [0,p),  cols j < row (+ unit diagonal)
//  mode 1: w_bnd -= L21 z                rows [0,F-p), cols [0,p)
//  mode 2: z -= U12 x(bnd)               rows [0,p),  cols [0,F-p)
//  mode 3: x(piv) = Uinv z               rows [0,p),  cols j >= row
// With the side blocks of a front replaced by Lt = L21 Linv and Ut = Uinv U12
// (mf_factor_level does this for the levels solved by products), each
// direction is one product over the front's pivot columns or pivot rows:
//  mode 4: [z; w_bnd] = [Linv; -Lt] (P w_piv) + [0; w_bnd]
//          rows [0,F), cols j < min(row, p) (+ unit diagonal for rows < p)
//  mode 5: x(piv) = [Uinv, -Ut] [z; x(bnd)]  rows [0,p), cols [row, F)
// RT rows per workgroup: 64 (one row per lane, the four waves splitting the
// columns) or 16 (lanes 16 c + r take row r, sixteen column groups), the
// narrow form giving few-front levels four times the workgroups without
// splitting the columns.
template <typename R, int NR, int RT>
__global__ void __launch_bounds__(256) gemv_kernel(MfDev mf, const cplx_t<R>* __restrict__ arena, cplx_t<R>* __restrict__ W,
                                                   cplx_t<R>* __restrict__ Z, cplx_t<R>* __restrict__ xout, int nrhs,
                                                   int r0, int f0, int mode, int nchunks, cplx_t<R>* __restrict__ partial,
                                                   int prow, const cplx_t<R>* __restrict__ xin) {
  using C = cplx_t<R>;
  static_assert(RT == 64 || RT == 16, "row tiles of 64 or 16");
  constexpr int CG = 256 / RT;   // column groups of a workgroup
  const FrontDev f = mf.fronts[f0 + blockIdx.y];
  const int F = f.F, p = f.p;
  const int nrows = (mode == 1) ? F - p : (mode == 4) ? F : p;
  const int chunk = blockIdx.x % nchunks;
  const int row0 = (blockIdx.x / nchunks) * RT;
  if (row0 >= nrows) return;
  const int lane = threadIdx.x % RT, grp = threadIdx.x / RT;   // row in the tile, column group
  const int row = row0 + lane;
  const C* A = arena + f.foff;   // first p columns, leading dimension F
  const C* U = arena + f.uoff;   // U12, leading dimension ldu
  const int ldu = f.ldu;
  const int* idx = mf.idx + f.idx;
  const int* perm = mf.perm + f.perm;
  C* w = W + f.voff * nrhs;
  C* z = Z + f.voff * nrhs;
  const InstDev& I = mf.inst[f.inst];
  C* xo = xout + I.Noff * nrhs;
  const int64_t NI = I.N;
  int jlo, jhi;
  if (mode == 0 || mode == 4) { jlo = 0; jhi = min(p, row0 + RT); }
  else if (mode == 1) { jlo = 0; jhi = p; }
  else if (mode == 2) { jlo = 0; jhi = F - p; }
  else if (mode == 3) { jlo = row0; jhi = p; }
  else { jlo = row0; jhi = F; }
  if (nchunks > 1) {
    const int span = jhi - jlo, csz = (span + nchunks - 1) / nchunks;
    jlo = jlo + chunk * csz;
    jhi = min(jhi, jlo + csz);
  }
  C acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = cmake<C>(0, 0);
  const bool live = row < nrows;
  // Matrix column j of this product starts at A + coff + j * F (row offset
  // included); the vector entries of a tile of kVT columns are staged in LDS
  // first (their gathers go through perm / idx), so the main loop only streams
  // the matrix, several loads in flight per lane.
  // (U12 columns, mode 2 and the columns j >= p of mode 5, come from U.)
  const int64_t coff = (mode == 1) ? p + row : row;
  auto entry = [&](int j) {
    const bool use = live && j < jhi && ((mode == 0 || mode == 4) ? j < row : (mode == 3 || mode == 5) ? j >= row : true);
    if (!use) return cmake<C>(0, 0);
    if (mode == 2) return U[(int64_t)j * ldu + row];
    if (mode == 5 && j >= p) return U[(int64_t)(j - p) * ldu + row];
    return A[coff + (int64_t)j * F];
  };
  // Each wave's first kPre columns are loaded before the first tile's vector
  // entries are gathered, so that the two latencies overlap.
  constexpr int kPre = 8 / (NR == 4 ? 2 : 1) / (sizeof(R) == 8 ? 2 : 1);
  C apre[kPre];
#pragma unroll
  for (int u = 0; u < kPre; ++u) apre[u] = entry(jlo + grp + CG * u);
  const int orow = ((mode == 3 || mode == 5) && live) ? idx[row] : 0;
  // Mode 4 without split: the finishing step's gathered entries of the
  // tile's rows are staged with the first tile (by the threads beyond its
  // columns), not gathered after the products.
  const bool fin4 = mode == 4 && nchunks == 1;
  constexpr int kVT = 256;
  __shared__ C vs[kVT][NR];
  __shared__ C gs[RT][NR];
  for (int jt = jlo; jt < jhi || (fin4 && jt == jlo); jt += kVT) {
    const int jn = max(0, min(kVT, jhi - jt));
    const int nst = jn * NR + ((fin4 && jt == jlo) ? RT * NR : 0);
    for (int t = threadIdx.x; t < nst; t += 256) {
      if (t >= jn * NR) {
        const int u = t - jn * NR, l = u / NR, r = u - l * NR, i = row0 + l;
        if (r0 + r < nrhs && i < nrows)
          gs[l][r] = gathered<R>(mf, f, W, xin + I.Noff * nrhs, NI, nrhs, r0 + r, i < p ? perm[i] : i);
        continue;
      }
      const int jj = t / NR, r = t - jj * NR, j = jt + jj;
      C v = cmake<C>(0, 0);
      if (r0 + r < nrhs) {
        if (mode == 4) v = gathered<R>(mf, f, W, xin + I.Noff * nrhs, NI, nrhs, r0 + r, perm[j]);
        else if (mode == 0) v = w[perm[j] * nrhs + r0 + r];
        else if (mode == 2) v = xo[(int64_t)(r0 + r) * NI + idx[p + j]];
        else if (mode == 5 && j >= p) v = cneg(xo[(int64_t)(r0 + r) * NI + idx[j]]);
        else v = z[j * nrhs + r0 + r];
      }
      vs[jj][r] = v;
    }
    __syncthreads();
    int jj0 = grp;
    if (jt == jlo) {
#pragma unroll
      for (int u = 0; u < kPre; ++u) {
        const int jj = grp + CG * u;
        if (jj < jn)
#pragma unroll
          for (int r = 0; r < NR; ++r) cfma(acc[r], apre[u], vs[jj][r]);
      }
      jj0 = grp + CG * kPre;
    }
#pragma unroll 8
    for (int jj = jj0; jj < jn; jj += CG) {
      const C a = entry(jt + jj);
#pragma unroll
      for (int r = 0; r < NR; ++r) cfma(acc[r], a, vs[jj][r]);
    }
    __syncthreads();
  }
  __shared__ C red[CG][RT][NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) red[grp][lane][r] = acc[r];
  __syncthreads();
  if (grp != 0 || !live) return;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r0 + r >= nrhs) break;
    C s;
    if constexpr (CG == 4) {
      s = cadd(cadd(red[0][lane][r], red[1][lane][r]), cadd(red[2][lane][r], red[3][lane][r]));
    } else {   // (pairwise, in a fixed order)
      C h[CG / 2];
#pragma unroll
      for (int q = 0; q < CG / 2; ++q) h[q] = cadd(red[2 * q][lane][r], red[2 * q + 1][lane][r]);
#pragma unroll
      for (int w = CG / 4; w >= 1; w /= 2)
#pragma unroll
        for (int q = 0; q < w; ++q) h[q] = cadd(h[2 * q], h[2 * q + 1]);
      s = h[0];
    }
    const int rr = r0 + r;
    if (nchunks > 1) {
      partial[(((int64_t)blockIdx.y * nchunks + chunk) * prow + row) * nrhs + rr] = s;
    } else if (mode == 4 && row < p) {
      z[row * nrhs + rr] = cadd(s, gs[lane][r]);
    } else if (mode == 4) {
      w[row * nrhs + rr] = csub(gs[lane][r], s);
    } else if (mode == 0) {
      z[row * nrhs + rr] = cadd(s, w[perm[row] * nrhs + rr]);
    } else if (mode == 1) {
      C& d = w[(p + row) * nrhs + rr];
      d = csub(d, s);
    } else if (mode == 2) {
      C& d = z[row * nrhs + rr];
      d = csub(d, s);
    } else {
      xo[(int64_t)rr * NI + orow] = s;
    }
  }
}

// Whole-front substitution steps for levels with many small fronts (one
// workgroup per front, vectors in LDS, the pivot block kept in LU form).
//   forward:  w = gather(x, children's boundary updates); y = L11^{-1} P w_piv;
//             w_bnd -= L21 y; writes z = y and the updated w_bnd.
//   backward: y = z - U12 x_bnd; x_piv = U11^{-1} y.
// The triangular solves go in 32-row blocks: one wave solves the diagonal
// block with shuffles, the whole workgroup updates the rows beyond it.
constexpr int kTriBS = 32;
// Column loads in flight per thread in the strip products (more in FP32,
// where they cost half the registers).
template <typename R> constexpr int kStripUnroll = sizeof(R) == 4 ? 16 : 8;

template <typename R, int NR>
__device__ inline void fwd_front_body(const MfDev& mf, const cplx_t<R>* __restrict__ arena, cplx_t<R>* __restrict__ W,
                                      cplx_t<R>* __restrict__ Z, const cplx_t<R>* __restrict__ x, int nrhs, int r0,
                                      int fi) {
  using C = cplx_t<R>;
  constexpr int BS = kTriBS;
  const FrontDev& f = mf.fronts[fi];
  const int F = f.F, p = f.p;
  const C* A = arena + f.foff;   // first p columns of the factor, leading dimension F
  const int* perm = mf.perm + f.perm;
  const int* idx = mf.idx + f.idx;
  const InstDev& I = mf.inst[f.inst];
  const C* xi = x + I.Noff * nrhs;
  C* w = W + f.voff * nrhs;
  C* z = Z + f.voff * nrhs;
  const int nr = min(NR, nrhs - r0);
  __shared__ C D[BS][BS + 1];
  extern __shared__ unsigned char smem[];
  C* wv = reinterpret_cast<C*>(smem);   // F x NR: the front vector
  C* y = wv + F * NR;                   // p x NR: permuted pivot part, solved in place
  // Each thread's entries of the next diagonal block (strictly lower part),
  // loaded while the previous block's strip update runs and stored to LDS
  // after it (workgroups of 256 threads).
  constexpr int kDP = BS * BS / 256;
  C dpre[kDP];
  auto fetch_d = [&](int b) {
    const int n = min(BS, p - b);
#pragma unroll
    for (int u = 0; u < kDP; ++u) {
      const int t = threadIdx.x + 256 * u, jj = t / BS, i = t - jj * BS;
      dpre[u] = (i < n && jj < n && i > jj) ? A[(int64_t)(b + jj) * F + b + i] : cmake<C>(0, 0);
    }
  };
  auto store_d = [&] {
#pragma unroll
    for (int u = 0; u < kDP; ++u) {
      const int t = threadIdx.x + 256 * u, jj = t / BS, i = t - jj * BS;
      D[i][jj] = dpre[u];
    }
  };
  fetch_d(0);
  for (int t = threadIdx.x; t < F * NR; t += blockDim.x) {
    const int i = t / NR, r = t - i * NR;
    wv[t] = (i < p && r < nr) ? xi[(int64_t)(r0 + r) * I.N + idx[i]] : cmake<C>(0, 0);
  }
  __syncthreads();
  for (int c = 0; c < f.nchild; ++c) {
    const FrontDev& ch = mf.fronts[f.child[c]];
    const int Kc = ch.F - ch.p;
    const int* map = mf.map + ch.map;
    const C* wc = W + (ch.voff + ch.p) * nrhs;
    for (int t = threadIdx.x; t < Kc * NR; t += blockDim.x) {
      const int i = t / NR, r = t - i * NR;
      if (r < nr) {
        C& d = wv[map[i] * NR + r];
        d = cadd(d, wc[(int64_t)i * nrhs + r0 + r]);
      }
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < p * NR; t += blockDim.x) {
    const int i = t / NR, r = t - i * NR;
    y[t] = wv[perm[i] * NR + r];
  }
  store_d();
  __syncthreads();
  const int lane = threadIdx.x & 63;
  for (int b0 = 0; b0 < p; b0 += BS) {
    const int bs = min(BS, p - b0);
    if (threadIdx.x < 64) {
      C yi[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) yi[r] = (lane < bs) ? y[(b0 + lane) * NR + r] : cmake<C>(0, 0);
      // Column jj of the block: y_jj is final in lane jj, read as a scalar.
#pragma unroll
      for (int jj = 0; jj < BS; ++jj) {
        if (jj < bs) {
          // D is zero on and above the diagonal and below row bs.
          const C l = (lane < BS) ? D[lane][jj] : cmake<C>(0, 0);
#pragma unroll
          for (int r = 0; r < NR; ++r) cfms(yi[r], l, lane_read(yi[r], jj));
        }
      }
      if (lane < bs)
#pragma unroll
        for (int r = 0; r < NR; ++r) y[(b0 + lane) * NR + r] = yi[r];
    }
    __syncthreads();
    if (b0 + BS < p) fetch_d(b0 + BS);
    // The block's columns applied to every row below it: the rest of the
    // pivot block (y) and the boundary rows (w_bnd -= L21 y, a strip at a time).
    for (int i = b0 + bs + threadIdx.x; i < F; i += blockDim.x) {
      C* v = (i < p) ? y + i * NR : wv + i * NR;
      C acc[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[r] = v[r];
#pragma unroll kStripUnroll<R>
      for (int jj = 0; jj < bs; ++jj) {
        const C l = A[(int64_t)(b0 + jj) * F + i];
#pragma unroll
        for (int r = 0; r < NR; ++r) cfms(acc[r], l, y[(b0 + jj) * NR + r]);
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) v[r] = acc[r];
    }
    if (b0 + BS < p) store_d();   // (the solve has read this block's D)
    __syncthreads();
  }
  for (int t = threadIdx.x; t < F * NR; t += blockDim.x) {
    const int i = t / NR, r = t - i * NR;
    if (r >= nr) continue;
    if (i < p) z[i * nrhs + r0 + r] = y[t];
    else w[i * nrhs + r0 + r] = wv[t];
  }
}

template <typename R, int NR>
__device__ inline void bwd_front_body(const MfDev& mf, const cplx_t<R>* __restrict__ arena,
                                      const cplx_t<R>* __restrict__ Z, cplx_t<R>* __restrict__ xout, int nrhs, int r0,
                                      int fi) {
  using C = cplx_t<R>;
  constexpr int BS = kTriBS;
  const FrontDev& f = mf.fronts[fi];
  const int F = f.F, p = f.p, K = F - p;
  const C* A = arena + f.foff;   // pivot block (first p columns, leading dimension F)
  const C* U = arena + f.uoff;   // U12, leading dimension ldu
  const int ldu = f.ldu;
  const int* idx = mf.idx + f.idx;
  const C* z = Z + f.voff * nrhs;
  const InstDev& I = mf.inst[f.inst];
  C* xo = xout + I.Noff * nrhs;
  const int nr = min(NR, nrhs - r0);
  __shared__ C D[BS][BS + 1];   // strictly upper part of the diagonal block
  __shared__ C Dd[BS];          // its diagonal
  extern __shared__ unsigned char smem[];
  C* y = reinterpret_cast<C*>(smem);    // p x NR
  C* xb = y + p * NR;                   // K x NR: solution at the boundary points
  // Each thread's entries of the next diagonal block (upper part with the
  // diagonal), loaded while the previous step runs and stored to LDS after it
  // (workgroups of 256 threads).
  constexpr int kDP = BS * BS / 256;
  C dpre[kDP];
  auto fetch_d = [&](int b) {
    const int n = min(BS, p - b);
#pragma unroll
    for (int u = 0; u < kDP; ++u) {
      const int t = threadIdx.x + 256 * u, jj = t / BS, i = t - jj * BS;
      dpre[u] = (i < n && jj < n && i <= jj) ? A[(int64_t)(b + jj) * F + b + i] : cmake<C>(0, 0);
    }
  };
  auto store_d = [&] {
#pragma unroll
    for (int u = 0; u < kDP; ++u) {
      const int t = threadIdx.x + 256 * u, jj = t / BS, i = t - jj * BS;
      D[i][jj] = (i == jj) ? cmake<C>(0, 0) : dpre[u];
      if (i == jj) Dd[i] = dpre[u];
    }
  };
  fetch_d(((p - 1) / BS) * BS);
  for (int t = threadIdx.x; t < p * NR; t += blockDim.x) {
    const int i = t / NR, r = t - i * NR;
    y[t] = (r < nr) ? z[i * nrhs + r0 + r] : cmake<C>(0, 0);
  }
  for (int t = threadIdx.x; t < K * NR; t += blockDim.x) {
    const int j = t / NR, r = t - j * NR;
    xb[t] = (r < nr) ? xo[(int64_t)(r0 + r) * I.N + idx[p + j]] : cmake<C>(0, 0);
  }
  __syncthreads();
  // y -= U12 x_bnd
  for (int i = threadIdx.x; i < p; i += blockDim.x) {
    C acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = y[i * NR + r];
#pragma unroll kStripUnroll<R>
    for (int j = 0; j < K; ++j) {
      const C u = U[(int64_t)j * ldu + i];
#pragma unroll
      for (int r = 0; r < NR; ++r) cfms(acc[r], u, xb[j * NR + r]);
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) y[i * NR + r] = acc[r];
  }
  store_d();
  __syncthreads();
  const int lane = threadIdx.x & 63;
  for (int b0 = ((p - 1) / BS) * BS; b0 >= 0; b0 -= BS) {
    const int bs = min(BS, p - b0);
    if (threadIdx.x < 64) {
      C yi[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) yi[r] = (lane < bs) ? y[(b0 + lane) * NR + r] : cmake<C>(0, 0);
      // Column jj from the last: x_jj = y_jj / u_jj in lane jj, read as a scalar.
#pragma unroll
      for (int jj = BS - 1; jj >= 0; --jj) {
        if (jj < bs) {
          const C u = (lane < BS) ? D[lane][jj] : cmake<C>(0, 0);   // zero from the diagonal down
          const C d = Dd[jj];
          const C dinv = cabs2(d) > 0 ? crecip(d) : cmake<C>(0, 0);
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const C xj = cmul(lane_read(yi[r], jj), dinv);
            if (lane == jj) yi[r] = xj;
            cfms(yi[r], u, xj);
          }
        }
      }
      if (lane < bs)
#pragma unroll
        for (int r = 0; r < NR; ++r) y[(b0 + lane) * NR + r] = yi[r];
    }
    __syncthreads();
    if (b0 > 0) fetch_d(b0 - BS);
    for (int i = threadIdx.x; i < b0; i += blockDim.x) {
      C acc[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[r] = y[i * NR + r];
#pragma unroll kStripUnroll<R>
      for (int jj = 0; jj < bs; ++jj) {
        const C u = A[(int64_t)(b0 + jj) * F + i];
#pragma unroll
        for (int r = 0; r < NR; ++r) cfms(acc[r], u, y[(b0 + jj) * NR + r]);
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) y[i * NR + r] = acc[r];
    }
    if (b0 > 0) store_d();   // (the solve has read this block's D)
    __syncthreads();
  }
  for (int t = threadIdx.x; t < p * NR; t += blockDim.x) {
    const int i = t / NR, r = t - i * NR;
    if (r < nr) xo[(int64_t)(r0 + r) * I.N + idx[i]] = y[t];
  }
}

template <typename R, int NR>
__global__ void __launch_bounds__(256) fwd_front_kernel(MfDev mf, const cplx_t<R>* __restrict__ arena,
                                                        cplx_t<R>* __restrict__ W, cplx_t<R>* __restrict__ Z,
                                                        const cplx_t<R>* __restrict__ x, int nrhs, int r0, int f0) {
  fwd_front_body<R, NR>(mf, arena, W, Z, x, nrhs, r0, f0 + blockIdx.x);
}

template <typename R, int NR>
__global__ void __launch_bounds__(256) bwd_front_kernel(MfDev mf, const cplx_t<R>* __restrict__ arena,
                                                        const cplx_t<R>* __restrict__ Z, cplx_t<R>* __restrict__ xout,
                                                        int nrhs, int r0, int f0) {
  bwd_front_body<R, NR>(mf, arena, Z, xout, nrhs, r0, f0 + blockIdx.x);
}

// Persistent form of the whole-front kernels for a run of consecutive
// small-front levels: one cooperative launch whose workgroups stride over the
// fronts of a level, with a grid-wide barrier between levels (forward: leaves
// up; backward: top down).  The runtime guarantees that all workgroups of a
// cooperative launch are resident, so the barrier always completes.
constexpr int kMaxRunLevels = 16;
struct LevelRun {
  int nlev;
  int begin[kMaxRunLevels + 1];
};

template <typename R, int NR, bool FWD>
__global__ void __launch_bounds__(256) front_levels_kernel(MfDev mf, const cplx_t<R>* __restrict__ arena,
                                                           cplx_t<R>* __restrict__ W, cplx_t<R>* __restrict__ Z,
                                                           const cplx_t<R>* __restrict__ x, cplx_t<R>* __restrict__ xout,
                                                           int nrhs, int r0, LevelRun run) {
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  for (int t = 0; t < run.nlev; ++t) {
    const int l = FWD ? t : run.nlev - 1 - t;
    for (int fi = run.begin[l] + blockIdx.x; fi < run.begin[l + 1]; fi += gridDim.x) {
      if (FWD) fwd_front_body<R, NR>(mf, arena, W, Z, x, nrhs, r0, fi);
      else bwd_front_body<R, NR>(mf, arena, Z, xout, nrhs, r0, fi);
      __syncthreads();
    }
    grid.sync();
  }
}

// ------------------------------------------------------------------ factor store
// Streamed storage: after a level is factored, each front's factor part goes
// from its F x F working front to the compact store: the first p columns
// (L11 / U11 and L21, F rows each) to foff with leading dimension F, and
// the U12 rows [0, p) of columns [p, F) to uoff with leading dimension p.
// blockIdx.x = chunk of cols_per_wg columns, blockIdx.y = front.
template <typename R>
__global__ void __launch_bounds__(256) factor_store_kernel(MfDev mf, const cplx_t<R>* __restrict__ arena,
                                                           cplx_t<R>* __restrict__ store, int f0, int cols_per_wg) {
  const FrontDev& f = mf.fronts[f0 + blockIdx.y];
  const int j0 = blockIdx.x * cols_per_wg;
  if (j0 >= f.F) return;
  const int j1 = min(f.F, j0 + cols_per_wg);
  const cplx_t<R>* A = arena + f.off;
  for (int j = j0; j < j1; ++j) {
    const cplx_t<R>* src = A + (int64_t)j * f.F;
    if (j < f.p) {
      cplx_t<R>* dst = store + f.foff + (int64_t)j * f.F;
      for (int i = threadIdx.x; i < f.F; i += blockDim.x) dst[i] = src[i];
    } else {
      cplx_t<R>* dst = store + f.uoff + (int64_t)(j - f.p) * f.ldu;
      for (int i = threadIdx.x; i < f.p; i += blockDim.x) dst[i] = src[i];
    }
  }
}

// ------------------------------------------------------------------ blocked substitution
// Levels of a few large fronts keep their LU in place and go through the
// pivot rows in 32-row block steps, each step one launch over all fronts of
// the level: every workgroup forms the block's solution from the 32 x 32
// inverse the diagonal-block LU left in dinv (a product of 32 x 32 by the
// block's vector, repeated per workgroup instead of a separate launch),
// and applies the block's columns to its own tile of 256 rows.
//   forward (lower, unit diagonal, rows in pivot order):
//     blk_perm:  z_piv = P w_piv   (w: the gathered front vector)
//     step k:    y_k = Linv_kk z_k;  z_i -= L_ik y_k for rows i beyond block k
//                (y_k kept in w's pivot part, copied to z after the last step)
//     then w_bnd -= L21 z (gemv_kernel mode 1)
//   backward (upper), after z -= U12 x_bnd (gemv_kernel mode 2):
//     step k (last block first): x_k = Uinv_kk z_k, written to the grid
//                vector; z_i -= U_ik x_k for rows i before block k.
template <typename R>
__global__ void blk_perm_kernel(MfDev mf, const cplx_t<R>* __restrict__ W, cplx_t<R>* __restrict__ Z, int nrhs,
                                int f0, int copy_back) {
  const FrontDev& f = mf.fronts[f0 + blockIdx.y];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= f.p * nrhs) return;
  const int i = t / nrhs, r = t - i * nrhs;
  const int src = copy_back ? i : mf.perm[f.perm + i];
  Z[(f.voff + i) * nrhs + r] = W[(f.voff + src) * nrhs + r];
}

constexpr int kBlkRows = 256;

template <typename R, int NR, bool FWD>
__global__ void __launch_bounds__(256) blk_step_kernel(MfDev mf, const cplx_t<R>* __restrict__ fac,
                                                       const cplx_t<R>* __restrict__ dinv, cplx_t<R>* __restrict__ W,
                                                       cplx_t<R>* __restrict__ Z, cplx_t<R>* __restrict__ xout,
                                                       int nrhs, int r0, int f0, int k0) {
  using C = cplx_t<R>;
  const FrontDev& f = mf.fronts[f0 + blockIdx.y];
  const int F = f.F, p = f.p;
  if (k0 >= p) return;
  const int kb = min(kDB, p - k0);
  // rows of this workgroup: beyond the block (forward) or before it (backward)
  const int rlo = FWD ? k0 + kb : 0, rhi = FWD ? p : k0;
  const int row0 = rlo + blockIdx.x * kBlkRows;
  if (blockIdx.x > 0 && row0 >= rhi) return;
  const int nr = min(NR, nrhs - r0);
  const C* Dk = dinv + (int64_t)2 * kDB * kDB * (f.dblk + k0 / kDB) + (FWD ? 0 : kDB * kDB);
  C* z = Z + f.voff * nrhs;
  __shared__ C zk[kDB][NR];
  __shared__ C ys[kDB][NR];
  const int tid = threadIdx.x;
  if (tid < kDB * NR) {
    const int i = tid / NR, r = tid - i * NR;
    zk[i][r] = (i < kb && r < nr) ? z[(k0 + i) * nrhs + r0 + r] : cmake<C>(0, 0);
  }
  __syncthreads();
  if (tid < kDB * NR) {
    // y_i = sum_c inv(i, c) zk_c over the block (column-major 32 x 32; the
    // entries beyond kb are not set, so the sum stops at kb)
    const int i = tid / NR, r = tid - i * NR;
    C acc = cmake<C>(0, 0);
    if (i < kb)
      for (int c = 0; c < kb; ++c) cfma(acc, Dk[c * kDB + i], zk[c][r]);
    ys[i][r] = acc;
  }
  __syncthreads();
  if (blockIdx.x == 0 && tid < kb * NR) {
    const int i = tid / NR, r = tid - i * NR;
    if (r < nr) {
      if (FWD) {
        W[(f.voff + k0 + i) * nrhs + r0 + r] = ys[i][r];
      } else {
        const InstDev& I = mf.inst[f.inst];
        xout[I.Noff * nrhs + (int64_t)(r0 + r) * I.N + mf.idx[f.idx + k0 + i]] = ys[i][r];
      }
    }
  }
  const int row = row0 + tid;
  if (row >= rhi) return;
  const C* A = fac + f.foff + (int64_t)k0 * F + row;   // column k0 + c at A + c F
  C acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = (r < nr) ? z[row * nrhs + r0 + r] : cmake<C>(0, 0);
#pragma unroll 8
  for (int c = 0; c < kb; ++c) {
    const C a = A[(int64_t)c * F];
#pragma unroll
    for (int r = 0; r < NR; ++r) cfms(acc[r], a, ys[c][r]);
  }
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (r < nr) z[row * nrhs + r0 + r] = acc[r];
}

// Sums the split-K partial products of gemv_kernel and applies the mode's
// finishing step (see gemv_kernel).
template <typename R>
__global__ void gemv_finish_kernel(MfDev mf, cplx_t<R>* __restrict__ W, cplx_t<R>* __restrict__ Z,
                                   cplx_t<R>* __restrict__ xout, int nrhs, int f0, int mode, int nchunks,
                                   const cplx_t<R>* __restrict__ partial, int prow, const cplx_t<R>* __restrict__ xin) {
  using C = cplx_t<R>;
  const FrontDev f = mf.fronts[f0 + blockIdx.y];
  const int nrows = (mode == 1) ? f.F - f.p : (mode == 4) ? f.F : f.p;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows * nrhs) return;
  const int row = t / nrhs, rr = t - row * nrhs;
  C* w = W + f.voff * nrhs;
  C* z = Z + f.voff * nrhs;
  const InstDev& I = mf.inst[f.inst];
  // (mode 4: the gathered entry's dependent loads go out before the partial sums)
  const C g = (mode == 4) ? gathered<R>(mf, f, W, xin + I.Noff * nrhs, I.N, nrhs, rr,
                                        row < f.p ? mf.perm[f.perm + row] : row)
                          : cmake<C>(0, 0);
  C s = cmake<C>(0, 0);
  for (int c = 0; c < nchunks; ++c)
    s = cadd(s, partial[(((int64_t)blockIdx.y * nchunks + c) * prow + row) * nrhs + rr]);
  if (mode == 4 && row < f.p) {
    z[row * nrhs + rr] = cadd(s, g);
  } else if (mode == 4) {
    w[row * nrhs + rr] = csub(g, s);
  } else if (mode == 0) {
    z[row * nrhs + rr] = cadd(s, w[mf.perm[f.perm + row] * nrhs + rr]);
  } else if (mode == 1) {
    C& d = w[(f.p + row) * nrhs + rr];
    d = csub(d, s);
  } else if (mode == 2) {
    C& d = z[row * nrhs + rr];
    d = csub(d, s);
  } else {
    xout[I.Noff * nrhs + (int64_t)rr * I.N + mf.idx[f.idx + row]] = s;
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
constexpr int kOuterNB = 256;   // columns per outer block of the tournament-pivoted levels

}  // namespace

template <typename R>
void mf_factor_level(hipStream_t st, const MfDev& mf, void* arena_v, void* xwork_v, void* tbuf_v, void* dinv_v,
                     int* tpbuf, int f0, int f1, int maxF, int maxP, int blk0, int blk1, int max_children, int form,
                     int pivoting, int variant, const int* hF, const int* hP, hipStream_t inv_st,
                     hipEvent_t lu_done) {
  const bool partial_pivoting = pivoting == kPivotPartial;
  const bool tournament = pivoting == kPivotTournament;
  const bool pair_steps = (variant & kVarPair) != 0;
  const bool tile64 = (variant & kVarTile64) != 0;
  const bool fused = (variant & kVarFused) != 0 && !pair_steps && !partial_pivoting && !tournament;
  const bool invert = form == kFormInverse || form == kFormSide;
  using C = cplx_t<R>;
  C* arena = static_cast<C*>(arena_v);
  C* xwork = static_cast<C*>(xwork_v);
  C* dinv = static_cast<C*>(dinv_v);
  const int nf = f1 - f0;
  // (a level without children takes its fronts' largest entries from the
  // assembly itself)
  const bool norm_in_assembly = max_children == 0 && !partial_pivoting;
  if (blk1 > blk0) {
    assemble_kernel<R><<<blk1 - blk0, 256, 0, st>>>(mf, arena, blk0, norm_in_assembly ? 1 : 0);
    SPP_LAUNCH_CHECK();
  }
  for (int s = 0; s < max_children; ++s) {
    const int cols = 4;
    dim3 grid(ceil_div(maxF, cols), nf);
    extend_add_kernel<R><<<grid, 256, 0, st>>>(mf, arena, f0, s, cols);
    SPP_LAUNCH_CHECK();
  }
  if (!partial_pivoting && !norm_in_assembly) {
    const int64_t chunk = 16384;
    front_norm_kernel<R><<<dim3((unsigned)ceil_div((int64_t)maxF * maxF, chunk), nf), 256, 0, st>>>(mf, arena, f0,
                                                                                                   chunk);
    SPP_LAUNCH_CHECK();
  }
  const int steps = (maxP + kNB - 1) / kNB;
  const int tiles = (int)ceil_div(maxF, kBM);
  const int tiles128 = (int)ceil_div(maxF, 128);   // tall / wide tiles of modes 3 and 7
  auto gemm_timed = [&](double fl, auto&& launch) {
    timer_begin(KC_GEMM, st);
    launch();
    SPP_LAUNCH_CHECK();
    timer_end(KC_GEMM, st, 0.0, fl);
  };
  if (tournament) {
    // Outer blocks of kOuterNB columns: inside one, each 32-column block
    // takes the earlier blocks' updates on its column strip, has its pivot
    // rows chosen by the tournament and swapped up, takes the updates on its
    // row strip, then its diagonal-block LU and L21 / U12; the outer block's
    // trailing update then goes as one rank-kOuterNB product.
    const int maxsets = (int)ceil_div(maxP, kTpRows);
    int* bufA = tpbuf;
    int* bufB = tpbuf + (size_t)nf * maxsets * kDB;
    for (int k0 = 0; k0 < maxP; k0 += kOuterNB) {
      for (int c = k0; c < std::min(maxP, k0 + kOuterNB); c += kNB) {
        const int s = c / kNB;
        double fl8 = 0, fl9 = 0, fl7 = 0;
        if (g_timer)
          for (int i = 0; i < nf; ++i) {
            if (c >= hP[i]) continue;
            const double kb = std::min(kNB, hP[i] - c), m = hF[i] - c - kb, w = c - k0;
            fl8 += 8.0 * (m + kb) * kb * w;
            fl9 += 8.0 * kb * m * w;
            fl7 += 16.0 * m * kb * kb;
          }
        if (c > k0)
          gemm_timed(fl8, [&] {
            gemm_kernel<R, 8><<<dim3(tiles128, nf), 256, 0, st>>>(mf, arena, xwork, dinv, f0, s, kNB, tiles128, k0);
          });
        timer_begin(KC_PANEL, st);
        int sets = (int)ceil_div(maxP - c, kTpRows);
        tp_select_kernel<R><<<dim3(sets, nf), 256, 0, st>>>(mf, arena, bufA, f0, c, maxsets);
        SPP_LAUNCH_CHECK();
        int* in = bufA;
        int* out = bufB;
        for (int lev = 1; sets > 1; ++lev) {
          const int next = (int)ceil_div(sets, kTpFan);
          tp_reduce_kernel<R><<<dim3(next, nf), 256, 0, st>>>(mf, arena, in, out, f0, c, lev, maxsets);
          SPP_LAUNCH_CHECK();
          std::swap(in, out);
          sets = next;
        }
        tp_swap_kernel<R><<<dim3(ceil_div(maxF, 64), nf), 64, 0, st>>>(mf, arena, in, mf.ipiv, f0, c, maxsets);
        SPP_LAUNCH_CHECK();
        timer_end(KC_PANEL, st, 0.0, 0.0);
        if (c > k0)
          gemm_timed(fl9, [&] {
            gemm_kernel<R, 9><<<dim3(2 * tiles128, nf), 256, 0, st>>>(mf, arena, xwork, dinv, f0, s, kNB, tiles128,
                                                                       k0);
          });
        timer_begin(KC_PANEL, st);
        diag_lu_kernel<R><<<nf, 256, 0, st>>>(mf, arena, dinv, f0, c, kNB);
        SPP_LAUNCH_CHECK();
        timer_end(KC_PANEL, st, 0.0, 0.0);
        gemm_timed(fl7, [&] {
          gemm_kernel<R, 7><<<dim3(2 * tiles128, nf), 256, 0, st>>>(mf, arena, xwork, dinv, f0, s, kNB, tiles128);
        });
      }
      double flt = 0;
      if (g_timer)
        for (int i = 0; i < nf; ++i) {
          if (k0 >= hP[i]) continue;
          const double w = std::min(kOuterNB, hP[i] - k0), mn = hF[i] - k0 - w;
          flt += 8.0 * mn * mn * w;
        }
      gemm_timed(flt, [&] {
        gemm_kernel<R, 0><<<dim3(tiles * tiles, nf), 256, 0, st>>>(mf, arena, xwork, dinv, f0, k0 / kOuterNB,
                                                                   kOuterNB, tiles);
      });
    }
  }
  if (!partial_pivoting && !tournament && steps > 0) {
    // First diagonal block; each later one is factored inside the previous
    // step's trailing-update launch (levels of few fronts) or on its own.
    timer_begin(KC_PANEL, st);
    diag_lu_kernel<R><<<nf, 256, 0, st>>>(mf, arena, dinv, f0, 0, kNB);
    SPP_LAUNCH_CHECK();
    timer_end(KC_PANEL, st, 0.0, 0.0);
  }
  // L21 / U12 of one step: 64 x 64 tiles (mode 6) or 128 x 32 / 32 x 128
  // tiles (mode 7), as the level's variant says.
  auto l21_u12 = [&](int s, double fl) {
    gemm_timed(fl, [&] {
      if (tile64)
        gemm_kernel<R, 6><<<dim3(2 * tiles, nf), 256, 0, st>>>(mf, arena, xwork, dinv, f0, s, kNB, tiles);
      else
        gemm_kernel<R, 7><<<dim3(2 * tiles128, nf), 256, 0, st>>>(mf, arena, xwork, dinv, f0, s, kNB, tiles128);
    });
  };
  // Paired steps (wide levels by default: many fronts fill the device, and
  // their trailing updates move the front through HBM at every step): the
  // second block's column and row take the first step's update on their
  // own, then one rank-64 trailing update serves both steps, halving that
  // traffic.
  if (!partial_pivoting && !tournament && pair_steps) {
    // One kernel per timed interval (bench.py divides a class's time by its
    // intervals): L21 / U12 of each step 16 m kb^2, the second block's
    // column and row 8 kb kb2 (m + m - kb2), the trailing update 8 mn^2 w.
    for (int s = 0; s < steps;) {
      const int k0 = s * kNB;
      const bool pair = s + 1 < steps;
      double fl7a = 0, fl7b = 0, fln = 0, flt = 0;
      if (g_timer)
        for (int i = 0; i < nf; ++i) {
          if (k0 >= hP[i]) continue;
          const double kb = std::min(kNB, hP[i] - k0), m = hF[i] - k0 - kb;
          const double kb2 = pair ? std::max(0, std::min(kNB, hP[i] - k0 - kNB)) : 0;
          const double w = kb + kb2, mn = hF[i] - k0 - w;
          fl7a += 16.0 * m * kb * kb;
          fl7b += 16.0 * (m - kb2) * kb2 * kb2;
          fln += 8.0 * kb * kb2 * (m + (m - kb2));
          flt += 8.0 * mn * mn * w;
        }
      if (s > 0) {
        timer_begin(KC_PANEL, st);
        diag_lu_kernel<R><<<nf, 256, 0, st>>>(mf, arena, dinv, f0, k0, kNB);
        SPP_LAUNCH_CHECK();
        timer_end(KC_PANEL, st, 0.0, 0.0);
      }
      l21_u12(s, fl7a);
      if (pair) {
        gemm_timed(fln, [&] {
          gemm_kernel<R, 3><<<dim3(2 * tiles128, nf), 256, 0, st>>>(mf, arena, xwork, dinv, f0, s, kNB, tiles128);
        });
        timer_begin(KC_PANEL, st);
        diag_lu_kernel<R><<<nf, 256, 0, st>>>(mf, arena, dinv, f0, k0 + kNB, kNB);
        SPP_LAUNCH_CHECK();
        timer_end(KC_PANEL, st, 0.0, 0.0);
        l21_u12(s + 1, fl7b);
        gemm_timed(flt, [&] {
          gemm_kernel<R, 0><<<dim3(tiles * tiles, nf), 256, 0, st>>>(mf, arena, xwork, dinv, f0, s / 2, 2 * kNB,
                                                                     tiles);
        });
        s += 2;
      } else {
        gemm_timed(flt, [&] {
          gemm_kernel<R, 0><<<dim3(tiles * tiles, nf), 256, 0, st>>>(mf, arena, xwork, dinv, f0, s, kNB, tiles);
        });
        s += 1;
      }
    }
  }
  for (int s = 0; s < steps && fused; ++s) {
    // Trailing update of step s (8 mn^2 kb per front) and the L21 / U12 of
    // step s - 1 (16 m kb^2), one launch (gemm_fused_kernel).
    const int k0 = s * kNB;
    double fl = 0;
    if (g_timer)
      for (int i = 0; i < nf; ++i) {
        if (k0 < hP[i]) {
          const double kb = std::min(kNB, hP[i] - k0), mn = hF[i] - k0 - kb;
          fl += 8.0 * mn * mn * kb;
        }
        if (s > 0 && k0 - kNB < hP[i]) {
          const double kb = std::min(kNB, hP[i] - (k0 - kNB)), m = hF[i] - (k0 - kNB) - kb;
          fl += 16.0 * m * kb * kb;
        }
      }
    const int ndiag = s + 1 < steps ? 1 : 0, nwb = s > 0 ? 2 * tiles : 0;
    gemm_timed(fl, [&] {
      gemm_fused_kernel<R><<<dim3(ndiag + nwb + tiles * tiles, nf), 256, 0, st>>>(mf, arena, xwork, dinv, f0, s, kNB,
                                                                                  tiles, ndiag, nwb);
    });
  }
  if (fused && steps > 0) {   // the last step's L21 / U12
    const int k0 = (steps - 1) * kNB;
    double fl = 0;
    if (g_timer)
      for (int i = 0; i < nf; ++i) {
        if (k0 >= hP[i]) continue;
        const double kb = std::min(kNB, hP[i] - k0), m = hF[i] - k0 - kb;
        fl += 16.0 * m * kb * kb;
      }
    l21_u12(steps - 1, fl);
  }
  for (int s = 0; s < steps && !tournament && !fused && (partial_pivoting || !pair_steps); ++s) {
    const int k0 = s * kNB;
    if (partial_pivoting) {
      timer_begin(KC_PANEL, st);
      // Pivot search over all remaining fully-summed rows of the column.
      if (maxF <= 512) panel2_kernel<R, 256, 2><<<nf, 256, 0, st>>>(mf, arena, mf.ipiv, f0, k0, kNB);
      else if (maxF <= 1024) panel2_kernel<R, 512, 2><<<nf, 512, 0, st>>>(mf, arena, mf.ipiv, f0, k0, kNB);
      else if (maxF <= 2048) panel2_kernel<R, 512, 4><<<nf, 512, 0, st>>>(mf, arena, mf.ipiv, f0, k0, kNB);
      else if (maxF <= 4096) panel2_kernel<R, 1024, 4><<<nf, 1024, 0, st>>>(mf, arena, mf.ipiv, f0, k0, kNB);
      else panel_kernel<R><<<nf, 256, 0, st>>>(mf, arena, mf.ipiv, f0, k0, kNB, 0);
      SPP_LAUNCH_CHECK();
      timer_end(KC_PANEL, st, 0.0, 0.0);
      if (maxF <= 4096) {   // (the global-memory panel applies its interchanges itself)
        laswp_kernel<R><<<dim3(ceil_div(maxF, 64), nf), 64, 0, st>>>(mf, arena, mf.ipiv, f0, k0, kNB);
        SPP_LAUNCH_CHECK();
      }
      trsm_kernel<R><<<dim3(ceil_div(maxF, 256), nf), 256, 0, st>>>(mf, arena, xwork, f0, s, kNB, 0);
    } else {
      // L21 = A21 Uinv_kk and U12 = Linv_kk P A12 on MFMA in one launch (one
      // tile strip each); the block's row order P is applied while loading
      // A12, the rows' L parts are reordered once after the last step.
      // 16 m kb^2 real flops per front (m = F - k0 - kb rows and columns).
      double fl = 0;
      if (g_timer)
        for (int i = 0; i < nf; ++i) {
          if (k0 >= hP[i]) continue;
          const double kb = std::min(kNB, hP[i] - k0), m = hF[i] - k0 - kb;
          fl += 16.0 * m * kb * kb;
        }
      l21_u12(s, fl);
    }
    SPP_LAUNCH_CHECK();
    {
      // Trailing updates of this step, 8 m n k real flops per front.
      double fl = 0;
      if (g_timer)
        for (int i = 0; i < nf; ++i) {
          if (k0 >= hP[i]) continue;
          const double kb = std::min(kNB, hP[i] - k0), mn = hF[i] - k0 - kb;
          fl += 8.0 * mn * mn * kb;
        }
      timer_begin(KC_GEMM, st);
      // Single steps take the next diagonal block into the trailing launch
      // (the step's serial part overlaps the update).
      if (!partial_pivoting && s + 1 < steps)
        gemm_next_kernel<R><<<dim3(tiles * tiles + 1, nf), 256, 0, st>>>(mf, arena, xwork, dinv, f0, s, kNB, tiles);
      else
        gemm_kernel<R, 0><<<dim3(tiles * tiles, nf), 256, 0, st>>>(mf, arena, xwork, dinv, f0, s, kNB, tiles);
      SPP_LAUNCH_CHECK();
      timer_end(KC_GEMM, st, 0.0, fl);
    }
  }
  if (!partial_pivoting && steps > 1) {
    const int cchunks = (int)ceil_div(maxP, 64);
    leftswap_kernel<R><<<dim3(steps * cchunks, nf), 256, 0, st>>>(mf, arena, f0, cchunks);
    SPP_LAUNCH_CHECK();
  }
  if (partial_pivoting || tournament) {   // (the block-local LU writes the permutation itself)
    const bool lds = (size_t)2 * sizeof(int) * maxP <= 65536;
    perm_kernel<<<nf, 256, lds ? 2 * sizeof(int) * maxP : 0, st>>>(mf, mf.ipiv, f0, lds ? 1 : 0, tournament ? 1 : 0);
    SPP_LAUNCH_CHECK();
    if (form == kFormBlocked && partial_pivoting) {
      diag_inv_kernel<R><<<dim3(ceil_div(maxP, kDB), nf), 256, 0, st>>>(mf, arena, dinv, f0);
      SPP_LAUNCH_CHECK();
    }
  }
  if (!invert) return;
  // Inverses of L11 and U11 for levels solved by matrix-vector products
  // (on inv_st after the LU, where the caller runs them beside the next
  // level; block-locally pivoted levels only).
  if (inv_st && lu_done && !partial_pivoting && !tournament) {
    SPP_HIP(hipEventRecord(lu_done, st));
    SPP_HIP(hipStreamWaitEvent(inv_st, lu_done, 0));
    st = inv_st;
  }
  const int ptiles = (int)ceil_div(maxP, kBM);
  if (!partial_pivoting) {
    inv_init_kernel<R><<<dim3(ceil_div((int64_t)maxP * maxP, 256 * 4), nf), 256, 0, st>>>(mf, xwork, dinv, f0);
    SPP_LAUNCH_CHECK();
    C* tbuf = static_cast<C*>(tbuf_v);
    for (int h = kDB; h < maxP; h *= 2) {
      const int pairs = (int)ceil_div(maxP, 2 * h);
      const int ht = (int)ceil_div(h, kBM);
      double fl = 0;
      if (g_timer)
        for (int i = 0; i < nf; ++i)
          for (int o = 0; o + h < hP[i]; o += 2 * h) {
            const double nbv = std::min(h, hP[i] - o - h);
            fl += 2 * 8.0 * nbv * h * (h + nbv) / 2;   // both triangles, products cut to the nonzero half
          }
      for (int phase = 0; phase < 2; ++phase) {   // (the two phases have equal flops)
        timer_begin(KC_INV, st);
        inv_gemm_kernel<R><<<dim3(ht * ht, nf, 2 * pairs), 256, 0, st>>>(mf, arena, xwork, tbuf, f0, h, phase, ht);
        SPP_LAUNCH_CHECK();
        timer_end(KC_INV, st, 0.0, fl / 2);
      }
    }
  } else {
    identity_kernel<R><<<dim3(ceil_div((int64_t)maxP * maxP, 256 * 4), nf), 256, 0, st>>>(mf, xwork, f0);
    SPP_LAUNCH_CHECK();
    for (int mode = 1; mode <= 2; ++mode) {
      for (int s = 0; s < steps; ++s) {
        trsm_kernel<R><<<dim3(ceil_div(maxP, 256), nf), 256, 0, st>>>(mf, arena, xwork, f0, s, kNB, mode);
        SPP_LAUNCH_CHECK();
        if (mode == 1)
          gemm_kernel<R, 1><<<dim3(ptiles * ptiles, nf), 256, 0, st>>>(mf, arena, xwork, dinv, f0, s, kNB, ptiles);
        else
          gemm_kernel<R, 2><<<dim3(ptiles * ptiles, nf), 256, 0, st>>>(mf, arena, xwork, dinv, f0, s, kNB, ptiles);
        SPP_LAUNCH_CHECK();
      }
    }
  }
  // Lt = L21 XL and Ut = XU U12 replace the side blocks, so that each
  // substitution direction is one product per front (gemv modes 4 and 5).
  int maxK = 0;
  if (form == kFormSide)
    for (int i = 0; i < nf; ++i) maxK = std::max(maxK, hF[i] - hP[i]);
  if (maxK > 0) {
    // 8 (F - p) p^2 real flops per front (two products cut to the triangle).
    double fl = 0;
    if (g_timer)
      for (int i = 0; i < nf; ++i) fl += 8.0 * (hF[i] - hP[i]) * (double)hP[i] * hP[i];
    const int tiles_m = (int)ceil_div(std::max(maxK, maxP), kBM);
    timer_begin(KC_INV, st);
    inv_side_kernel<R><<<dim3(tiles_m * tiles_m, nf, 2), 256, 0, st>>>(mf, arena, xwork, f0, tiles_m);
    SPP_LAUNCH_CHECK();
    timer_end(KC_INV, st, 0.0, fl);
  }
  const int64_t merge_items = std::max<int64_t>((int64_t)maxP * maxP, (int64_t)maxK * maxP);
  merge_inverse_kernel<R><<<dim3(ceil_div(merge_items, 256 * 4), nf), 256, 0, st>>>(mf, arena, xwork, f0, maxK > 0);
  SPP_LAUNCH_CHECK();
}

int mf_level_solve_form(int nfronts, int maxF, int maxP, bool c64, bool streamed) {
  // Explicit inverses turn every substitution step into row-parallel
  // matrix-vector products (many workgroups per front).  Building them costs
  // setup time: cheap on FP32 MFMA (complex64 fronts: always), dearer on
  // FP64, where levels with very many small fronts keep the LU in place and
  // run one workgroup per front (its vectors, (F + p) x 4 complex values,
  // within 64 KB of LDS).
  if (nfronts >= 512 && maxP <= 512 && (int64_t)(maxF + maxP) * 4 * (c64 ? 8 : 16) <= 65536) return kFormLU;
  // Large pivot blocks: their inverse work (2 p F per front) would rival the
  // factor itself, so they keep the LU and go in block steps.
  if (maxP > (streamed ? 1024 : 4096)) return kFormBlocked;
  // The side products Lt = L21 Linv and Ut = Uinv U12 halve the launches per
  // level and direction; they pay where the level's products are short
  // (few fronts: launch latency dominates), not on the wide leaf levels,
  // whose substitution already streams at full width.
  return nfronts < 512 ? kFormSide : kFormInverse;
}

void q_apply(hipStream_t st, const MfDev& mf, const double2* r, void* y, int nrhs, bool to_float) {
  const int ntypes = 1 << mf.d;
  int nb = 0;
  for (int t = 0; t < ntypes; ++t) nb = std::max(nb, mf.nB_max[t]);
  timer_begin(KC_QAPPLY, st);
  dim3 grid((unsigned)mf.anchors_max, nrhs * ntypes, mf.ninst);
  if (to_float)
    q_apply_kernel<float2><<<grid, 256, sizeof(double2) * nb, st>>>(mf, r, static_cast<float2*>(y), nrhs);
  else
    q_apply_kernel<double2><<<grid, 256, sizeof(double2) * nb, st>>>(mf, r, static_cast<double2*>(y), nrhs);
  SPP_LAUNCH_CHECK();
  timer_end(KC_QAPPLY, st, 32.0 * mf.Ntot * nrhs, 0.0);
}

int gemv_chunks_default(int rows, int cols, int nf, int nrhs, int64_t partial_cap) {
  const int rtiles = (int)ceil_div(rows, 64);
  int nchunks = 1;
  if ((int64_t)rtiles * nf < 1024) {
    nchunks = (int)std::min<int64_t>(std::max(1, cols / 64), 2048 / ((int64_t)rtiles * nf));
    if (nchunks < 1) nchunks = 1;
  }
  while (nchunks > 1 && (int64_t)nf * nchunks * rows * nrhs > partial_cap) --nchunks;
  return nchunks;
}

namespace {
__global__ void reset_status_kernel(MfDev mf, int nfronts) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nfronts) mf.fnorm[t] = 0u;
  if (t == 0) {
    mf.info[0] = 0;
    mf.info[9] = 0;
    mf.info[10] = 0;
    mf.pstat[0] = 0u;            // largest growth
    mf.pstat[1] = 0x7f7fffffu;   // smallest pivot ratio: FLT_MAX
  }
}
}  // namespace

void mf_reset_status(hipStream_t st, const MfDev& mf, int nfronts) {
  reset_status_kernel<<<(unsigned)ceil_div(std::max(nfronts, 1), 256), 256, 0, st>>>(mf, nfronts);
  SPP_LAUNCH_CHECK();
}

std::string gemv_tune_key(int rows, int cols, int nf, int mode, int nrhs, int csize) {
  return tune_key("gemv_chunks", {rows, cols, nf, mode, nrhs, csize});
}

// Row-tiled products; large fronts split their columns over nchunks
// workgroups (deterministic partial sums, then gemv_finish_kernel).
template <typename R>
void mf_gemv(hipStream_t st, const MfDev& mf, const void* arena_v, void* W_v, void* Z_v, void* xout_v, const void* xin_v,
             int nrhs, int f0, int nf, int rows, int cols, int mode, double ent, void* partial_v, int64_t partial_cap,
             int nchunks) {
  using C = cplx_t<R>;
  const C* arena = static_cast<const C*>(arena_v);
  C* W = static_cast<C*>(W_v);
  C* Z = static_cast<C*>(Z_v);
  C* xout = static_cast<C*>(xout_v);
  const C* xin = static_cast<const C*>(xin_v);
  C* partial = static_cast<C*>(partial_v);
  if (nchunks < 0)
    nchunks = tune_get(gemv_tune_key(rows, cols, nf, mode, nrhs, (int)sizeof(C)),
                       gemv_chunks_default(rows, cols, nf, nrhs, partial_cap));
  // (0: 16-row tiles, columns not split; kGemvNarrowSplit + c: 16-row tiles,
  // columns split c ways; else 64-row tiles, columns split nchunks ways)
  bool narrow = nchunks == 0;
  if (nchunks >= kGemvNarrowSplit) {
    narrow = true;
    nchunks -= kGemvNarrowSplit;
  }
  const int rt = narrow ? 16 : 64;
  const int rtiles = (int)ceil_div(rows, rt);
  nchunks = std::max(1, std::min(nchunks, std::max(1, cols)));
  while (nchunks > 1 && (int64_t)nf * nchunks * rows * nrhs > partial_cap) --nchunks;
  dim3 grid(rtiles * nchunks, nf);
  // ent: factor entries of the level read per pass over the right-hand sides.
  const double passes = (nrhs / 4) + (nrhs % 4);
  timer_begin(KC_GEMV, st);
  int r0 = 0;
  while (r0 < nrhs) {
    if (nrhs - r0 >= 4) {
      if (narrow)
        gemv_kernel<R, 4, 16><<<grid, 256, 0, st>>>(mf, arena, W, Z, xout, nrhs, r0, f0, mode, nchunks, partial, rows,
                                                    xin);
      else
        gemv_kernel<R, 4, 64><<<grid, 256, 0, st>>>(mf, arena, W, Z, xout, nrhs, r0, f0, mode, nchunks, partial, rows,
                                                    xin);
      r0 += 4;
    } else {
      if (narrow)
        gemv_kernel<R, 1, 16><<<grid, 256, 0, st>>>(mf, arena, W, Z, xout, nrhs, r0, f0, mode, nchunks, partial, rows,
                                                    xin);
      else
        gemv_kernel<R, 1, 64><<<grid, 256, 0, st>>>(mf, arena, W, Z, xout, nrhs, r0, f0, mode, nchunks, partial, rows,
                                                    xin);
      r0 += 1;
    }
    SPP_LAUNCH_CHECK();
  }
  if (nchunks > 1) {
    gemv_finish_kernel<R><<<dim3(ceil_div((int64_t)rows * nrhs, 256), nf), 256, 0, st>>>(
        mf, W, Z, xout, nrhs, f0, mode, nchunks, partial, rows, xin);
    SPP_LAUNCH_CHECK();
  }
  timer_end(KC_GEMV, st, ent * passes * sizeof(C), 8.0 * ent * nrhs);
}

template <typename R>
void mf_solve(hipStream_t st, const MfDev& mf, const void* arena_v, void* w_v, void* z_v, const void* x_in,
              void* x_out, int nrhs, const int* level_begin, const int* level_maxF, const int* level_maxK,
              const int* level_maxP, const double* level_ent, const int* level_form, int nlevels, void* partial_v,
              int64_t partial_cap, bool persistent, hipEvent_t* level_events, hipEvent_t inv_early,
              hipEvent_t inv_last) {
  using C = cplx_t<R>;
  // level_events (tuning): events 4 l and 4 l + 1 bracket level l's forward
  // part, 4 l + 2 and 4 l + 3 its backward part (levels one at a time).
  if (level_events) persistent = false;
  struct Mark {   // records its event (if any) when the level's iteration ends
    hipEvent_t e;
    hipStream_t s;
    ~Mark() {
      if (e) (void)hipEventRecord(e, s);
    }
  };
  auto ev = [&](int l, int which) { return level_events ? level_events[4 * l + which] : nullptr; };
  const C* arena = static_cast<const C*>(arena_v);
  C* W = static_cast<C*>(w_v);
  C* Z = static_cast<C*>(z_v);
  const C* xin = static_cast<const C*>(x_in);
  C* xout = static_cast<C*>(x_out);
  C* partial = static_cast<C*>(partial_v);
  // Row-tiled products; large fronts split their columns over several
  // workgroups (deterministic partial sums, then gemv_finish_kernel).
  auto gemv = [&](int f0, int nf, int rows, int cols, int mode, double ent) {
    mf_gemv<R>(st, mf, arena, W, Z, xout, xin, nrhs, f0, nf, rows, cols, mode, ent, partial, partial_cap, -1);
  };
  // Whole-front kernels of the levels solved with the LU in place.
  auto front = [&](int f0, int nf, int maxF, int maxP, int maxK, bool fwd, double ent) {
    const double passes = (nrhs / 4) + (nrhs % 4);
    timer_begin(KC_TRI, st);
    int r0 = 0;
    while (r0 < nrhs) {
      const int nr = (nrhs - r0 >= 4) ? 4 : 1;
      if (fwd) {
        const size_t lds = sizeof(C) * (size_t)(maxF + maxP) * nr;
        if (nr == 4) fwd_front_kernel<R, 4><<<nf, 256, lds, st>>>(mf, arena, W, Z, xin, nrhs, r0, f0);
        else fwd_front_kernel<R, 1><<<nf, 256, lds, st>>>(mf, arena, W, Z, xin, nrhs, r0, f0);
      } else {
        const size_t lds = sizeof(C) * (size_t)(maxP + maxK) * nr;
        if (nr == 4) bwd_front_kernel<R, 4><<<nf, 256, lds, st>>>(mf, arena, Z, xout, nrhs, r0, f0);
        else bwd_front_kernel<R, 1><<<nf, 256, lds, st>>>(mf, arena, Z, xout, nrhs, r0, f0);
      }
      SPP_LAUNCH_CHECK();
      r0 += nr;
    }
    timer_end(KC_TRI, st, ent * passes * sizeof(C), 8.0 * ent * nrhs);
  };
  // Blocked levels: 32-row block steps (blk_step_kernel).  Forward: gather,
  // permute into z, the steps (solutions kept in w's pivot part), copy back.
  auto blocked = [&](int f0, int nf, int maxF, int maxP, int maxK, bool fwd, double ent) {
    const C* dk = static_cast<const C*>(mf.dkeep);
    const int pt = (int)ceil_div((int64_t)maxP * nrhs, 256);
    if (fwd) {
      fwd_gather_kernel<R><<<dim3(ceil_div(maxF, kGatherRows), nf), 256, 0, st>>>(mf, W, xin, nrhs, f0);
      SPP_LAUNCH_CHECK();
      blk_perm_kernel<R><<<dim3(pt, nf), 256, 0, st>>>(mf, W, Z, nrhs, f0, 0);
      SPP_LAUNCH_CHECK();
    }
    const double passes = (nrhs / 4) + (nrhs % 4);
    timer_begin(KC_SOLVE_BLK, st);
    const int nblk = (maxP + kDB - 1) / kDB;
    for (int s = 0; s < nblk; ++s) {
      const int k0 = (fwd ? s : nblk - 1 - s) * kDB;
      const int rows = fwd ? maxP - k0 - kDB : k0;
      const unsigned gx = (unsigned)std::max<int64_t>(1, ceil_div(std::max(rows, 1), kBlkRows));
      int r0 = 0;
      while (r0 < nrhs) {
        const int nr = (nrhs - r0 >= 4) ? 4 : 1;
        if (fwd) {
          if (nr == 4) blk_step_kernel<R, 4, true><<<dim3(gx, nf), 256, 0, st>>>(mf, arena, dk, W, Z, xout, nrhs, r0, f0, k0);
          else blk_step_kernel<R, 1, true><<<dim3(gx, nf), 256, 0, st>>>(mf, arena, dk, W, Z, xout, nrhs, r0, f0, k0);
        } else {
          if (nr == 4) blk_step_kernel<R, 4, false><<<dim3(gx, nf), 256, 0, st>>>(mf, arena, dk, W, Z, xout, nrhs, r0, f0, k0);
          else blk_step_kernel<R, 1, false><<<dim3(gx, nf), 256, 0, st>>>(mf, arena, dk, W, Z, xout, nrhs, r0, f0, k0);
        }
        SPP_LAUNCH_CHECK();
        r0 += nr;
      }
    }
    timer_end(KC_SOLVE_BLK, st, ent * passes * sizeof(C), 8.0 * ent * nrhs);
    if (fwd) {
      blk_perm_kernel<R><<<dim3(pt, nf), 256, 0, st>>>(mf, W, Z, nrhs, f0, 1);
      SPP_LAUNCH_CHECK();
    }
  };
  // A run of consecutive small-front levels [l0, l1) as one cooperative launch
  // (false if it does not apply: too many levels, too much LDS, or the device
  // cannot hold enough workgroups).
  auto front_run = [&](int l0, int l1, bool fwd) {
    if (!persistent || l1 - l0 < 2 || l1 - l0 > kMaxRunLevels) return false;
    LevelRun run;
    run.nlev = l1 - l0;
    int mF = 0, mP = 0, mK = 0, mN = 0;
    double ent = 0;
    for (int l = l0; l < l1; ++l) {
      run.begin[l - l0] = level_begin[l];
      mF = std::max(mF, level_maxF[l]);
      mP = std::max(mP, level_maxP[l]);
      mK = std::max(mK, level_maxK[l]);
      mN = std::max(mN, level_begin[l + 1] - level_begin[l]);
      ent += fwd ? level_ent[3 * l] + level_ent[3 * l + 2] : level_ent[3 * l + 1] + level_ent[3 * l + 2];
    }
    run.begin[run.nlev] = level_begin[l1];
    const size_t lds_row = sizeof(C) * (size_t)(fwd ? mF + mP : mP + mK);
    if (lds_row * (nrhs >= 4 ? 4 : 1) > 65536) return false;
    int dev = 0, cus = 0;
    SPP_HIP(hipGetDevice(&dev));
    SPP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    auto kernel_of = [&](int nr) {
      return fwd ? (nr == 4 ? (const void*)front_levels_kernel<R, 4, true> : (const void*)front_levels_kernel<R, 1, true>)
                 : (nr == 4 ? (const void*)front_levels_kernel<R, 4, false> : (const void*)front_levels_kernel<R, 1, false>);
    };
    for (int nr : {1, 4}) {
      if (nr == 4 && nrhs < 4) continue;
      int per_cu = 0;
      SPP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel_of(nr), 256, lds_row * nr));
      if (per_cu < 1) return false;
    }
    const double passes = (nrhs / 4) + (nrhs % 4);
    timer_begin(KC_TRI, st);
    int r0 = 0;
    while (r0 < nrhs) {
      const int nr = (nrhs - r0 >= 4) ? 4 : 1;
      const void* f = kernel_of(nr);
      int per_cu = 0;
      SPP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, 256, lds_row * nr));
      const unsigned grid = (unsigned)std::min<int64_t>((int64_t)per_cu * cus, mN);
      MfDev mfv = mf;
      const C* a = arena;
      C* w = W;
      C* z = Z;
      const C* xi = xin;
      C* xo = xout;
      int nrhs_v = nrhs, r0_v = r0;
      void* args[] = {&mfv, &a, &w, &z, &xi, &xo, &nrhs_v, &r0_v, &run};
      SPP_HIP(hipLaunchCooperativeKernel(f, dim3(grid), dim3(256), args, (unsigned)(lds_row * nr), st));
      r0 += nr;
    }
    timer_end(KC_TRI, st, ent * passes * sizeof(C), 8.0 * ent * nrhs);
    return true;
  };
  // level_ent per level: sum over fronts of p (p - 1) / 2, p (p + 1) / 2 and (F - p) p.
  for (int l = 0; l < nlevels; ++l) {
    const int f0 = level_begin[l], nf = level_begin[l + 1] - f0;
    const int mK = level_maxK[l], mP = level_maxP[l];
    const double* e = level_ent + 3 * l;
    if (level_form[l] == kFormInverse || level_form[l] == kFormSide) {
      hipEvent_t& w = (l == nlevels - 1) ? inv_last : inv_early;
      if (w) SPP_HIP(hipStreamWaitEvent(st, w, 0));
      w = nullptr;
    }
    if (level_events) SPP_HIP(hipEventRecord(ev(l, 0), st));
    const Mark done{ev(l, 1), st};
    if (level_form[l] == kFormLU) {
      int l1 = l + 1;
      while (l1 < nlevels && level_form[l1] == kFormLU) ++l1;
      if (front_run(l, l1, true)) {
        l = l1 - 1;
        continue;
      }
      front(f0, nf, level_maxF[l], mP, mK, true, e[0] + e[2]);
      continue;
    }
    if (level_form[l] == kFormBlocked) {
      blocked(f0, nf, level_maxF[l], mP, mK, true, e[0]);
      if (mK > 0) gemv(f0, nf, mK, mP, 1, e[2]);
      continue;
    }
    if (level_form[l] == kFormSide) {
      gemv(f0, nf, level_maxF[l], mP, 4, e[0] + e[2]);   // gathers its own input
    } else {
      fwd_gather_kernel<R><<<dim3(ceil_div(level_maxF[l], kGatherRows), nf), 256, 0, st>>>(mf, W, xin, nrhs, f0);
      SPP_LAUNCH_CHECK();
      gemv(f0, nf, mP, mP, 0, e[0]);
      if (mK > 0) gemv(f0, nf, mK, mP, 1, e[2]);
    }
  }
  for (int l = nlevels - 1; l >= 0; --l) {
    const int f0 = level_begin[l], nf = level_begin[l + 1] - f0;
    const int mK = level_maxK[l], mP = level_maxP[l];
    const double* e = level_ent + 3 * l;
    if (level_events) SPP_HIP(hipEventRecord(ev(l, 2), st));
    const Mark done{ev(l, 3), st};
    if (level_form[l] == kFormLU) {
      int l0 = l;
      while (l0 > 0 && level_form[l0 - 1] == kFormLU) --l0;
      if (front_run(l0, l + 1, false)) {
        l = l0;
        continue;
      }
      front(f0, nf, level_maxF[l], mP, mK, false, e[1] + e[2]);
      continue;
    }
    if (level_form[l] == kFormBlocked) {
      if (mK > 0) gemv(f0, nf, mP, mK, 2, e[2]);
      blocked(f0, nf, level_maxF[l], mP, mK, false, e[1]);
      continue;
    }
    if (level_form[l] == kFormSide) {
      gemv(f0, nf, mP, level_maxF[l], 5, e[1] + e[2]);
    } else {
      if (mK > 0) gemv(f0, nf, mP, mK, 2, e[2]);
      gemv(f0, nf, mP, mP, 3, e[1]);
    }
  }
}

template <typename R>
void mf_store_factors(hipStream_t st, const MfDev& mf, const void* arena, void* store, int f0, int nf, int maxF) {
  const int cols = 4;
  factor_store_kernel<R><<<dim3(ceil_div(maxF, cols), nf), 256, 0, st>>>(
      mf, static_cast<const cplx_t<R>*>(arena), static_cast<cplx_t<R>*>(store), f0, cols);
  SPP_LAUNCH_CHECK();
}

template <typename R>
void cast_vectors(hipStream_t st, const void* in, void* out, int64_t count, int to_double) {
  if (count <= 0) return;
  cast_kernel<R><<<ceil_div(count, 256), 256, 0, st>>>(in, out, count, to_double);
  SPP_LAUNCH_CHECK();
}

template void mf_factor_level<double>(hipStream_t, const MfDev&, void*, void*, void*, void*, int*, int, int, int, int, int, int,
                                      int, int, int, int, const int*, const int*, hipStream_t, hipEvent_t);
template void mf_factor_level<float>(hipStream_t, const MfDev&, void*, void*, void*, void*, int*, int, int, int, int, int, int,
                                     int, int, int, int, const int*, const int*, hipStream_t, hipEvent_t);
template void mf_solve<double>(hipStream_t, const MfDev&, const void*, void*, void*, const void*, void*, int,
                               const int*, const int*, const int*, const int*, const double*, const int*, int, void*,
                               int64_t, bool, hipEvent_t*, hipEvent_t, hipEvent_t);
template void mf_solve<float>(hipStream_t, const MfDev&, const void*, void*, void*, const void*, void*, int,
                              const int*, const int*, const int*, const int*, const double*, const int*, int, void*,
                              int64_t, bool, hipEvent_t*, hipEvent_t, hipEvent_t);
template void mf_gemv<double>(hipStream_t, const MfDev&, const void*, void*, void*, void*, const void*, int, int, int, int, int, int,
                              double, void*, int64_t, int);
template void mf_gemv<float>(hipStream_t, const MfDev&, const void*, void*, void*, void*, const void*, int, int, int, int, int, int,
                             double, void*, int64_t, int);
template void mf_store_factors<double>(hipStream_t, const MfDev&, const void*, void*, int, int, int);
template void mf_store_factors<float>(hipStream_t, const MfDev&, const void*, void*, int, int, int);
template void cast_vectors<double>(hipStream_t, const void*, void*, int64_t, int);
template void cast_vectors<float>(hipStream_t, const void*, void*, int64_t, int);

}  // namespace spp
