// Setup kernels: the shift split (eq. Dsq), the Fourier symbol of G (eq. G),
// and the sparsifying stencils T_S and C_S of Section 2.3.
//
// T_S = G(S, gamma^c) G(beta, gamma^c)^+ is computed without forming the
// N-wide blocks: for a full-row-rank A = G(beta, gamma^c) the pseudoinverse is
// A^H (A A^H)^{-1}, and both products it needs are sums over gamma^c, i.e. a
// sum over the whole grid minus a sum over gamma:
//   G(X, gamma^c) G(Y, gamma^c)^H = (G G^H)(X, Y) - G(X, gamma) G(Y, gamma)^H.
// G is the circulant with symbol sigma_k, so G G^H is the circulant with
// symbol |sigma_k|^2, and for real sigma G(Y, gamma)^H = G(gamma, Y).  (A
// vector field's G has a real symmetric d x d symbol per wave vector: the
// same holds over its unknowns, with G G^H of symbol G(k)^2.)  Hence
//   T_S [ (G G^H)(beta, beta) - G(beta, gamma) G(gamma, beta) ]
//       = (G G^H)(S, beta) - G(S, gamma) G(gamma, beta),
// an |beta| x |beta| system, and C_S = [I  -T_S] G(gamma, gamma).
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace spp {

namespace {

constexpr int kRedThreads = 256;

__device__ inline double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  __syncthreads();
  return r;
}

// w of eq. (Dsq): Helmholtz (0) omega^2 / c^2, Schroedinger (1) ell^2 V,
// Maxwell (2) omega^2 eps.
__device__ inline double coeff_w(int kind, double c, double omega, double ell) {
  return kind == 0 ? omega * omega / (c * c) : kind == 2 ? omega * omega * c : ell * ell * c;
}

__global__ void coeff_partial_kernel(int kind, const double* __restrict__ coeff, int64_t N,
                                     double omega, double ell, double* __restrict__ partial) {
  __shared__ double sh[16];
  double sum = 0, bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double c = coeff[i];
    const double w = coeff_w(kind, c, omega, ell);
    if (!isfinite(c) || !isfinite(w) || (kind != 1 && !(c > 0))) bad += 1;
    else sum += w;
  }
  const double s = block_sum(sum, sh);
  const double b = block_sum(bad, sh);
  if (threadIdx.x == 0) { partial[2 * blockIdx.x] = s; partial[2 * blockIdx.x + 1] = b; }
}

__global__ void coeff_final_kernel(const double* __restrict__ partial, int nblocks, double* out) {
  __shared__ double sh[16];
  double s = 0, b = 0;
  for (int i = threadIdx.x; i < nblocks; i += blockDim.x) { s += partial[2 * i]; b += partial[2 * i + 1]; }
  s = block_sum(s, sh);
  b = block_sum(b, sh);
  if (threadIdx.x == 0) { out[0] = s; out[1] = b; }
}

__global__ void coeff_finish_kernel(int kind, const double* __restrict__ coeff, int64_t N, int d, int n,
                                    double omega, double ell, double energy, double s,
                                    double* __restrict__ q, double* __restrict__ sigma,
                                    double2* __restrict__ sig_c, double2* __restrict__ sig2_c) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= N) return;
  const double w = coeff_w(kind, coeff[j], omega, ell);
  // Helmholtz and Maxwell: q = s - w.  Schroedinger: q = ell^2 V - ell^2 E + s.
  q[j] = (kind == 1) ? w - ell * ell * energy + s : s - w;
  int64_t r = j;
  double k2 = 0;
  for (int i = 0; i < d; ++i) {
    int ri = (int)(r % n);
    r /= n;
    int k = (ri >= n / 2) ? ri - n : ri;
    k2 += (double)k * k;
  }
  const double pi = 3.14159265358979323846;
  const double sg = 1.0 / (4.0 * pi * pi * k2 - s) / (double)N;   // sigma_k / N
  sigma[j] = sg;
  sig_c[j] = cmake<double2>(sg, 0.0);
  sig2_c[j] = cmake<double2>(sg * sg * (double)N, 0.0);         // |sigma_k|^2 / N
}

// Maxwell (Section 4 extension): the d x d symbol of G = (curl curl - s)^{-1}
// and of G G^H = G^2 per wave vector, / N, as nc^2 grids (component pair
// (a, b) at (a nc + b) N).  curl is built from first derivatives, whose wave
// numbers drop the Nyquist index: kt_a = k_a, 0 at r_a = n/2.  Then
// G(k) = (I - kt kt^T / |kt|^2) / (4 pi^2 |kt|^2 - s) - kt kt^T / (|kt|^2 s),
// and -I / s where kt = 0.
__global__ void maxwell_symbol_kernel(int d, int n, int64_t N, double s, double2* __restrict__ sig,
                                      double2* __restrict__ sig2) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= N) return;
  double kt[3] = {0, 0, 0};
  int64_t r = j;
  for (int a = d - 1; a >= 0; --a) {   // C order: the last axis is fastest
    const int ra = (int)(r % n);
    r /= n;
    kt[a] = (ra == n / 2) ? 0.0 : (double)((ra > n / 2) ? ra - n : ra);
  }
  double k2 = 0;
  for (int a = 0; a < d; ++a) k2 += kt[a] * kt[a];
  const double pi = 3.14159265358979323846;
  const double trans = 1.0 / (4.0 * pi * pi * k2 - s);
  double G[3][3];
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      const double proj = k2 > 0 ? kt[a] * kt[b] / k2 : 0.0;
      G[a][b] = ((a == b ? 1.0 : 0.0) - proj) * trans - proj / s;
    }
  const double inv_n = 1.0 / (double)N;
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      double g2 = 0;
      for (int c = 0; c < d; ++c) g2 += G[a][c] * G[c][b];
      sig[(int64_t)(a * d + b) * N + j] = cmake<double2>(G[a][b] * inv_n, 0.0);
      sig2[(int64_t)(a * d + b) * N + j] = cmake<double2>(g2 * inv_n, 0.0);
    }
}

// G-type block gather over the unknowns of a set's point list, point-major
// (unknown u = point u / nc, component u % nc; nc = 1: the points):
// out[i][j] = g_(ca, cb)[(off_rows[i] - off_cols[j]) mod n], row-major, the
// nc^2 kernels N = n^d entries apart.
__global__ void gather_block_kernel(const double2* __restrict__ g, int d, int n, int64_t N, int nc,
                                    const int* __restrict__ off, int row0, int nrows, int col0, int ncols,
                                    double2* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows * ncols) return;
  const int i = t / ncols, j = t - i * ncols;
  const int ur = row0 + i, uc = col0 + j;
  const int* a = off + (ur / nc) * d;
  const int* b = off + (uc / nc) * d;
  int64_t gi = 0;
  for (int x = 0; x < d; ++x) gi = gi * n + (((a[x] - b[x]) % n) + n) % n;
  out[t] = g[(int64_t)((ur % nc) * nc + uc % nc) * N + gi];
}

// C = beta C + alpha A B, all row-major, plain (setup-size) complex GEMM.
__global__ void small_gemm_kernel(int m, int nn, int k, double2 alpha, const double2* __restrict__ A, int lda,
                                  const double2* __restrict__ B, int ldb, double beta,
                                  double2* __restrict__ C, int ldc) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m * nn) return;
  const int i = t / nn, j = t - i * nn;
  double2 acc = cmake<double2>(0, 0);
  for (int l = 0; l < k; ++l) cfma(acc, A[i * lda + l], B[l * ldb + j]);
  double2 c = (beta == 0.0) ? cmake<double2>(0, 0) : cscale(C[i * ldc + j], beta);
  C[i * ldc + j] = cadd(c, cmul(alpha, acc));
}

// Solves X A = Bm for X (nS x nB) with A (nB x nB), both row-major, through
// the transposed system A^T X^T = Bm^T: Gaussian elimination with partial
// pivoting on the augmented [A^T | Bm^T] (nB x (nB + nS)), one workgroup.
struct SolveJob {
  int nB, nS;
  const double2* A;
  int lda;
  const double2* Bm;
  int ldb;
  double2* aug;
  double2* X;
  int ldx;
  int* info;
};
struct SolveJobs {
  SolveJob job[8];
};

// Register-resident elimination for small systems (nB <= 64, 1024 threads):
// wave w holds rows w, w + 16, ... and lane l columns l and l + 64 of the
// augmented [A^T | Bm^T(:, r0 : r0 + nR)] (1024 threads measured faster
// than 512 with twice the rows each); rows stay in place (the pivot order
// is recorded) and each step exchanges only the pivot row and the pivot
// column through LDS.  The right-hand sides go in chunks of at most 64, one
// workgroup each: every chunk repeats the same elimination of A^T (the same
// pivots, the same arithmetic), so the result does not depend on the split.
constexpr int kRsWaves = 16, kRsRows = 4, kRsCols = 2, kRsChunk = 64;   // nB <= 64, W <= 128

__device__ void right_solve_regs(const SolveJob& J, int r0, int nR) {
  const int nB = J.nB, W = nB + nR;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;   // ty < kRsWaves
  __shared__ double2 prow[kRsCols * 64];
  __shared__ double2 mcol[64];
  __shared__ unsigned long long keys[2];
  __shared__ int order[64], rstep[64];
  auto key_of = [](double v, int row) {
    return ((unsigned long long)__double_as_longlong(v) & ~0xFFFULL) | (unsigned long long)(4095 - row);
  };
  double2 v[kRsRows][kRsCols];
#pragma unroll
  for (int a = 0; a < kRsRows; ++a)
#pragma unroll
    for (int b = 0; b < kRsCols; ++b) {
      const int r = ty + kRsWaves * a, c = tx + 64 * b;
      double2 x = cmake<double2>(0, 0);
      if (r < nB && c < W) x = (c < nB) ? J.A[c * J.lda + r] : J.Bm[(r0 + c - nB) * J.ldb + r];
      v[a][b] = x;
    }
  if (threadIdx.x < 2) keys[threadIdx.x] = 0;
  __syncthreads();
  if (tx == 0)
#pragma unroll
    for (int a = 0; a < kRsRows; ++a)
      if (ty + kRsWaves * a < nB) atomicMax(&keys[0], key_of(cabs2(v[a][0]), ty + kRsWaves * a));
  __syncthreads();
  unsigned long long done = 0;
  for (int k = 0; k < nB; ++k) {
    const unsigned long long key = keys[k & 1];
    const int piv = 4095 - (int)(key & 0xFFF);
    if (threadIdx.x == 0) {
      if (!(__longlong_as_double((long long)(key & ~0xFFFULL)) > 0.0)) *J.info = 1;
      keys[(k + 1) & 1] = 0;
      order[k] = piv;
      rstep[piv] = k;
    }
    // Publish the pivot row and column k.
    if (ty == (piv % kRsWaves))
#pragma unroll
      for (int a = 0; a < kRsRows; ++a)
        if (a == (piv / kRsWaves))
#pragma unroll
          for (int b = 0; b < kRsCols; ++b) prow[tx + 64 * b] = v[a][b];
    if (tx == (k & 63))
#pragma unroll
      for (int b = 0; b < kRsCols; ++b)
        if (b == (k >> 6))
#pragma unroll
          for (int a = 0; a < kRsRows; ++a) mcol[ty + kRsWaves * a] = v[a][b];
    __syncthreads();
    done |= 1ULL << piv;
    const double2 pinv = crecip(prow[k]);
    // (the lane holding column k + 1 posts one key for its rows: the
    // largest, so 16 atomics a step rather than one per row)
    unsigned long long kmax = 0;
#pragma unroll
    for (int a = 0; a < kRsRows; ++a) {
      const int r = ty + kRsWaves * a;
      if (r >= nB || ((done >> r) & 1ULL)) continue;
      const double2 f = cmul(mcol[r], pinv);
#pragma unroll
      for (int b = 0; b < kRsCols; ++b) {
        const int c = tx + 64 * b;
        if (c > k && c < W) {
          cfms(v[a][b], f, prow[c]);
          if (c == k + 1) kmax = max(kmax, key_of(cabs2(v[a][b]), r));
        }
      }
    }
    if (kmax) atomicMax(&keys[(k + 1) & 1], kmax);
    __syncthreads();
  }
  // Back substitution on the right-hand-side columns, last pivot first:
  // x_k = rhs(order[k]) / U(k, k), then the rows of earlier pivots lose
  // U(m, k) x_k.
  for (int k = nB - 1; k >= 0; --k) {
    const int piv = order[k];
    if (tx == (k & 63))
#pragma unroll
      for (int b = 0; b < kRsCols; ++b)
        if (b == (k >> 6))
#pragma unroll
          for (int a = 0; a < kRsRows; ++a) mcol[ty + kRsWaves * a] = v[a][b];
    __syncthreads();
    const double2 uinv = crecip(mcol[piv]);
    if (ty == (piv % kRsWaves))
#pragma unroll
      for (int a = 0; a < kRsRows; ++a)
        if (a == (piv / kRsWaves))
#pragma unroll
          for (int b = 0; b < kRsCols; ++b) {
            const int c = tx + 64 * b;
            if (c >= nB && c < W) {
              v[a][b] = cmul(v[a][b], uinv);
              prow[c] = v[a][b];
            }
          }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < kRsRows; ++a) {
      const int r = ty + kRsWaves * a;
      if (r >= nB || rstep[r] >= k) continue;
      const double2 f = mcol[r];
#pragma unroll
      for (int b = 0; b < kRsCols; ++b) {
        const int c = tx + 64 * b;
        if (c >= nB && c < W) cfms(v[a][b], f, prow[c]);
      }
    }
    __syncthreads();
  }
  // X^T = the solved right-hand sides in pivot order: X[i][m] = x_m(nB + i).
#pragma unroll
  for (int a = 0; a < kRsRows; ++a) {
    const int r = ty + kRsWaves * a;
    if (r >= nB) continue;
    const int m = rstep[r];
#pragma unroll
    for (int b = 0; b < kRsCols; ++b) {
      const int c = tx + 64 * b;
      if (c >= nB && c < W) J.X[(r0 + c - nB) * J.ldx + m] = v[a][b];
    }
  }
}

// One workgroup per set type (blockIdx.x) and chunk of right-hand sides
// (blockIdx.y, register form only): the types' systems are independent.
__global__ void __launch_bounds__(64 * kRsWaves) right_solve_kernel(SolveJobs jobs) {
  const SolveJob& J = jobs.job[blockIdx.x];
  if (J.nS == 0) return;   // (a set type with no points)
  if (J.nB <= kRsWaves * kRsRows) {   // (launched with 64 kRsWaves threads)
    const int r0 = blockIdx.y * kRsChunk;
    if (r0 < J.nS) right_solve_regs(J, r0, min(kRsChunk, J.nS - r0));
    return;
  }
  if (blockIdx.y != 0) return;
  const int nB = J.nB, nS = J.nS, lda = J.lda, ldb = J.ldb, ldx = J.ldx;
  const double2* __restrict__ A = J.A;
  const double2* __restrict__ Bm = J.Bm;
  double2* aug = J.aug;
  double2* __restrict__ X = J.X;
  int* info = J.info;
  const int W = nB + nS;
  for (int t = threadIdx.x; t < nB * W; t += blockDim.x) {
    const int r = t / W, c = t - r * W;
    aug[t] = (c < nB) ? A[c * lda + r] : Bm[(c - nB) * ldb + r];
  }
  // Pivot keys: for v >= 0 the IEEE bits order like integers; the low 12
  // bits carry 4095 - row (largest modulus, ties to the lowest row; nB <=
  // 4096).  The search of column c + 1 is fused into the update of step c
  // (the lanes updating that column post their rows' keys), so a step needs
  // two barriers: after the row swap and after the update.  Two key slots
  // alternate between columns.
  __shared__ unsigned long long keys[2];
  auto key_of = [](double v, int row) {
    return ((unsigned long long)__double_as_longlong(v) & ~0xFFFULL) | (unsigned long long)(4095 - row);
  };
  if (threadIdx.x < 2) keys[threadIdx.x] = 0;
  __syncthreads();
  for (int r = threadIdx.x; r < nB; r += blockDim.x) atomicMax(&keys[0], key_of(cabs2(aug[r * W]), r));
  __syncthreads();
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6, ny = blockDim.x >> 6;
  for (int c = 0; c < nB; ++c) {
    const unsigned long long key = keys[c & 1];
    const int piv = 4095 - (int)(key & 0xFFF);
    if (threadIdx.x == 0) {
      if (!(__longlong_as_double((long long)(key & ~0xFFFULL)) > 0.0)) *info = 1;
      keys[(c + 1) & 1] = 0;   // (last read at step c - 1, before its barriers)
    }
    if (piv != c)
      for (int t = threadIdx.x; t < W - c; t += blockDim.x) {
        const double2 a = aug[c * W + c + t];
        aug[c * W + c + t] = aug[piv * W + c + t];
        aug[piv * W + c + t] = a;
      }
    __syncthreads();
    const double2 inv = crecip(aug[c * W + c]);
    // Rows over waves, columns over lanes (row-major: coalesced).
    for (int r = c + 1 + ty; r < nB; r += ny) {
      const double2 f = cmul(aug[r * W + c], inv);
      for (int cc = c + 1 + tx; cc < W; cc += 64) {
        double2& d = aug[r * W + cc];
        cfms(d, f, aug[c * W + cc]);
        if (cc == c + 1) atomicMax(&keys[(c + 1) & 1], key_of(cabs2(d), r));
      }
    }
    __syncthreads();
  }
  for (int c = nB - 1; c >= 0; --c) {
    const double2 inv = crecip(aug[c * W + c]);
    for (int t = threadIdx.x; t < nS; t += blockDim.x) aug[c * W + nB + t] = cmul(aug[c * W + nB + t], inv);
    __syncthreads();
    for (int t = threadIdx.x; t < c * nS; t += blockDim.x) {
      const int r = t / nS, cc = nB + t % nS;
      cfms(aug[r * W + cc], aug[r * W + c], aug[c * W + cc]);
    }
    __syncthreads();
  }
  // X^T = aug[:, nB:], so X[i][j] = aug[j][nB + i].
  for (int t = threadIdx.x; t < nS * nB; t += blockDim.x) {
    const int i = t / nB, j = t - i * nB;
    X[i * ldx + j] = aug[j * W + nB + i];
  }
}

__global__ void transpose_kernel(const double2* __restrict__ A, int rows, int cols, double2* __restrict__ At) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * cols) return;
  const int i = t / cols, j = t - i * cols;
  At[j * rows + i] = A[t];
}

}  // namespace

int coeff_reduce_blocks(int64_t N) {
  int64_t b = (N + kRedThreads * 8 - 1) / (kRedThreads * 8);
  return static_cast<int>(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

void coeff_reduce(hipStream_t st, int kind, const double* coeff, int64_t N, double omega, double ell,
                  double* partial, int nblocks, double* out) {
  coeff_partial_kernel<<<nblocks, kRedThreads, 0, st>>>(kind, coeff, N, omega, ell, partial);
  SPP_LAUNCH_CHECK();
  coeff_final_kernel<<<1, kRedThreads, 0, st>>>(partial, nblocks, out);
  SPP_LAUNCH_CHECK();
}

void coeff_finish(hipStream_t st, int kind, const double* coeff, int64_t N, int d, int n, double omega,
                  double ell, double energy, double s, double* q, double* sigma, double2* sig_c,
                  double2* sig2_c) {
  coeff_finish_kernel<<<ceil_div(N, 256), 256, 0, st>>>(kind, coeff, N, d, n, omega, ell, energy, s, q,
                                                        sigma, sig_c, sig2_c);
  SPP_LAUNCH_CHECK();
}

size_t stencil_work_elems(const StencilDev& S) {
  return (size_t)S.nG * S.nG + (size_t)S.nG * S.nB + (size_t)S.nB * (S.nB + S.nS);
}

void maxwell_symbols(hipStream_t st, int d, int n, double s, double2* sig, double2* sig2) {
  const int64_t N = (d == 2) ? (int64_t)n * n : (int64_t)n * n * n;
  maxwell_symbol_kernel<<<ceil_div(N, 256), 256, 0, st>>>(d, n, N, s, sig, sig2);
  SPP_LAUNCH_CHECK();
}

void stencil_build(hipStream_t st, int d, int n, const double2* g, const double2* g2, StencilDev* types, int ntypes,
                   double2* work, int* info, int nc) {
  const int64_t Npts = (d == 2) ? (int64_t)n * n : (int64_t)n * n * n;
  if (ntypes > 8) throw Error(-7, "at most 8 set types");
  for (int t = 0; t < ntypes; ++t)
    if (types[t].nB > 4096) throw Error(-7, "stencil boundary set larger than 4096 unknowns");
  const int T = 256;
  SolveJobs jobs{};
  std::vector<double2*> ggg(ntypes), mm(ntypes);
  double2* w = work;
  for (int t = 0; t < ntypes; ++t) {
    StencilDev& S = types[t];
    const int nS = S.nS, nB = S.nB, nG = S.nG;
    if (nS == 0) {   // a set type with no points: nothing to solve
      jobs.job[t] = SolveJob{0, 0, nullptr, 1, nullptr, 1, nullptr, S.T, 1, info + t};
      continue;
    }
    double2* Ggg = w;                          // nG x nG
    double2* M = Ggg + (size_t)nG * nG;        // nG x nB: (G G^H)(gamma, beta) - G(gamma,gamma) G(gamma,beta)
    double2* aug = M + (size_t)nG * nB;        // nB x (nB + nS)
    w += stencil_work_elems(S);
    ggg[t] = Ggg;
    mm[t] = M;
    gather_block_kernel<<<ceil_div((int64_t)nG * nG, T), T, 0, st>>>(g, d, n, Npts, nc, S.off, 0, nG, 0, nG, Ggg);
    SPP_LAUNCH_CHECK();
    gather_block_kernel<<<ceil_div((int64_t)nG * nB, T), T, 0, st>>>(g2, d, n, Npts, nc, S.off, 0, nG, nS, nB, M);
    SPP_LAUNCH_CHECK();
    small_gemm_kernel<<<ceil_div((int64_t)nG * nB, T), T, 0, st>>>(
        nG, nB, nG, cmake<double2>(-1.0, 0.0), Ggg, nG, Ggg + nS, nG, 1.0, M, nB);
    SPP_LAUNCH_CHECK();
    // T_S M(beta, :) = M(S, :)
    jobs.job[t] = SolveJob{nB, nS, M + (size_t)nS * nB, nB, M, nB, aug, S.T, nB, info + t};
  }
  int chunks = 1;
  for (int t = 0; t < ntypes; ++t)
    if (types[t].nB <= kRsWaves * kRsRows) chunks = std::max(chunks, (int)ceil_div(types[t].nS, kRsChunk));
  right_solve_kernel<<<dim3(ntypes, chunks), 64 * kRsWaves, 0, st>>>(jobs);
  SPP_LAUNCH_CHECK();
  for (int t = 0; t < ntypes; ++t) {
    StencilDev& S = types[t];
    const int nS = S.nS, nB = S.nB, nG = S.nG;
    if (nS == 0) continue;
    // C_S = G(S, gamma) - T_S G(beta, gamma)
    SPP_HIP(hipMemcpy2DAsync(S.C, sizeof(double2) * nG, ggg[t], sizeof(double2) * nG, sizeof(double2) * nG, nS,
                             hipMemcpyDeviceToDevice, st));
    small_gemm_kernel<<<ceil_div((int64_t)nS * nG, T), T, 0, st>>>(
        nS, nG, nB, cmake<double2>(-1.0, 0.0), S.T, nB, ggg[t] + (size_t)nS * nG, nG, 1.0, S.C, nG);
    SPP_LAUNCH_CHECK();
    transpose_kernel<<<ceil_div((int64_t)nS * nB, T), T, 0, st>>>(S.T, nS, nB, S.Tt);
    SPP_LAUNCH_CHECK();
    transpose_kernel<<<ceil_div((int64_t)nS * nG, T), T, 0, st>>>(S.C, nS, nG, S.Ct);
    SPP_LAUNCH_CHECK();
  }
}

}  // namespace spp
