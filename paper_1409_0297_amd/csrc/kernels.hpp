// Host-callable launchers of the HIP kernels, grouped by source file.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <initializer_list>
#include <string>

struct spp_cnn;

namespace spp {

// ------------------------------------------------------------- timing
// Optional per-kernel-class HIP event timing (enabled per factor by
// SPP_F_TIMING).  The launchers bracket the launches of each class with
// events on the launch stream and record the algorithmic bytes and flops of
// that launch; spp_kernel_timing() reads the totals back.
enum KernelClass {
  KC_FFT = 0, KC_GEMV = 1, KC_TRI = 2, KC_GEMM = 3, KC_PANEL = 4, KC_QAPPLY = 5, KC_INV = 6, KC_SOLVE_BLK = 7,
  KC_COUNT = 8
};
struct KernelTimer;
extern thread_local KernelTimer* g_timer;
void timer_begin(int cls, hipStream_t st);
void timer_end(int cls, hipStream_t st, double bytes, double flops);

// ------------------------------------------------------------- fft.hip
void fft_make_twiddles(double2* tw, int n, hipStream_t st);
bool fft_supported(int n);
// pre and mid are per-instance real arrays of N entries; batch entry b uses
// array b / per (per = right-hand sides per instance).
void fft_axis(hipStream_t st, const double2* in, double2* out, const double2* tw, int n,
              int64_t outer, int64_t inner, int64_t N, int batch, int dir,
              const double* pre, const double* mid, const double2* add, int per);
void fft_multi(hipStream_t st, const double2* in, double2* out, double2* tmp, const double2* tw,
               int d, int n, int batch, const double* pre, const double* sigma, const double2* add,
               int per);
void fft_inverse_all(hipStream_t st, const double2* in, double2* out, const double2* tw, int d, int n);
// Vector fields (Maxwell, d components, component-major [nrhs][d][n^d]):
// out = add + G (pre in), G = (curl curl - s)^{-1} applied per wave vector
// as its d x d symbol (see maxwell_symbol_kernel) between a forward and an
// inverse transform of the nrhs d grids; pre (real, n^d, shared by the
// components) and add are optional.  tmp: nrhs d n^d entries.
void fft_vector_green(hipStream_t st, const double2* in, double2* out, double2* tmp, const double2* tw, int d,
                      int n, int nrhs, double s, const double* pre, const double2* add);

// ------------------------------------------------------------- stencil.hip
// Sum of w_j = omega^2 / c_j^2 (Helmholtz, kind 0) or ell^2 V_j (kind 1) over
// the grid, and a flag for non-finite or non-positive input; result written to
// out[0] (sum) and out[1] (bad-entry count) in device memory.
void coeff_reduce(hipStream_t st, int kind, const double* coeff, int64_t N, double omega,
                  double ell, double* partial, int nblocks, double* out);
int coeff_reduce_blocks(int64_t N);
// q_j and sigma_k / N (FFT order), plus the complex arrays whose inverse
// transforms are the kernels of G and of G G^H.
void coeff_finish(hipStream_t st, int kind, const double* coeff, int64_t N, int d, int n,
                  double omega, double ell, double energy, double s, double* q, double* sigma,
                  double2* sig_c, double2* sig2_c);

struct StencilDev {
  int nS, nB, nG;      // unknowns (nc per point, point-major)
  const int* off;      // nG / nc points x d offsets (device)
  double2* T;          // nS x nB, row-major
  double2* C;          // nS x nG, row-major
  double2* Tt;         // nB x nS (T transposed), row-major
  double2* Ct;         // nG x nS (C transposed), row-major
};
// Builds T_S and C_S for every set type from the kernels g (of G) and g2 (of
// G G^H); the least-squares solves of all types run in one launch.  info[t]
// is set for a singular Gram matrix of type t.
// nc unknowns per point (vector fields): g and g2 hold nc^2 kernels (pair
// (a, b) at (a nc + b) n^d), the types' sizes count unknowns (point-major).
void stencil_build(hipStream_t st, int d, int n, const double2* g, const double2* g2,
                   StencilDev* types, int ntypes, double2* work, int* info, int nc = 1);
// Maxwell: the d^2 symbols of G = (curl curl - s)^{-1} and of G G^H, each / N
// (see maxwell_symbol_kernel), for fft_inverse_all per component pair.
void maxwell_symbols(hipStream_t st, int d, int n, double s, double2* sig, double2* sig2);
// Work entries one set type needs (stencil_build needs their sum over the types).
size_t stencil_work_elems(const StencilDev& S);

// ------------------------------------------------------------- mf.hip
struct FrontDev {
  int64_t off;         // F x F front (column-major) in the arena
  int64_t voff;        // solve vector slot (positions)
  int64_t foff;        // factor for the substitution: first p columns (ld F) ...
  int64_t uoff;        // ... and U12 (p x (F - p), ld ldu), in the factor base
  int ldu;             // (arena when resident, factor store when streamed)
  int64_t xoff;        // inverse work slot (2 p F: XL, XU, then Lt, Ut), relative to the level's work base
  int F, p;
  int idx;             // global indices of the F front points (pivots first)
  int map;             // F - p parent positions of the boundary points
  int perm;            // p ints: pivot row permutation
  int dblk;            // first diagonal-block slot (ceil(p / 32) slots of 2 x 32 x 32 entries)
  int inst;            // problem instance the front belongs to
  int parent;          // parent front (-1 at a root)
  int nchild;
  int child[8];
  int gptr;            // F + 1 offsets into MfDev::gsrc: the children's boundary
                       // rows that land on each position (in child order)
};

struct AsmBlockDev { int front, type, anchor, rowpos, colpos; };

struct TypeDev {       // per set type, for assembly / Q apply
  int nS, nB, nG;
  const int* off;
  const double2* T;
  const double2* C;
  const double2* Tt;
  const double2* Ct;
  const float2* Tt32;   // Tt rounded to complex64 (factors of complex64 fronts), else null
};

// One problem of a batch: its grid, potential and stencils.  Grid vectors of
// a batch are stored instance after instance, [nrhs][N] each, so instance i
// starts at Noff * nrhs.
struct InstDev {
  int d, n, b, m;
  int64_t N;           // unknowns per right-hand side (nc npts)
  int64_t Noff;        // sum of N over the earlier instances
  const double* q;     // per grid point
  TypeDev types[8];
  int nc;              // unknowns per point (Maxwell: d components, stored
                       // component-major: unknown (c, j) at c npts + j)
  int64_t npts;        // grid points n^d
};

struct MfDev {
  const FrontDev* fronts;
  const AsmBlockDev* blocks;
  const int* pos;
  const int* idx;
  const int* map;
  const int* gptr;     // per front, F + 1 offsets (see FrontDev::gptr)
  const int64_t* gsrc; // vector-arena position of each child boundary row
  int* perm;           // final row permutation of each front's pivot block
  int* ipiv;           // LAPACK-style interchange record written by the panel
  int* prow;           // block-local pivoting: row order of each 32-row block (front rows)
  int* info;           // [0] = breakdown front + 1 (0 if none); [1..8] stencil
                       // Gram breakdown per set type; [9] count of pivots below
                       // piv_warn; [10] = 1 if a pivot was below piv_tol
  unsigned* fnorm;     // per front: largest |entry| as assembled (float bits)
  unsigned* pstat;     // [0] pivot growth, [1] smallest |u_kk| / fnorm (float bits)
  float piv_tol;       // breakdown threshold on |u_kk| / fnorm (1e3 FP64 eps)
  float piv_warn;      // small-pivot threshold (1e3 eps of the front precision)
  const void* dkeep;   // 32 x 32 diagonal-block inverses kept for blocked levels
  const InstDev* inst; // device array, one entry per instance
  // Host-side summary (launch geometry).
  int ninst, d;
  int64_t anchors_max; // largest (n / b)^d over the instances
  int64_t Ntot;        // sum of N
  int nB_max[8];       // largest |beta| per set type
};

// Pivoting of a level's partial LUs:
//  kPivotBlockLocal: pivot within each 32-row diagonal block (default);
//  kPivotPartial:    over all remaining fully-summed rows, column by column
//                    (one-workgroup panel factorisation);
//  kPivotTournament: the 32 pivot rows of each block chosen over all
//                    remaining fully-summed rows by a tournament of LUs with
//                    partial pivoting over row chunks, then factored as a
//                    block (large fronts: many workgroups per front).
constexpr int kPivotBlockLocal = 0, kPivotPartial = 1, kPivotTournament = 2;
// Candidate-row buffer a tournament-pivoted level needs (ints).
inline int64_t mf_tournament_ints(int nfronts, int maxP) { return 2LL * nfronts * ((maxP + 255) / 256) * 32; }

// Step schedule of a block-locally pivoted level (bits of `variant`):
//  kVarPair:   two elimination steps per trailing update (the second block's
//              column and row take the first step's update on their own,
//              then one rank-64 product); without it, one step per trailing
//              update with the next diagonal block factored inside it;
//  kVarTile64: L21 / U12 of each step on 64 x 64 tiles (twice the workgroups,
//              shorter launches) instead of 128 x 32 / 32 x 128 tiles;
//  kVarFused:  (single steps) one launch per step: the trailing tiles form
//              their own L21 rows and U12 columns, the next diagonal block
//              is factored and the previous step's L21 / U12 written in the
//              same launch (gemm_fused_kernel).
// mf_default_variant is the untuned choice: pairs on levels of more than 64
// fronts (they fill the device, their trailing updates stream the fronts),
// single steps with 64 x 64 L21 / U12 tiles on the others.
constexpr int kVarPair = 1, kVarTile64 = 2, kVarFused = 4, kVarAll = 7;
inline int mf_default_variant(int nfronts) { return nfronts > 64 ? kVarPair : kVarTile64; }

// inv_st / lu_done (optional): the explicit inverses of an Inverse or Side
// level go to stream inv_st after the level's LU (lu_done recorded on st,
// waited for on inv_st), so that they run beside the next level's
// factorisation: they read and write only this level's pivot rows and
// columns, L21 and U12 (the next level reads its children's Schur
// complements), and xwork / tbuf, which no LU step of a block-locally
// pivoted level uses.  The caller joins inv_st before the factor is used.
template <typename R>
void mf_factor_level(hipStream_t st, const MfDev& mf, void* arena, void* xwork, void* tbuf, void* dinv, int* tpbuf,
                     int f0, int f1, int maxF, int maxP, int blk0, int blk1,
                     int max_children, int form, int pivoting, int variant,
                     const int* hF, const int* hP,   // host: F and p of the level's fronts
                     hipStream_t inv_st = nullptr, hipEvent_t lu_done = nullptr);
// How a level's fronts are kept for the substitution:
//  kFormLU:      LU in place, one workgroup per front solves;
//  kFormInverse: L11^{-1}, U11^{-1} over the pivot block, L21 and U12 kept:
//                four matrix-vector products per level and solve;
//  kFormSide:    as kFormInverse with L21 L11^{-1} and U11^{-1} U12 over the
//                side blocks: one product per level and direction.
//  kFormBlocked: LU in place, 32-row block steps over all fronts of the level
//                with the diagonal-block inverses kept from the factorisation
//                (few large fronts, whose explicit inverses would be too big).
constexpr int kFormLU = 0, kFormInverse = 1, kFormSide = 2, kFormBlocked = 3;
int mf_level_solve_form(int nfronts, int maxF, int maxP, bool c64, bool streamed);

// Streamed storage: copies each front's factor part of a level from its
// working front in the arena to the factor store (see layout_plan).
template <typename R>
void mf_store_factors(hipStream_t st, const MfDev& mf, const void* arena, void* store, int f0, int nf, int maxF);

// y = Q r for every instance of the batch (vectors in the batch layout);
// y is complex64 (float2) with to_float, else complex128.
void q_apply(hipStream_t st, const MfDev& mf, const double2* r, void* y, int nrhs, bool to_float = false);

template <typename R>
void mf_solve(hipStream_t st, const MfDev& mf, const void* arena, void* w, void* z,
              const void* x_in, void* x_out, int nrhs,
              const int* level_begin, const int* level_maxF, const int* level_maxK,
              const int* level_maxP, const double* level_ent, const int* level_form, int nlevels,
              void* partial, int64_t partial_cap, bool persistent,
              hipEvent_t* level_events = nullptr,   // optional: 4 per level, see mf_solve
              hipEvent_t inv_early = nullptr, hipEvent_t inv_last = nullptr);
// (inv_early / inv_last, optional: the stream waits for inv_early before the
// first level solved by products except the last one, and for inv_last
// before the last level if that one is solved by products; the explicit
// inverses of those levels may still be in the making on another stream.)

template <typename R>
void cast_vectors(hipStream_t st, const void* in, void* out, int64_t count, int to_double);

// ------------------------------------------------------------- krylov.hip
// h_out[i] (+)= V_i^H w per right-hand side; if h_acc, also h_acc[i] += V_i^H w.
// dj (optional, for graph replays): the iteration index j in device memory;
// then nvec = j + 1 and h_out / h_acc / v / h_sub are offset by j * jstride.
// Partial-sum slots per vector and right-hand side that kr_dots needs.
int64_t kr_dot_slots(int64_t N);
void kr_dots(hipStream_t st, const double2* V, int64_t vstride, int nvec, const double2* w,
             int nrhs, int64_t N, double2* partial, double2* h_out, int hstride, int accumulate,
             double2* h_acc, int acc_stride, const int* dj = nullptr, int64_t h_jstride = 0,
             int64_t acc_jstride = 0);
void kr_update(hipStream_t st, const double2* V, int64_t vstride, int nvec, double2* w,
               int nrhs, int64_t N, const double2* h, int hstride, const int* dj = nullptr,
               int64_t h_jstride = 0);
// Givens step fused into kr_norm_scale (H null: none): for right-hand side r
// of the launch, column c0 + r of H / cs / sn / g at iteration j (or *dj).
struct KrGivens {
  double2* H = nullptr;
  int hcol = 0, hrhs = 0;
  double* cs = nullptr;
  double2* sn = nullptr;
  double2* g = nullptr;
  int j = 0, ldg = 0;
  double* resid = nullptr;
  double* resid_host = nullptr;   // optional: device alias of pinned host memory
  int c0 = 0;
};
void kr_norm_scale(hipStream_t st, const double2* w, double2* v, int nrhs, int64_t N,
                   double* partial, double2* h_sub, int hstride, const int* dj = nullptr,
                   int64_t v_jstride = 0, int64_t h_jstride = 0, const KrGivens& gv = KrGivens());
// The rest of a CGS2 step after its first projection h1 (eager form):
// w -= V h1 with the second projection's partial dots in the same pass,
// h2 = V^H w (h_acc += h2), then w -= V h2 with the partial sums of |w|^2
// (npart, as kr_norm_scale leaves them); kr_normalize then finishes
// v = w / ||w||, the subdiagonal entry and the Givens step.
void kr_cgs2_second(hipStream_t st, const double2* V, int64_t vstride, int nvec, double2* w, int nrhs, int64_t N,
                    const double2* h1, int h1stride, double2* dpart, double2* h2, int h2stride, double2* h_acc,
                    int acc_stride, double* npart);
void kr_normalize(hipStream_t st, const double2* w, double2* v, int nrhs, int64_t N, double* partial,
                  double2* h_sub, int hstride, const KrGivens& gv = KrGivens());
void kr_givens(hipStream_t st, double2* H, int hcol_stride, int hrhs_stride, double* cs, double2* sn,
               double2* g, int j, int nrhs, int ldg, double* resid, const int* active,
               const int* dj = nullptr);
void kr_backsolve(hipStream_t st, const double2* H, int hcol_stride, int hrhs_stride, const double2* g,
                  int ldg, double2* y, int k, int nrhs, const int* kvec);
// u = Z y (accumulate: u += Z y) per right-hand side with kvec[rhs] vectors.
void kr_combine(hipStream_t st, const double2* Z, int64_t zstride, int nvec, const double2* y,
                int ldy, double2* u, int nrhs, int64_t N, const int* kvec, bool accumulate = false);
void kr_norms(hipStream_t st, const double2* v, int nrhs, int64_t N, double* partial, double* out);
void kr_sub(hipStream_t st, const double2* a, const double2* b, double2* out, int64_t count);
void kr_scale_init(hipStream_t st, const double2* g, double2* v0, const double* norms, int nrhs,
                   int64_t N, double2* gvec, int ldg);
// dst + j dst_jstride <- src + j src_jstride (count values), j = *dj.
void kr_copy_j(hipStream_t st, const double2* src, int64_t src_jstride, double2* dst,
               int64_t dst_jstride, int64_t count, const int* dj);
// *c = value, or *c += value (a kernel, so that it can sit in a captured graph).
void kr_set_counter(hipStream_t st, int* c, int value, bool add);

// ------------------------------------------------------------- tune.cpp
// Tuned launch parameters (see tune.cpp): tune_get returns the tuned value of
// a shape key, or fallback.
std::string tune_key(const char* kind, std::initializer_list<int64_t> sizes);
int tune_get(const std::string& key, int fallback);
void tune_force(const std::string& key, int value);   // value < 0 clears
void tune_set(const std::string& key, int value);
bool tune_has(const std::string& key);
void tune_save();
float tune_time(hipStream_t st, int reps, const std::function<void()>& fn, void* flush = nullptr,
                size_t flush_bytes = 0);

// FFT lines per workgroup: heuristic, valid candidates, key (fft.hip).
int fft_lines_default(int n, int64_t outer, int64_t inner);
bool fft_lines_valid(int n, int64_t outer, int64_t inner, int L);
std::string fft_tune_key(int n, int64_t outer, int64_t inner, int batch);

// Clears the status words of a factorisation pass: info[0] (breakdown
// front), info[9] and info[10] (small pivots, fatal flag), the pivot
// statistics (largest growth 0, smallest pivot ratio FLT_MAX) and the
// largest entry of each of the nfronts fronts; one launch (mf.hip).
void mf_reset_status(hipStream_t st, const MfDev& mf, int nfronts);

// One substitution product (gemv_kernel mode) of a level of fronts with a
// given split-K chunk count over 64-row tiles (1 .. kGemvNarrowSplit - 1),
// or 16-row tiles with the columns not split (0) or split c ways
// (kGemvNarrowSplit + c), or the tuned or heuristic choice (< 0); mf.hip.
// xin: the forward input (read by mode 4, which gathers its own vector).
constexpr int kGemvNarrowSplit = 1024;
template <typename R>
void mf_gemv(hipStream_t st, const MfDev& mf, const void* arena, void* W, void* Z, void* xout, const void* xin, int nrhs,
             int f0, int nf, int rows, int cols, int mode, double ent, void* partial, int64_t partial_cap, int nchunks);
int gemv_chunks_default(int rows, int cols, int nf, int nrhs, int64_t partial_cap);
std::string gemv_tune_key(int rows, int cols, int nf, int mode, int nrhs, int csize);

// ------------------------------------------------------------- scratch.hip
// Device scratch of the no-allocation entry points: kNoAllocScratchBytes per
// GPU in a file-scope device array; noalloc_scratch() returns its device
// address on the current device (looked up once per device).
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
void* noalloc_scratch();

// ------------------------------------------------------------- cnn.hip
// Learned preconditioner stage: y = out_scale * net(in_scale * x) per sample,
// x, y complex128 [batch][n^2].
void cnn_apply(struct ::spp_cnn* net, const double2* x, double2* y, int batch, double in_scale, double out_scale,
               hipStream_t st);
int cnn_grid(const struct ::spp_cnn* net);

}  // namespace spp
