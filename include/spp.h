/*
 * spp.h -- C ABI of the MI355X sparsifying-preconditioner library.
 *
 * The library solves the periodic pseudospectral systems of
 *   L. Ying, "Sparsifying preconditioner for pseudospectral approximations of
 *   indefinite systems on periodic structures" (arXiv:1409.0297):
 * the Helmholtz equation (-Delta - omega^2 / c(x)^2) u = f on [0,1)^d (eq. helm)
 * and the rescaled Schroedinger equation (-Delta + ell^2 V(ell y) - ell^2 E) u = f
 * (eq. schr), both written as (-Delta - s + q) u = f (eq. Dsq) and discretised
 * on an n^d grid as (L - s + q) u = f (eq. Lsq).  It solves the equivalent
 * integral form (I + G q) u = G f with G = (L - s)^{-1} (eq. G, Section 2.2)
 * by flexible GMRES in FP64, right-preconditioned with M = P^{-1} Q, where Q
 * is the sparsifying stencil operator and P = Q + C q its sparse truncation
 * (Sections 2.2-2.3), factorised by nested-dissection multifrontal LU.
 *
 * Section 4 names the Maxwell equation for the electric field,
 *   (curl curl - omega^2 eps(x)) E = f  (units with c = 1),
 * as the method's next case without giving an algorithm; kind SPP_MAXWELL
 * is this library's reading of it.  E and f have d components (2D: the
 * in-plane field E_0, E_1 of a field independent of the third coordinate;
 * 3D: all three; component a points along grid axis a).  curl is built from
 * spectral first derivatives whose Nyquist wave number is dropped, so curl
 * curl has the d x d symbol 4 pi^2 (|kt|^2 I - kt kt^T) per wave vector
 * (kt_a = k_a, 0 at the index n/2).  With w = omega^2 eps the split of eq.
 * (Dsq) gives s = mean(w), q = s - w, G = (curl curl - s)^{-1} with symbol
 * (I - kt kt^T / |kt|^2) / (4 pi^2 |kt|^2 - s) - kt kt^T / (|kt|^2 s), and
 * the same integral form (I + G q) E = G f.  The sets of Section 2.3 and the
 * nested-dissection boxes are unchanged; a set's unknowns are all components
 * of its points, T_S is the same least-squares fit over them, and a box
 * eliminates its points with all their components.
 *
 * Conventions for every entry point
 *  - Grid functions are C-order arrays over j in [0,n)^d (last axis fastest).
 *    Complex data is interleaved (re, im) double, i.e. C99 double complex.
 *    A batch of nrhs grid functions is stored [nrhs][n^d]; a Maxwell field
 *    is d grid functions, component-major, so nrhs fields are stored
 *    [nrhs][d][n^d] and every vector argument below holds d n^d entries per
 *    right-hand side.
 *  - Pointers documented as DEVICE point to GPU memory owned by the caller
 *    (typically allocated by PyTorch); HOST pointers to CPU memory.  The
 *    library never frees caller memory.  It owns only what a spp_factor
 *    holds (factors, stencils, work space), released by spp_destroy.
 *  - All GPU work is ordered on the hipStream_t passed in (0 = the null
 *    stream).  Calls returning host outputs synchronise that stream.  One
 *    exception: during spp_setup of resident fronts, the zeroing of the front
 *    arena and the explicit inverses of the levels solved by products run on
 *    a second stream the library owns (one per device, default priority),
 *    beside the stencils and the next level's LU.  spp_setup returns once
 *    the LU is complete; the last inverses may still run.  Every later call
 *    that reads the factor, on any stream, waits for them on that stream
 *    before its first read of them, so the caller needs no synchronisation
 *    of its own.
 *  - Every function returns SPP_OK (0) or a negative error code; no C++
 *    exception crosses this boundary.  spp_last_error() gives a message for
 *    the most recent failure on the calling thread.
 *  - A spp_factor is not thread-safe; distinct handles are independent.
 */
#ifndef SPP_H_
#define SPP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* spp_stream_t; /* same type as hipStream_t */

enum {
  SPP_OK = 0,
  SPP_EINVAL = -1,           /* bad dim/n/b, null pointer, non-finite input   */
  SPP_ESINGULAR_SHIFT = -2,  /* L - s could not be moved off singularity      */
  SPP_EBREAKDOWN = -3,       /* zero, non-finite or tiny pivot in a front     */
  SPP_NOT_CONVERGED = -4,    /* max_iter reached; u, iters, relres still valid */
  SPP_ENOMEM = -5,           /* device allocation failed                       */
  SPP_EHIP = -6,             /* a HIP runtime call failed                      */
  SPP_ENOTIMPL = -7          /* combination of options not implemented         */
};

typedef enum { SPP_HELMHOLTZ = 0, SPP_SCHRODINGER = 1, SPP_MAXWELL = 2 } spp_kind;

/* Arithmetic of the frontal matrices and the triangular solves. */
typedef enum {
  SPP_C128 = 0,        /* complex128 fronts, FP64 MFMA                         */
  SPP_C64_FRONTS = 1   /* complex64 fronts and substitution, FP32 MFMA; the
                          operator apply, residuals and GMRES stay FP64        */
} spp_prec;

/* Order in which nested-dissection boxes merge above the leaves (Section 2.3,
   Figure 1): all 2^d children at once, or two at a time along the axes in
   turn.  Both give the same P^{-1}; they differ in front sizes. */
typedef enum { SPP_ORDER_OCTREE = 0, SPP_ORDER_BISECT = 1 } spp_order;

typedef struct {
  int32_t dim;          /* d in {2, 3}                                          */
  int32_t n;            /* grid points per axis; even                            */
  int32_t b;            /* leaf box width in grid steps; b | n, n/b = 2^L >= 2   */
  int32_t kind;         /* spp_kind                                              */
  double omega;         /* Helmholtz / Maxwell frequency omega (eq. helm)        */
  double ell, energy;   /* Schroedinger size ell and energy E (eq. schr)         */
  const double* coeff;  /* DEVICE, n^d reals: c(x_j) for Helmholtz,
                           V(ell x_j) for Schroedinger, eps(x_j) > 0 for
                           Maxwell; read during setup only.  Maxwell leaf
                           boxes: d (b + 1)^d <= 1024 (2D b <= 21, 3D b <= 5),
                           else SPP_ENOTIMPL                                    */
} spp_problem;

#define SPP_F_UNPRECONDITIONED 1  /* GMRES with M = I (for comparisons)        */
#define SPP_F_TIMING 2            /* bracket the launches of each kernel class
                                     with HIP events (see spp_kernel_timing)   */
#define SPP_F_PARTIAL_PIVOTING 4  /* pivot over all remaining fully-summed rows
                                     of a front; default: pivot within each
                                     32-row diagonal block of the front        */
#define SPP_F_PERSISTENT 16       /* substitution of runs of consecutive
                                     small-front levels as one cooperative
                                     launch with grid barriers between levels
                                     (not inside graph replays)               */
#define SPP_F_AUTOTUNE 32         /* run spp_autotune before the first solve of
                                     each right-hand-side count               */
#define SPP_F_NO_SIDE 64          /* levels of few fronts keep L21 and U12 (four
                                     substitution products per level and solve)
                                     instead of L21 L11^-1 and U11^-1 U12 (one
                                     product per level and direction): less
                                     setup work, more launches per solve      */
#define SPP_F_STREAMED 128        /* streamed front storage even where every
                                     front would fit: the arena holds the
                                     fronts of two adjacent levels, factors
                                     go to a compact store (p^2 + 2 p (F - p)
                                     entries per front).  Chosen by itself
                                     when the sum of F^2 over all fronts
                                     would exceed 85% of free device memory
                                     (3D grids such as 128^3)                  */
#define SPP_F_GRAPHS 8            /* capture one FGMRES iteration in a HIP graph
                                     (once per factor and nrhs) and replay it
                                     with the step index in device memory;
                                     ignored with SPP_F_TIMING or a learned
                                     stage attached                            */

/* Device memory for a factor's large blocks (the front arena, or in the
   streamed storage mode the factor store and the working-front arena):
   alloc(bytes, ctx) returns `bytes` of device memory on the current device
   (aligned to 256 bytes) or NULL, which setup reports as SPP_ENOMEM;
   free(ptr, ctx) releases a block alloc returned.  The factor calls free on
   its blocks in spp_destroy, after synchronising.  A caching framework
   allocator (PyTorch's) can be passed here.  Both NULL: the library's own
   hipMalloc-backed cache. */
typedef void* (*spp_alloc_fn)(size_t bytes, void* ctx);
typedef void (*spp_free_fn)(void* ptr, void* ctx);

typedef struct {
  int32_t prec;         /* spp_prec                                              */
  int32_t order;        /* spp_order                                             */
  double tol;           /* stop when the true residual of (I + G q) u = G f is
                           <= tol * ||G f|| (Section 3: GMRES to a relative
                           tolerance)                                            */
  int32_t max_iter;     /* total FGMRES iterations over all cycles, <= 500      */
  int32_t flags;        /* SPP_F_* bits                                          */
  int32_t restart;      /* Krylov vectors per cycle (FGMRES(restart)); 0 = no
                           restart (one cycle of up to max_iter).  A cycle also
                           ends, and another starts from the true residual,
                           when the Givens estimate met tol but the true
                           residual did not                                     */
  int32_t pattern;      /* stencil sets of Q (Section 2.3): 0 = the cells,
                           faces, edges and vertices of the leaf boxes (the
                           paper's choice); 1 = every point its own set with
                           the neighbourhood mu(j) = gamma({j}) (the pattern
                           Section 2.3 sets aside; for comparisons)            */
  spp_alloc_fn alloc;   /* optional allocator hook (both or neither)             */
  spp_free_fn free;
  void* alloc_ctx;      /* passed to alloc / free                                */
} spp_options;

typedef struct {
  double s;             /* shift actually used (after any perturbation)         */
  int32_t shift_moves;  /* how many times s was perturbed (Section 2.2)          */
  int32_t n_fronts, n_levels, max_front;
  int64_t factor_entries;   /* sum over fronts of p^2 + 2 p (F - p)              */
  int64_t factor_bytes;     /* bytes the substitution reads per application      */
  double factor_flops;      /* real flops of the partial factorisations          */
  double t_setup_ms;        /* wall time of the last spp_setup                   */
  double t_factor_ms;       /* of which the multifrontal factorisation: GPU time
                               to its last LU step (the explicit inverses of the
                               levels solved by products run beside it on a
                               second stream and may end during the first
                               solve, which waits for them)                    */
  double t_solve_ms;        /* wall time of the last spp_solve                   */
  int32_t last_iters;       /* GMRES iterations of the last solve (max over RHS) */
  int32_t breakdown_front;  /* front index of a pivot breakdown, else -1         */
  int32_t last_cycles;      /* FGMRES cycles of the last solve (1 = no restart)  */
  int32_t storage;          /* 0: every front resident in one arena; 1: streamed
                               (factors kept compact, fronts of two adjacent
                               levels resident at a time)                       */
  double pivot_growth;      /* max over fronts of the largest entry of the
                               updated 32 x 32 diagonal blocks (before and after
                               their LU) over the largest entry of the front as
                               assembled: the growth of the Schur updates        */
  double min_pivot;         /* min over fronts of |u_kk| / max |front entry|;
                               below 1e3 FP64 eps (a pivot lost in the rounding
                               of the assembled entries) the setup reports
                               SPP_EBREAKDOWN with breakdown_front set          */
  int64_t device_bytes;     /* device memory the memory plan asked for at setup
                               (factor storage and work space)                  */
  int32_t small_pivots;     /* pivots with |u_kk| / max |front entry| below 1e3
                               eps of the front precision: not a breakdown (the
                               FP64 FGMRES corrects the factor), but a sign of
                               an ill-conditioned front                         */
  int32_t reserved_stats;
} spp_stats_t;

typedef struct spp_factor spp_factor;

/* ---- setup: a1-a6 ----------------------------------------------------------
 * Computes s and q (eq. Dsq, with s the grid mean and the perturbation rule of
 * Section 2.2), the Green kernel (eq. G), the stencils T_S and C_S of every
 * set type (eq. Qc and Section 2.3), assembles P = Q + C q directly into the
 * nested-dissection fronts and factorises them.  On success *out owns all
 * device memory of the factor.  Errors: SPP_EINVAL (bad sizes, null pointers,
 * non-finite coeff), SPP_ESINGULAR_SHIFT, SPP_EBREAKDOWN, SPP_ENOMEM, SPP_EHIP. */
int spp_setup(const spp_problem* problem, const spp_options* options,
              spp_stream_t stream, spp_factor** out);

/* ---- batched setup ---------------------------------------------------------
 * Sets up `count` independent problems (1 <= count <= 4096) in one factor,
 * e.g. several media, frequencies or grid sizes (Sections 3.1-3.2 solve one
 * such family at a time).  All problems must have the same dim; n, b, kind,
 * omega, ell, energy and coeff may differ.  Maxwell problems are set up one
 * per factor (SPP_ENOTIMPL in a batch of more than one).  Their nested-dissection fronts
 * are factorised level by level in shared launches, and spp_solve then runs
 * one FGMRES per (problem, right-hand side) pair in lock step, each with its
 * own stopping test.  Batch vectors are the problems' vectors one after the
 * other: problem i occupies [nrhs][n_i^d] starting at nrhs * sum_{j<i} n_j^d
 * complex entries; iters / relres are indexed problem * nrhs + rhs.  The
 * component calls below apply to the whole batch in the same layout.
 * Errors as for spp_setup; on error no factor is returned (*out = NULL),
 * except SPP_EBREAKDOWN as for spp_setup.  spp_setup(p, o, s, out) is
 * spp_setup_batch(p, 1, o, s, out). */
int spp_setup_batch(const spp_problem* problems, int32_t count, const spp_options* options,
                    spp_stream_t stream, spp_factor** out);

/* ---- solve: a7-a11 ---------------------------------------------------------
 * f: DEVICE complex128 [nrhs][n^d]; u: DEVICE complex128 [nrhs][n^d], written.
 * iters: HOST int32[nrhs], FGMRES iterations summed over cycles; relres:
 * HOST double[nrhs], the true relative residual ||G f - (I + G q) u|| / ||G f||
 * of each returned u (Section 2.2: the integral form; Section 3: GMRES to a
 * relative tolerance).  Returns SPP_NOT_CONVERGED (u, iters and relres still
 * written) if any right-hand side's true residual is above tol once max_iter
 * iterations are spent.  A zero right-hand side gives u = 0, 0 iterations. */
int spp_solve(spp_factor* factor, const void* f, int32_t nrhs, void* u,
              int32_t* iters, double* relres, spp_stream_t stream);

/* ---- batched solve with per-problem right-hand sides -------------------------
 * For a factor of `count` problems (spp_setup_batch): f[i] and u[i] are
 * DEVICE complex128 [nrhs[i]][n_i^d] arrays of problem i (f[i] may be NULL
 * only if nrhs[i] == 0; u[i] is written); nrhs: HOST int32[count], each in
 * [0, 64].  iters / relres: HOST arrays of sum_i nrhs[i] entries, problem by
 * problem.  All problems iterate in lock step, as in spp_solve with
 * max_i nrhs[i] columns each (problems with fewer right-hand sides carry zero
 * columns, which converge at once).  Returns as spp_solve; SPP_EINVAL for a
 * count mismatch or bad pointers. */
int spp_solve_batch(spp_factor* factor, const void* const* f, const int32_t* nrhs,
                    void* const* u, int32_t* iters, double* relres, spp_stream_t stream);

/* Times candidate launch parameters on this factor's shapes (lines per
   workgroup of each FFT pass, column chunks of each substitution product with
   explicit inverses) for nrhs right-hand sides and keeps the fastest in a
   process-wide table keyed by kernel, architecture and shape; later factors
   with the same shapes use it.  If the environment variable SPP_TUNE_CACHE
   names a file, the table is read from it at first use and rewritten here. */
int spp_autotune(spp_factor* factor, int32_t nrhs, spp_stream_t stream);

/* The process-wide tuning table, entry by entry.  key: NUL-terminated text
   "<kind>@<arch>:<size>:<size>...", as the table file holds it.  Kinds:
     fft_lines    lines per workgroup of an FFT pass;
     gemv_chunks  column chunks of a substitution product over 64-row tiles
                  (1 .. 1023), or 0: 16-row tiles, columns not split, or
                  1024 + c: 16-row tiles, columns split c ways;
     mf_form      solve form of a level, keyed by front bytes (8 complex64,
                  16 complex128), fronts, largest F, largest p:
                  0 LU in place, 1 inverses of L11 / U11, 2 side products;
     mf_steps     step schedule of that level: bit 0 paired steps (one
                  rank-64 update per two 32-column steps), bit 1 L21 / U12 on
                  64 x 64 tiles (else 128 x 32 / 32 x 128), bit 2 (single
                  steps) one launch per step, the trailing tiles forming their
                  own L21 / U12 pieces.
   Setups (with SPP_F_AUTOTUNE and resident storage) fill the mf_ entries by
   timing every candidate on the factorisation itself; a level's solve form
   counts its substitution as 20 preconditioner applies per factorisation.
   Factors set up later use the table whether or not they tune; an entry that
   does not apply to a level (LU in place on fronts whose vectors exceed the
   solve kernels' LDS) is ignored there.
   spp_tune_set: value >= 0 sets the entry, value < 0 removes it; not written
   to the SPP_TUNE_CACHE file until the next tuning run saves the table.
   spp_tune_get: *value = the entry, SPP_EINVAL if absent (or key null). */
int spp_tune_set(const char* key, int32_t value);
int spp_tune_get(const char* key, int32_t* value);

/* ---- components of the hot path, exposed for testing and benchmarking ----- */

/* w = (I + G q) z (Section 2.2); z, w DEVICE complex128 [nrhs][n^d]; may alias. */
int spp_apply_operator(spp_factor* factor, const void* z, void* w, int32_t nrhs,
                       spp_stream_t stream);

/* w = (I + G q) z exactly as spp_apply_operator computes it (same kernels),
   for callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the FFT
   intermediate lives in a library-owned static device scratch of 64 MiB per
   GPU instead of the factor's grown work buffers, and the call makes no
   allocation.  z, w DEVICE complex128 [nrhs][n^d] in the batch layout; may
   alias.  Requires nrhs * (sum of n_i^d) * 16 bytes <= 64 MiB, else
   SPP_EINVAL.  Every call on a GPU shares that GPU's scratch, so calls that
   overlap on one GPU (different streams or threads) race; calls ordered on
   one stream do not.  No kernel timing is recorded. */
int spp_apply_operator_noalloc(spp_factor* factor, const void* z, void* w, int32_t nrhs,
                               spp_stream_t stream);

/* g = G f (eq. G); DEVICE complex128 [nrhs][n^d]; may alias. */
int spp_apply_green(spp_factor* factor, const void* f, void* g, int32_t nrhs,
                    spp_stream_t stream);

/* y = Q r, (Q r)_S = r_S - T_S r_beta(S) (Section 2.3); DEVICE; must not alias. */
int spp_apply_q(spp_factor* factor, const void* r, void* y, int32_t nrhs,
                spp_stream_t stream);

/* z = P^{-1} Q r, the preconditioner (Section 2.2); DEVICE; may alias. */
int spp_apply_precond(spp_factor* factor, const void* r, void* z, int32_t nrhs,
                      spp_stream_t stream);

/* Shift s of the first problem (HOST double) and potential q of every problem
   (DEVICE double[sum n_i^d] in the batch layout with nrhs = 1; may be NULL).
   q is per grid point for Maxwell too (every component shares it). */
int spp_get_coefficients(const spp_factor* factor, double* s, double* q);

/* Shift s used by problem `problem` of a batch and how many times the rule of
   Section 2.2 perturbed it (HOST outputs, each may be NULL). */
int spp_get_shift(const spp_factor* factor, int32_t problem, double* s, int32_t* moves);

/* Stencil of set type `type` of the first problem (bit i set = axis i pinned to a leaf box face,
   so 0 is the cell and 2^d - 1 the vertex; Section 2.3).  All HOST outputs,
   each may be NULL: nS = |S|, nB = |beta(S)|; offsets: int32[(nS+nB)*dim],
   the grid offsets of S then beta(S) from the set's leaf box corner (the
   column order of Q(S, gamma(S)) = [I  -T_S]); T: complex128 [nS][nB];
   C: complex128 [nS][nS+nB] = [I  -T_S] G(gamma(S), gamma(S)).  Maxwell:
   nS and nB count unknowns (d per point, point-major: point i, component a
   at i d + a), T and C are over those unknowns, offsets still list the
   (nS + nB) / d points. */
int spp_get_stencil(const spp_factor* factor, int32_t type, int32_t* nS, int32_t* nB,
                    int32_t* offsets, void* T, void* C);

int spp_stats(const spp_factor* factor, spp_stats_t* out);

/* Kernel classes timed under SPP_F_TIMING. */
enum {
  SPP_K_FFT = 0,     /* FFT passes of the operator / Green apply (a2, a7, a8)        */
  SPP_K_GEMV = 1,    /* substitution products with the inverted pivot blocks (a9)     */
  SPP_K_TRI = 2,     /* in-workgroup triangular solves of small fronts (a9)           */
  SPP_K_GEMM = 3,    /* MFMA trailing updates / Schur complements of the fronts (a6)  */
  SPP_K_PANEL = 4,   /* pivoted panel factorisation (a6)                              */
  SPP_K_QAPPLY = 5,  /* sparsifying stencil apply Q r (a9)                            */
  SPP_K_INV = 6,     /* products that prepare the substitution, not part of the LU:
                        triangular inverses of the pivot blocks and the side
                        products L21 L11^-1, U11^-1 U12 (a6, few-front levels)      */
  SPP_K_SOLVE_BLK = 7 /* blocked triangular solves of streamed top fronts (a9)     */
};
/* Totals since setup (or the last reset) for one kernel class, all HOST
   outputs, each may be NULL: summed event time of its launches (ms, measured
   on the launch stream), number of launches, and the algorithmic bytes and
   real flops those launches had to move / perform.  Synchronises on the
   recorded events.  Zeros if the factor was set up without SPP_F_TIMING. */
int spp_kernel_timing(const spp_factor* factor, int32_t kclass, double* total_ms,
                      int64_t* launches, double* bytes, double* flops);
int spp_kernel_timing_reset(spp_factor* factor);

/* ---- learned flexible-GMRES stage (a small CNN) ------------------------------
 * A 3 x 3 circular convolutional network, bias-free, ReLU after every layer
 * but the last, mapping a complex grid function (real and imaginary parts as
 * two channels) on an n x n grid to another.  It is trained on pairs
 * (v, M v) of Krylov vectors and sparsifying-preconditioner outputs, and used
 * as a cheap preconditioner stage inside FGMRES (Section 2.2 uses M = P^{-1} Q
 * for every iteration; flexible GMRES allows M to change per iteration).
 * Activations and MFMA inputs are bf16 (SPP_CNN_BF16) or fp32 (SPP_CNN_F32);
 * accumulation and master weights are fp32.  Weights are float arrays in
 * (Cout, Cin, 3, 3) layout per layer, layers concatenated; the taps are
 * w[o][c][dy + 1][dx + 1] acting on x[c][(i + dy) mod n][(j + dx) mod n]. */
enum { SPP_CNN_BF16 = 0, SPP_CNN_F32 = 1 };
typedef struct spp_cnn spp_cnn;

/* channels: HOST int32[nlayers + 1], first and last 2, all in [1, 32];
   n: a multiple of 16; max_batch: samples per call.  Weights start at 0. */
int spp_cnn_create(int32_t n, int32_t nlayers, const int32_t* channels, int32_t dtype,
                   int32_t max_batch, spp_cnn** out);
/* Sets (w_in) and/or reads (w_out) the fp32 master weights, HOST float[count];
   setting them resets the Adam state.  count (HOST, may be NULL) = number of weights. */
int spp_cnn_weights(spp_cnn* net, const float* w_in, float* w_out, int64_t* count);
/* y = net(x) per sample; x, y DEVICE complex128 [batch][n^2]. */
int spp_cnn_forward(spp_cnn* net, const void* x, int32_t batch, void* y, spp_stream_t stream);
/* Forward and backward pass of loss = mean_b ||net(x_b) - t_b||^2 / ||t_b||^2;
   x, t DEVICE complex128 [batch][n^2].  Keeps the gradient on the device for
   spp_cnn_adam_step; loss (HOST double) and grads (HOST float[count], the
   weight layout) may be NULL. */
int spp_cnn_loss_grad(spp_cnn* net, const void* x, const void* t, int32_t batch,
                      double* loss, float* grads, spp_stream_t stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with the
   last gradient. */
int spp_cnn_adam_step(spp_cnn* net, float lr, spp_stream_t stream);
void spp_cnn_destroy(spp_cnn* net);
const char* spp_cnn_last_error(void);

/* Uses net as the first preconditioner stage of every FGMRES iteration of
   spp_solve: z = s^{-1} net(s v) with s = sqrt(n^2) (v has unit norm), judged
   by the sparsifying preconditioner's standard: the step is kept when every
   column's residual estimate falls to at most rho times its previous value
   (0 < rho < 1: the residual estimates never grow, so rho = 1 would keep
   every step),
   otherwise it is discarded and redone with z = P^{-1} Q v.  After three
   discarded steps in a row the network is not tried again in that solve.
   net = NULL detaches.  Requires a single 2D problem of the network's n and
   max_batch >= nrhs.  The factor does not own net. */
int spp_attach_cnn(spp_factor* factor, spp_cnn* net, double rho);
/* Steps of the last spp_solve that used the network (accepted) or redid the
   step with the sparsifying preconditioner (rejected). HOST outputs. */
int spp_learned_stats(const spp_factor* factor, int32_t* accepted, int32_t* rejected);
/* Copies the j-th Arnoldi vector v_j and its preconditioned z_j of the last
   spp_solve (DEVICE complex128, the batch vector layout), j < iterations. */
int spp_get_krylov(const spp_factor* factor, int32_t j, void* v, void* z);

/* Releases everything the factor owns (synchronises its last stream). */
void spp_destroy(spp_factor* factor);

const char* spp_error_string(int code);
const char* spp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SPP_H_ */
