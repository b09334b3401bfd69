// C ABI of the library (include/spp.h): handle management, setup and solve
// drivers.  Host code only; every arithmetic step runs in the HIP kernels.
//
// A factor always describes a batch of problems (one problem is a batch of
// one): their fronts are concatenated level by level so that each kernel
// launch of the factorisation and of the substitution covers every problem,
// and grid vectors are stored problem after problem, [nrhs][N_i] each.
#include "spp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "plan.hpp"

namespace spp {

struct KernelTimer {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[KC_COUNT];
  double bytes[KC_COUNT] = {0};
  double flops[KC_COUNT] = {0};
  int64_t launches[KC_COUNT] = {0};
  hipEvent_t pending[KC_COUNT] = {nullptr};
  ~KernelTimer() {
    for (auto& v : ev)
      for (auto& pr : v) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
  }
};

thread_local KernelTimer* g_timer = nullptr;

void timer_begin(int cls, hipStream_t st) {
  if (!g_timer) return;
  hipEvent_t e;
  SPP_HIP(hipEventCreate(&e));
  SPP_HIP(hipEventRecord(e, st));
  g_timer->pending[cls] = e;
}

void timer_end(int cls, hipStream_t st, double bytes, double flops) {
  if (!g_timer || !g_timer->pending[cls]) return;
  hipEvent_t e;
  SPP_HIP(hipEventCreate(&e));
  SPP_HIP(hipEventRecord(e, st));
  g_timer->ev[cls].emplace_back(g_timer->pending[cls], e);
  g_timer->pending[cls] = nullptr;
  g_timer->bytes[cls] += bytes;
  g_timer->flops[cls] += flops;
  g_timer->launches[cls] += 1;
}

void throw_hip(hipError_t e, const char* what, const char* file, int line) {
  std::string m = std::string(hipGetErrorString(e)) + " in " + what + " (" + file + ":" + std::to_string(line) + ")";
  if (e == hipErrorOutOfMemory) throw Error(SPP_ENOMEM, m);
  throw Error(SPP_EHIP, m);
}

}  // namespace spp

using namespace spp;

namespace {

thread_local std::string g_last_error;

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

using Geom = std::tuple<int, int, int, int, int, int>;   // d, n, b, ordering, stencil pattern, unknowns per point

// A nested-dissection plan (of one problem or of a batch) and its device-side
// index arrays.  Plans depend only on the geometries, so they are built once
// per process and device and shared by every factor with those geometries
// (read-only on the device).
// Device (and pinned host) blocks released by factors wait here for the next
// factor that asks for the same size on the same device: a setup per solve
// would otherwise pay hipMalloc / hipFree for every buffer, milliseconds for
// the multi-GB front arena.  Exact-size reuse; at most kMemCacheBytes held;
// the cache is emptied when an allocation fails (then retried) or through
// mem_trim.  Blocks enter the cache only once the device is idle.
std::mutex g_mem_mu;
auto& g_mem_free = *new std::multimap<std::pair<int, size_t>, void*>();
size_t g_mem_cached = 0;
constexpr size_t kMemCacheBytes = (size_t)64 << 30;
constexpr int kPinnedDev = -1;

void mem_trim() {
  std::lock_guard<std::mutex> lk(g_mem_mu);
  for (auto& kv : g_mem_free) {
    if (kv.first.first == kPinnedDev) (void)hipHostFree(kv.second);
    else (void)hipFree(kv.second);
  }
  g_mem_free.clear();
  g_mem_cached = 0;
}

void* mem_get(size_t bytes, bool pinned) {
  int dev = kPinnedDev;
  if (!pinned) SPP_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    auto it = g_mem_free.find({dev, bytes});
    if (it != g_mem_free.end()) {
      void* p = it->second;
      g_mem_free.erase(it);
      g_mem_cached -= bytes;
      return p;
    }
  }
  void* p = nullptr;
  hipError_t e = pinned ? hipHostMalloc(&p, bytes) : hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    mem_trim();
    if (pinned) SPP_HIP(hipHostMalloc(&p, bytes));
    else SPP_HIP(hipMalloc(&p, bytes));
  }
  return p;
}

// The caller has made sure no queued work still uses p.
void mem_put(void* p, size_t bytes, int dev) {
  {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    if (g_mem_cached + bytes <= kMemCacheBytes) {
      g_mem_free.emplace(std::make_pair(dev, bytes), p);
      g_mem_cached += bytes;
      return;
    }
  }
  if (dev == kPinnedDev) (void)hipHostFree(p);
  else (void)hipFree(p);
}

struct PlanDevice {
  Plan plan;
  std::vector<int> front_inst;
  int device = 0;
  FrontDev* fronts = nullptr;
  AsmBlockDev* blocks = nullptr;
  int *pos = nullptr, *idx = nullptr, *map = nullptr, *gptr = nullptr;
  int64_t* gsrc = nullptr;
  std::vector<int*> type_off;      // per problem, per set type: device offsets
  std::vector<double> level_ent;   // 3 per level, see mf_solve
  std::vector<std::vector<int>> level_F, level_p;
  int perm_total = 0;
  int dblk_total = 0;              // 32-column diagonal blocks over all fronts
  int64_t xwork_elems = 0;
  std::vector<void*> mem;
  ~PlanDevice() {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(device);
    for (void* p : mem) (void)hipFree(p);
    (void)hipSetDevice(cur);
  }
};

std::mutex g_plan_mu;
// Never destroyed: device memory of cached plans is released with the process,
// not by a static destructor running after the HIP runtime has shut down.
auto& g_plans = *new std::map<std::tuple<int, int, std::vector<Geom>>, std::shared_ptr<PlanDevice>>();
auto& g_host_plans = *new std::map<Geom, std::shared_ptr<Plan>>();

// Host plan of one geometry (caller holds g_plan_mu).
std::shared_ptr<Plan> host_plan_locked(const Geom& g) {
  auto it = g_host_plans.find(g);
  if (it != g_host_plans.end()) return it->second;
  auto P = std::make_shared<Plan>();
  std::string err = build_plan(std::get<0>(g), std::get<1>(g), std::get<2>(g), std::get<3>(g), *P, std::get<4>(g));
  if (err.empty()) err = expand_plan(*P, std::get<5>(g));
  if (!err.empty()) throw Error(SPP_EINVAL, err);
  g_host_plans[g] = P;
  return P;
}

std::shared_ptr<Plan> host_plan(const Geom& g) {
  std::lock_guard<std::mutex> lock(g_plan_mu);
  return host_plan_locked(g);
}

// storage: 0 resident, 1 streamed (layout_plan).
std::shared_ptr<PlanDevice> get_plan(const std::vector<Geom>& geoms, int storage) {
  int dev = 0;
  SPP_HIP(hipGetDevice(&dev));
  const auto key = std::make_tuple(dev, storage, geoms);
  std::lock_guard<std::mutex> lock(g_plan_mu);
  auto it = g_plans.find(key);
  if (it != g_plans.end()) return it->second;
  auto pd = std::make_shared<PlanDevice>();
  pd->device = dev;
  std::vector<std::shared_ptr<Plan>> parts;
  std::vector<const Plan*> raw;
  for (const Geom& g : geoms) {
    parts.push_back(host_plan_locked(g));
    raw.push_back(parts.back().get());
  }
  if (raw.size() == 1) {
    pd->plan = *raw[0];
    pd->front_inst.assign(pd->plan.fronts.size(), 0);
  } else {
    std::string err = combine_plans(raw, pd->plan, pd->front_inst);
    if (!err.empty()) throw Error(SPP_EINVAL, err);
  }
  layout_plan(pd->plan, storage);
  const Plan& P = pd->plan;
  PlanTables tab;
  {
    std::string err = build_tables(P, pd->front_inst, tab);
    if (!err.empty()) throw Error(SPP_EINVAL, err);
  }
  std::vector<FrontDev> fd(P.fronts.size());
  for (size_t fi = 0; fi < P.fronts.size(); ++fi) {
    const FrontTable& t = tab.fronts[fi];
    FrontDev& g = fd[fi];
    g.off = t.off; g.voff = t.voff; g.xoff = t.xoff;
    g.foff = t.foff; g.uoff = t.uoff; g.ldu = t.ldu;
    g.F = t.F; g.p = t.p; g.idx = t.idx; g.map = t.map; g.perm = t.perm; g.dblk = t.dblk;
    g.inst = t.inst; g.parent = t.parent; g.nchild = t.nchild;
    for (int c = 0; c < 8; ++c) g.child[c] = t.child[c];
    g.gptr = t.gptr;
  }
  pd->level_ent = tab.level_ent;
  pd->level_F = tab.level_F;
  pd->level_p = tab.level_p;
  pd->perm_total = tab.perm_total;
  pd->dblk_total = tab.dblk_total;
  pd->xwork_elems = tab.xwork_elems;
  std::vector<AsmBlockDev> bd(P.blocks.size());
  for (size_t i = 0; i < P.blocks.size(); ++i)
    bd[i] = AsmBlockDev{P.blocks[i].front, P.blocks[i].type, P.blocks[i].anchor, P.blocks[i].rowpos, P.blocks[i].colpos};
  auto upload = [&](const void* src, size_t bytes) {
    void* p = nullptr;
    SPP_HIP(hipMalloc(&p, std::max<size_t>(bytes, 4)));
    pd->mem.push_back(p);
    if (bytes) SPP_HIP(hipMemcpy(p, src, bytes, hipMemcpyHostToDevice));
    return p;
  };
  pd->gptr = static_cast<int*>(upload(tab.gptr.data(), tab.gptr.size() * sizeof(int)));
  pd->gsrc = static_cast<int64_t*>(upload(tab.gsrc.data(), tab.gsrc.size() * sizeof(int64_t)));
  pd->fronts = static_cast<FrontDev*>(upload(fd.data(), fd.size() * sizeof(FrontDev)));
  pd->blocks = static_cast<AsmBlockDev*>(upload(bd.data(), bd.size() * sizeof(AsmBlockDev)));
  pd->pos = static_cast<int*>(upload(P.pos.data(), P.pos.size() * sizeof(int)));
  pd->idx = static_cast<int*>(upload(P.idx.data(), P.idx.size() * sizeof(int)));
  pd->map = static_cast<int*>(upload(P.map.data(), P.map.size() * sizeof(int)));
  for (const Plan* part : raw)
    for (const SetType& T : part->types)
      pd->type_off.push_back(static_cast<int*>(upload(T.off.data(), T.off.size() * sizeof(int))));
  g_plans[key] = pd;
  return pd;
}

}  // namespace

// One problem of the batch.
struct SppInstance {
  int kind = 0;
  double omega = 0, ell = 1, energy = 0, s = 0;
  int moves = 0;
  int d = 0, n = 0, b = 0, m = 0;
  int bs = 0;                        // box width of the stencil sets (b, or 1 for points)
  int nc = 1;                        // unknowns per grid point (Maxwell: d field components)
  int64_t npts = 0;                  // grid points n^d
  int64_t N = 0, Noff = 0;           // unknowns nc npts, and their offset in a batch vector
  std::shared_ptr<Plan> plan;        // the problem's own plan (set types)
  StencilDev sten[8]{};
  const double2* tw = nullptr;
};

// A run of consecutive problems with the same grid: one contiguous
// [ninst * nrhs][N] block of a batch vector.
struct SppGroup {
  int inst0 = 0, ninst = 0;
  int d = 0, n = 0;
  int nc = 1;                        // grids per problem and right-hand side
  int64_t N = 0, Noff = 0;
  const double2* tw = nullptr;
};

struct spp_factor {
  std::shared_ptr<PlanDevice> pd;   // shared, read-only plan (see get_plan)
  const Plan* planp = nullptr;
  std::vector<SppInstance> inst;
  std::vector<SppGroup> groups;
  int64_t Ntot = 0;
  spp_options opt{};
  std::vector<std::pair<void*, size_t>> allocs;   // (block, bytes)
  int device = 0;
  double* q = nullptr;               // every problem's q, concatenated
  double* sigma = nullptr;           // every problem's Green symbol / N, concatenated
  std::map<int, double2*> tw_by_n;
  InstDev* inst_dev = nullptr;
  MfDev mf{};
  void* arena = nullptr;       // front arena (released after a streamed factorisation)
  void* fstore = nullptr;      // factor store (streamed storage)
  void* fac = nullptr;         // what the substitution reads: arena or fstore
  void* dkeep = nullptr;       // diagonal-block inverses of blocked levels
  size_t csize = 16;  // bytes per complex front entry
  std::vector<int> level_begin, level_maxF, level_maxK, level_maxP, level_form;
  std::vector<int> level_var;  // step schedule per level (kVarPair, kVarTile64)
  int64_t xwork_elems = 0;     // inverse work of the levels solved by products
  void* gpart = nullptr;       // split-K partial sums of the substitution
  int64_t gpart_cap = 0;
  // solve work (grown on demand)
  int cap_rhs = 0, cap_iter = 0;
  double2* tmp = nullptr;      // FFT scratch, nrhs * Ntot
  double2* qr = nullptr;       // Q r, nrhs * Ntot
  void* wv = nullptr;          // front vectors
  void* zv = nullptr;
  void* xc = nullptr;          // reduced-precision solve vector (complex64 fronts)
  double2 *V = nullptr, *Z = nullptr, *H = nullptr, *gv = nullptr, *sn = nullptr, *y = nullptr, *g0 = nullptr,
          *wk = nullptr, *h2 = nullptr, *dpart = nullptr;
  double *cs = nullptr, *rpart = nullptr, *resid = nullptr, *norms = nullptr;
  int* kvec = nullptr;
  double* h_resid = nullptr;   // pinned host copy of residual estimates
  double* h_resid_dev = nullptr;   // its device alias (written by the Givens step)
  size_t h_resid_bytes = 0;
  hipEvent_t resid_event = nullptr;   // marks the residual estimates' copy
  spp_stats_t stats{};
  int tuned_nrhs = 0;          // right-hand-side count the last autotune covered
  spp_cnn* cnn = nullptr;      // learned FGMRES stage (not owned)
  double cnn_rho = 0.9;
  int cnn_accepted = 0, cnn_rejected = 0;
  double2* gsave = nullptr;    // Givens right-hand side before a learned step
  int last_iters_all = 0;      // Krylov vectors kept from the last solve
  int last_nrhs = 0;
  // Captured FGMRES iteration (SPP_F_GRAPHS): one graph replayed per step with
  // the step index in device memory.
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t gstream = nullptr;
  // Level inverses beside the next level's LU: one event marks a level's LU,
  // the other the end of the inverse work.
  hipEvent_t inv_event[3] = {nullptr, nullptr, nullptr};
  hipEvent_t zero_event = nullptr;   // the arena's zeroing on the side stream
  // The last level's inverses may still run on the side stream when setup
  // returns (inv_event[1] marks their end): every use of the factor waits
  // for that event first (factor_ready), and the work buffers they use are
  // returned once it has passed (factor_settled).
  bool inv_pending = false;
  std::vector<void*> inv_buffers;
  int graph_nrhs = 0;
  bool graph_precond = true;
  int* dj = nullptr;
  double2 *vfix = nullptr, *zfix = nullptr;
  void drop_graph() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    graph_exec = nullptr;
    graph_nrhs = 0;
  }
  hipStream_t last_stream = nullptr;
  std::unique_ptr<KernelTimer> timer;
  // Blocks from the caller's allocator hook (spp_options::alloc), released
  // through spp_options::free.
  std::vector<void*> hook_blocks;
  // spp_solve_batch: right-hand sides and solutions packed into the batch
  // layout with the largest per-problem count (grown on demand).
  double2 *pack_f = nullptr, *pack_u = nullptr;
  int64_t pack_cap = 0;

  template <typename T> T* dalloc(size_t count) {
    if (count == 0) count = 1;
    const size_t bytes = (count * sizeof(T) + 255) / 256 * 256;
    void* p = mem_get(bytes, false);
    allocs.push_back({p, bytes});
    return static_cast<T*>(p);
  }
  // idle: the caller has already waited for every queued use of p (else the
  // whole device is drained first).
  void dfree(void* p, bool idle = false) {
    if (!p) return;
    auto it = std::find_if(allocs.begin(), allocs.end(), [&](const std::pair<void*, size_t>& a) { return a.first == p; });
    if (it == allocs.end()) return;
    const size_t bytes = it->second;
    allocs.erase(it);
    if (!idle) (void)hipDeviceSynchronize();   // (nothing queued may still use the block)
    mem_put(p, bytes, device);
  }
  // A large block of the factor: from the caller's hook if one was given.
  void* big_alloc(size_t bytes) {
    bytes = std::max<size_t>((bytes + 255) / 256 * 256, 256);
    if (!opt.alloc) return dalloc<char>(bytes);
    void* p = opt.alloc(bytes, opt.alloc_ctx);
    if (!p) throw Error(SPP_ENOMEM, "the allocator hook returned NULL for " + std::to_string(bytes) + " bytes");
    hook_blocks.push_back(p);
    return p;
  }
  void big_free(void* p) {
    if (!p) return;
    auto it = std::find(hook_blocks.begin(), hook_blocks.end(), p);
    if (it != hook_blocks.end()) {
      (void)hipDeviceSynchronize();
      hook_blocks.erase(it);
      opt.free(p, opt.alloc_ctx);
      return;
    }
    dfree(p);
  }
  ~spp_factor() {
    drop_graph();
    if (gstream) (void)hipStreamDestroy(gstream);
    for (hipEvent_t e : inv_event)
      if (e) (void)hipEventDestroy(e);
    if (zero_event) (void)hipEventDestroy(zero_event);
    (void)hipDeviceSynchronize();
    for (void* p : hook_blocks) opt.free(p, opt.alloc_ctx);
    for (const auto& a : allocs) mem_put(a.first, a.second, device);
    if (h_resid) mem_put(h_resid, h_resid_bytes, kPinnedDev);
    if (resid_event) (void)hipEventDestroy(resid_event);
  }
};

namespace {

// Makes the factor's kernel timer current for the duration of one ABI call.
struct TimerScope {
  KernelTimer* prev;
  explicit TimerScope(spp_factor* F) : prev(g_timer) { g_timer = (F && F->timer) ? F->timer.get() : nullptr; }
  ~TimerScope() { g_timer = prev; }
};

int fail(const Error& e) {
  g_last_error = e.what();
  return e.code;
}

template <typename F> int guarded(F&& fn) {
  try {
    return fn();
  } catch (const Error& e) {
    return fail(e);
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return SPP_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return SPP_EHIP;
  }
}

// min over the Fourier grid of |4 pi^2 |k|^2 - s| / |s| (how close L - s is to singular).
// min over wave numbers k in [-n/2, n/2)^d of |4 pi^2 |k|^2 - s|, relative to
// |s|: the last coordinate is taken next to the square root of what the
// others leave, so the scan is O(n^(d-1)).
// nyquist_zero: the wave numbers of first derivatives (the vector curl curl),
// whose Nyquist entry -n/2 counts as 0.
double shift_gap(int d, int n, double s, bool nyquist_zero = false) {
  const double c = 4.0 * M_PI * M_PI;
  const int h = n / 2;
  const int top = nyquist_zero ? h - 1 : h;   // largest |k| of the last coordinate
  auto sq = [&](int a) { return (nyquist_zero && a == -h) ? 0.0 : (double)a * a; };
  double best = INFINITY;
  auto last = [&](double partial) {   // partial = sum of the other squares
    const double rest = s / c - partial;
    const int k = rest > 0 ? (int)std::floor(std::sqrt(rest)) : 0;
    for (int t = std::max(0, k - 1); t <= std::min(top, k + 2); ++t)
      best = std::min(best, std::fabs(c * (partial + (double)t * t) - s));
  };
  if (d == 2) {
    for (int a = -h; a < h; ++a) last(sq(a));
  } else {
    for (int a = -h; a < h; ++a)
      for (int b = -h; b < h; ++b) last(sq(a) + sq(b));
  }
  return best / std::fabs(s);
}

// The stream that runs level inverses beside the factorisation, one per
// device for the life of the process (default priority; work from
// different factors is ordered on it by events only).
hipStream_t side_stream() {
  static std::mutex mu;
  static hipStream_t streams[64] = {nullptr};
  int dev = 0;
  SPP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) throw Error(-7, "device index beyond the side-stream table");
  std::lock_guard<std::mutex> lk(mu);
  if (!streams[dev]) SPP_HIP(hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking));
  return streams[dev];
}

void factor_ready(spp_factor* F, hipStream_t st) {
  if (F->inv_pending) SPP_HIP(hipStreamWaitEvent(st, F->inv_event[1], 0));
}

void factor_settled(spp_factor* F) {
  if (!F->inv_pending) return;
  SPP_HIP(hipEventSynchronize(F->inv_event[1]));
  for (void* p : F->inv_buffers) F->dfree(p);
  F->inv_buffers.clear();
  F->inv_pending = false;
}

int total_cols(const spp_factor* F, int nrhs) { return static_cast<int>(F->inst.size()) * nrhs; }

void ensure_solve_buffers(spp_factor* F, int nrhs, int iters) {
  if (nrhs <= F->cap_rhs && iters <= F->cap_iter) return;
  F->drop_graph();
  const int r = std::max(nrhs, F->cap_rhs), it = std::max(iters, F->cap_iter);
  for (void* p : {(void*)F->tmp, (void*)F->qr, F->wv, F->zv, F->xc, F->gpart, (void*)F->V, (void*)F->Z, (void*)F->H,
                  (void*)F->gv, (void*)F->sn, (void*)F->y, (void*)F->g0, (void*)F->wk, (void*)F->h2,
                  (void*)F->dpart, (void*)F->cs, (void*)F->rpart, (void*)F->resid, (void*)F->norms, (void*)F->kvec,
                  (void*)F->gsave, (void*)F->vfix, (void*)F->zfix, (void*)F->dj})
    F->dfree(p);
  if (F->h_resid) { mem_put(F->h_resid, F->h_resid_bytes, kPinnedDev); F->h_resid = nullptr; F->h_resid_dev = nullptr; }
  const int64_t N = F->Ntot;
  const int cols = total_cols(F, r);
  F->tmp = F->dalloc<double2>((size_t)r * N);
  F->qr = F->dalloc<double2>((size_t)r * N);
  F->wv = F->dalloc<char>((size_t)F->planp->vec_elems * r * F->csize);
  F->zv = F->dalloc<char>((size_t)F->planp->vec_elems * r * F->csize);
  F->xc = F->dalloc<char>((size_t)N * r * F->csize);
  F->gpart_cap = ((int64_t)1 << 20) * r;
  F->gpart = F->dalloc<char>((size_t)F->gpart_cap * F->csize);
  F->V = F->dalloc<double2>((size_t)(it + 1) * r * N);
  F->Z = F->dalloc<double2>((size_t)it * r * N);
  const size_t ld = it + 1;
  F->H = F->dalloc<double2>(ld * it * cols);
  F->gv = F->dalloc<double2>(ld * cols);
  F->sn = F->dalloc<double2>(ld * cols);
  F->y = F->dalloc<double2>(ld * cols);
  F->cs = F->dalloc<double>(ld * cols);
  F->g0 = F->dalloc<double2>((size_t)r * N);
  F->wk = F->dalloc<double2>((size_t)r * N);
  F->h2 = F->dalloc<double2>(ld * cols);
  F->gsave = F->dalloc<double2>(ld * cols);
  F->vfix = F->dalloc<double2>((size_t)r * N);
  F->zfix = F->dalloc<double2>((size_t)r * N);
  F->dj = F->dalloc<int>(1);
  int64_t nblk = 1;
  for (const SppGroup& g : F->groups) nblk = std::max<int64_t>(nblk, kr_dot_slots(g.N));
  F->dpart = F->dalloc<double2>((size_t)nblk * cols * (it + 1));
  F->rpart = F->dalloc<double>((size_t)(256 + 1) * cols + 64);
  F->resid = F->dalloc<double>(cols);
  F->norms = F->dalloc<double>(cols);
  F->kvec = F->dalloc<int>(cols);
  F->h_resid_bytes = sizeof(double) * cols;
  F->h_resid = static_cast<double*>(mem_get(F->h_resid_bytes, true));
  SPP_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&F->h_resid_dev), F->h_resid, 0));
  F->cap_rhs = r;
  F->cap_iter = it;
}

// w = (I + G q) z; one FFT call per group of equal grids, q and sigma per problem.
// A vector problem (Maxwell: one problem, d grids per right-hand side) runs
// its transforms over all nrhs d grids with the d x d Green symbol in between.
void apply_operator_to(spp_factor* F, const double2* z, double2* w, double2* tmp, int nrhs, hipStream_t st) {
  for (const SppGroup& g : F->groups) {
    const int64_t o = g.Noff * nrhs;
    if (g.nc > 1)
      fft_vector_green(st, z + o, w + o, tmp + o, g.tw, g.d, g.n, nrhs, F->inst[g.inst0].s, F->q + g.Noff, z + o);
    else
      fft_multi(st, z + o, w + o, tmp + o, g.tw, g.d, g.n, g.ninst * nrhs, F->q + g.Noff, F->sigma + g.Noff, z + o,
                nrhs);
  }
}

void apply_operator(spp_factor* F, const double2* z, double2* w, int nrhs, hipStream_t st) {
  apply_operator_to(F, z, w, F->tmp, nrhs, st);
}

void apply_green(spp_factor* F, const double2* f, double2* gout, int nrhs, hipStream_t st) {
  for (const SppGroup& g : F->groups) {
    const int64_t o = g.Noff * nrhs;
    if (g.nc > 1)
      fft_vector_green(st, f + o, gout + o, F->tmp + o, g.tw, g.d, g.n, nrhs, F->inst[g.inst0].s, nullptr, nullptr);
    else
      fft_multi(st, f + o, gout + o, F->tmp + o, g.tw, g.d, g.n, g.ninst * nrhs, nullptr, F->sigma + g.Noff, nullptr,
                nrhs);
  }
}

// persistent: cooperative launches for runs of small-front levels (not inside
// a graph capture).
// The preconditioner in two parts: the head (Q r, and its cast to the front
// precision) fills scratch vectors only, so it can run ahead of the decision
// whether its result is needed; the tail (the substitution and the cast
// back) writes z.
void precond_head(spp_factor* F, const double2* r, int nrhs, hipStream_t st) {
  if (F->opt.prec == SPP_C128) q_apply(st, F->mf, r, F->qr, nrhs);
  else q_apply(st, F->mf, r, F->xc, nrhs, true);   // rounded to complex64 on the store
}

void precond_tail(spp_factor* F, double2* z, int nrhs, hipStream_t st, bool persistent) {
  // (with inverses still in the making, the substitution waits for them only
  // before the levels that read them: the earlier levels' before the first
  // such level, the last level's before it)
  hipEvent_t early = F->inv_pending ? F->inv_event[2] : nullptr;
  hipEvent_t last = F->inv_pending ? F->inv_event[1] : nullptr;
  persistent = persistent && (F->opt.flags & SPP_F_PERSISTENT);
  const int nl = static_cast<int>(F->planp->levels.size());
  const double* ent = F->pd->level_ent.data();
  if (F->opt.prec == SPP_C128) {
    mf_solve<double>(st, F->mf, F->fac, F->wv, F->zv, F->qr, z, nrhs, F->level_begin.data(), F->level_maxF.data(), F->level_maxK.data(),
                     F->level_maxP.data(), ent, F->level_form.data(), nl, F->gpart, F->gpart_cap, persistent, nullptr,
                     early, last);
  } else {
    mf_solve<float>(st, F->mf, F->fac, F->wv, F->zv, F->xc, F->xc, nrhs, F->level_begin.data(), F->level_maxF.data(), F->level_maxK.data(),
                    F->level_maxP.data(), ent, F->level_form.data(), nl, F->gpart, F->gpart_cap, persistent, nullptr,
                    early, last);
    cast_vectors<float>(st, F->xc, z, (int64_t)nrhs * F->Ntot, 1);
  }
}

void apply_precond(spp_factor* F, const double2* r, double2* z, int nrhs, hipStream_t st, bool persistent = true) {
  precond_head(F, r, nrhs, st);
  precond_tail(F, z, nrhs, st, persistent);
}

// Tuning-table keys of a level's solve form and step schedule: front
// precision and the level's shape (fronts, largest F, largest p).
std::string form_tune_key(size_t csize, const Level& L) {
  return tune_key("mf_form", {(int64_t)csize, L.end - L.begin, L.maxF, L.maxP});
}
std::string var_tune_key(size_t csize, const Level& L) {
  return tune_key("mf_steps", {(int64_t)csize, L.end - L.begin, L.maxF, L.maxP});
}
// Forms a tuned level may take: the whole-front solve kernels hold the
// front's vectors of four right-hand sides and a 32 x 33 diagonal block in
// 64 KB of LDS; the side products unless the caller turned them off.
// (Blocked levels are not tuned.)
bool form_valid(int form, const Level& L, size_t csize, int32_t flags) {
  if (form == kFormLU) return ((int64_t)(L.maxF + L.maxP) * 4 + 32 * 33) * (int64_t)csize <= 65536;
  if (form == kFormInverse) return true;
  if (form == kFormSide) return !(flags & SPP_F_NO_SIDE);
  return false;
}
// The tuning pass weighs a level's substitution time (forward and backward)
// against its factorisation time as this many preconditioner applies per
// factorisation.
constexpr double kTuneAppliesPerFactor = 20.0;

void validate_problem(const spp_problem* pb) {
  if (!pb->coeff) throw Error(SPP_EINVAL, "coeff is null");
  if (pb->kind != SPP_HELMHOLTZ && pb->kind != SPP_SCHRODINGER && pb->kind != SPP_MAXWELL)
    throw Error(SPP_EINVAL, "unknown problem kind");
  if ((pb->kind == SPP_HELMHOLTZ || pb->kind == SPP_MAXWELL) && !(std::isfinite(pb->omega) && pb->omega > 0))
    throw Error(SPP_EINVAL, "omega");
  if (pb->kind == SPP_SCHRODINGER && !(std::isfinite(pb->ell) && pb->ell > 0 && std::isfinite(pb->energy)))
    throw Error(SPP_EINVAL, "ell / energy");
  if (!fft_supported(pb->n)) throw Error(SPP_EINVAL, "n must be of the form 2^a 3^b");
  std::string err = validate_grid(pb->dim, pb->n, pb->b);
  if (!err.empty()) throw Error(SPP_EINVAL, err);
  // Leaf sets are assembled and applied by one workgroup with their
  // neighbourhood's unknowns staged in LDS: nc |gamma(S)| <= 1024 (scalar
  // 2D: b <= 30, 3D: b <= 9; Maxwell, nc = d: 2D b <= 21, 3D b <= 5).
  const int nc = pb->kind == SPP_MAXWELL ? pb->dim : 1;
  const int g = (pb->dim == 2) ? (pb->b + 1) * (pb->b + 1) : (pb->b + 1) * (pb->b + 1) * (pb->b + 1);
  if (nc * g > 1024) throw Error(SPP_ENOTIMPL, "leaf box too large: unknowns per point times (b + 1)^d must be <= 1024");
}

// Times the candidate launch parameters of this factor's FFT passes and
// substitution products (right-hand-side count nrhs) and stores the fastest
// in the process-wide tuning table (and its file, if SPP_TUNE_CACHE is set).
void do_autotune(spp_factor* F, int nrhs, hipStream_t st) {
  ensure_solve_buffers(F, nrhs, F->opt.max_iter);
  KernelTimer* saved = g_timer;
  g_timer = nullptr;
  const int64_t vstride = (int64_t)nrhs * F->Ntot;
  // Scratch contents and the cache-flushing buffer are set up, and the factor's
  // pending inverses waited for, only when some key is missing (a factor
  // whose shapes are all tuned costs nothing here).
  const size_t flush_bytes = (size_t)768 << 20;
  void* flush = nullptr;
  auto prepare = [&] {
    if (flush) return;
    factor_ready(F, st);   // (the candidates run on the complete factor)
    SPP_HIP(hipMemsetAsync(F->wk, 0, sizeof(double2) * vstride, st));
    SPP_HIP(hipMemsetAsync(F->tmp, 0, sizeof(double2) * vstride, st));
    SPP_HIP(hipMemsetAsync(F->qr, 0, sizeof(double2) * vstride, st));
    SPP_HIP(hipMemsetAsync(F->wv, 0, (size_t)F->planp->vec_elems * nrhs * F->csize, st));
    SPP_HIP(hipMemsetAsync(F->zv, 0, (size_t)F->planp->vec_elems * nrhs * F->csize, st));
    SPP_HIP(hipMemsetAsync(F->xc, 0, (size_t)F->Ntot * nrhs * F->csize, st));
    flush = F->dalloc<char>(flush_bytes);
  };
  for (const SppGroup& g : F->groups) {
    const int batch = g.ninst * nrhs * g.nc;   // grids per pass
    const int64_t o = g.Noff * nrhs, n = g.n;
    std::vector<std::pair<int64_t, int64_t>> axes;
    if (g.d == 2) axes = {{n, 1}, {1, n}};
    else axes = {{n * n, 1}, {n, n}, {1, n * n}};
    for (const auto& ax : axes) {
      const std::string key = fft_tune_key(g.n, ax.first, ax.second, batch);
      if (tune_has(key)) continue;
      prepare();
      int best = fft_lines_default(g.n, ax.first, ax.second);
      float bt = 1e30f;
      for (int L = 1; (int64_t)L * n <= 4096; L *= 2) {
        if (!fft_lines_valid(g.n, ax.first, ax.second, L)) continue;
        tune_force(key, L);
        const float t = tune_time(st, 3, [&] {
          fft_axis(st, F->wk + o, F->tmp + o, g.tw, g.n, ax.first, ax.second, g.N / g.nc, batch, -1, nullptr,
                   nullptr, nullptr, nrhs * g.nc);
        });
        if (t < bt) { bt = t; best = L; }
      }
      tune_force(key, -1);
      tune_set(key, best);
    }
  }
  const Plan& P = *F->planp;
  // (the substitution candidates are timed with cold caches, see tune_time)
  for (size_t l = 0; l < P.levels.size(); ++l) {
    if (F->level_form[l] == kFormLU) continue;
    const Level& L = P.levels[l];
    const int nf = L.end - L.begin, mP = L.maxP, mF = L.maxF, mK = L.maxK;
    struct Prod { int rows, cols, mode; };
    std::vector<Prod> prods;
    if (F->level_form[l] == kFormBlocked) {
      if (mK > 0) prods = {{mK, mP, 1}, {mP, mK, 2}};
    } else if (F->level_form[l] == kFormSide) {
      prods = {{mF, mP, 4}, {mP, mF, 5}};
    } else {
      prods = {{mP, mP, 0}, {mP, mP, 3}};
      if (mK > 0) { prods.push_back({mK, mP, 1}); prods.push_back({mP, mK, 2}); }
    }
    for (const Prod& pr : prods) {
      const std::string key = gemv_tune_key(pr.rows, pr.cols, nf, pr.mode, nrhs, (int)F->csize);
      if (tune_has(key)) continue;
      prepare();
      int best = gemv_chunks_default(pr.rows, pr.cols, nf, nrhs, F->gpart_cap);
      float bt = 1e30f;
      // c = 0: 16-row tiles with the columns not split; c >= 1: 64-row tiles
      // with the columns split over c workgroups; kGemvNarrowSplit + c (c >= 2):
      // 16-row tiles with the columns split over c workgroups.
      auto candidate = [&](int v) {
        const float t = tune_time(st, 3, [&] {
          if (F->opt.prec == SPP_C128)
            mf_gemv<double>(st, F->mf, F->fac, F->wv, F->zv, F->qr, F->qr, nrhs, L.begin, nf, pr.rows, pr.cols, pr.mode,
                            0.0, F->gpart, F->gpart_cap, v);
          else
            mf_gemv<float>(st, F->mf, F->fac, F->wv, F->zv, F->xc, F->xc, nrhs, L.begin, nf, pr.rows, pr.cols, pr.mode,
                           0.0, F->gpart, F->gpart_cap, v);
        }, flush, flush_bytes);
        if (t < bt) { bt = t; best = v; }
      };
      for (int c = 0; c <= std::max(1, pr.cols / 16) && c <= 256; c = c ? 2 * c : 1) {
        if ((int64_t)nf * c * pr.rows * nrhs > F->gpart_cap) break;
        candidate(c);
      }
      for (int c = 2; c <= std::max(1, pr.cols / 64) && c <= 64; c *= 2) {
        if ((int64_t)nf * c * pr.rows * nrhs > F->gpart_cap) break;
        candidate(kGemvNarrowSplit + c);
      }
      tune_set(key, best);
    }
  }
  if (flush) {
    SPP_HIP(hipStreamSynchronize(st));
    F->dfree(flush);
    tune_save();
  }
  g_timer = saved;
  F->tuned_nrhs = nrhs;
}

// Tuning pass of the factorisation (SPP_F_AUTOTUNE, resident storage): the
// whole factorisation runs once per candidate, with HIP events around every
// level, and each level keeps its fastest candidate (levels are timed
// separately, so one run serves them all):
//  1. each solve form (LU in place, inverses, side products) on every level
//     where it is valid, scored as the level's factorisation time plus
//     kTuneAppliesPerFactor times its substitution time (one right-hand
//     side, forward and backward, the best of three);
//  2. with those forms, each step schedule (single, fused single or paired
//     steps; 64 x 64 or 128 x 32 / 32 x 128 L21 / U12 tiles), scored by
//     factorisation time.
// The choices go to the tuning table (keys mf_form / mf_steps with the
// level's shape) and into F's level_form / level_var.  factor_all(forms,
// vars, events) assembles and factors every level.
template <typename FactorAll>
void tune_factorisation(spp_factor* F, FactorAll&& factor_all, hipStream_t st) {
  const Plan& P = *F->planp;
  const int nl = static_cast<int>(P.levels.size());
  KernelTimer* saved_timer = g_timer;   // (tuning runs are not the caller's kernel time)
  g_timer = nullptr;
  std::vector<hipEvent_t> ev(4 * (size_t)nl);
  for (hipEvent_t& e : ev) SPP_HIP(hipEventCreate(&e));
  const size_t cs = F->csize;
  void* tw = F->dalloc<char>((size_t)P.vec_elems * cs);
  void* tz = F->dalloc<char>((size_t)P.vec_elems * cs);
  void* tin = F->dalloc<char>((size_t)F->Ntot * cs);
  void* tout = F->dalloc<char>((size_t)F->Ntot * cs);
  const int64_t tcap = (int64_t)1 << 20;
  void* tpart = F->dalloc<char>((size_t)tcap * cs);
  for (void* b : {tw, tz})
    SPP_HIP(hipMemsetAsync(b, 0, (size_t)P.vec_elems * cs, st));
  for (void* b : {tin, tout}) SPP_HIP(hipMemsetAsync(b, 0, (size_t)F->Ntot * cs, st));
  auto elapsed = [&](hipEvent_t a, hipEvent_t b) {
    float ms = 0;
    SPP_HIP(hipEventElapsedTime(&ms, a, b));
    return (double)ms;
  };
  // (small factorisations run each candidate twice and keep the faster run)
  const int reps = P.factor_flops < 2e11 ? 2 : 1;
  auto factor_times = [&](const std::vector<int>& forms, const std::vector<int>& vars) {
    std::vector<double> t(nl, 1e30);
    for (int r = 0; r < reps; ++r) {
      factor_all(forms, vars, ev.data());
      SPP_HIP(hipStreamSynchronize(st));
      for (int l = 0; l < nl; ++l) t[l] = std::min(t[l], elapsed(ev[2 * l], ev[2 * l + 1]));
    }
    return t;
  };
  auto solve_times = [&](const std::vector<int>& forms) {
    std::vector<double> t(nl, 1e30);
    const double* ent = F->pd->level_ent.data();
    for (int r = 0; r < 3; ++r) {
      if (F->opt.prec == SPP_C128)
        mf_solve<double>(st, F->mf, F->arena, tw, tz, tin, tout, 1, F->level_begin.data(), F->level_maxF.data(),
                         F->level_maxK.data(), F->level_maxP.data(), ent, forms.data(), nl, tpart, tcap, false,
                         ev.data());
      else
        mf_solve<float>(st, F->mf, F->arena, tw, tz, tin, tout, 1, F->level_begin.data(), F->level_maxF.data(),
                        F->level_maxK.data(), F->level_maxP.data(), ent, forms.data(), nl, tpart, tcap, false,
                        ev.data());
      SPP_HIP(hipStreamSynchronize(st));
      for (int l = 0; l < nl; ++l)
        t[l] = std::min(t[l], elapsed(ev[4 * l], ev[4 * l + 1]) + elapsed(ev[4 * l + 2], ev[4 * l + 3]));
    }
    return t;
  };
  std::vector<int> forms = F->level_form, vars = F->level_var;
  std::vector<double> best(nl, 1e30);
  std::vector<int> best_form = forms;
  for (int cand : {kFormLU, kFormInverse, kFormSide}) {
    std::vector<int> fc = forms;
    bool any = false;
    for (int l = 0; l < nl; ++l) {
      if (forms[l] == kFormBlocked || !form_valid(cand, P.levels[l], cs, F->opt.flags)) continue;
      fc[l] = cand;
      any = true;
    }
    if (!any) continue;
    const std::vector<double> tf = factor_times(fc, vars);
    const std::vector<double> ts = solve_times(fc);
    for (int l = 0; l < nl; ++l) {
      if (fc[l] != cand) continue;
      const double score = tf[l] + kTuneAppliesPerFactor * ts[l];
      if (score < best[l]) { best[l] = score; best_form[l] = cand; }
    }
  }
  std::vector<double> bt(nl, 1e30);
  std::vector<int> best_var = vars;
  for (int v : {kVarTile64, 0, kVarPair, kVarPair | kVarTile64, kVarFused | kVarTile64, kVarFused}) {
    const std::vector<int> vc(nl, v);
    const std::vector<double> tf = factor_times(best_form, vc);
    for (int l = 0; l < nl; ++l)
      if (tf[l] < bt[l]) { bt[l] = tf[l]; best_var[l] = v; }
  }
  for (int l = 0; l < nl; ++l) {
    if (forms[l] == kFormBlocked) continue;
    tune_set(form_tune_key(cs, P.levels[l]), best_form[l]);
    tune_set(var_tune_key(cs, P.levels[l]), best_var[l]);
  }
  tune_save();
  F->level_form = best_form;
  F->level_var = best_var;
  for (hipEvent_t& e : ev) (void)hipEventDestroy(e);
  for (void* b : {tw, tz, tin, tout, tpart}) F->dfree(b);
  g_timer = saved_timer;
}

int do_setup(const spp_problem* pbs, int count, const spp_options* op, hipStream_t st, spp_factor** out) {
  if (!pbs || !op || !out) throw Error(SPP_EINVAL, "null argument");
  *out = nullptr;
  if (count < 1 || count > 4096) throw Error(SPP_EINVAL, "batch size must be in [1, 4096]");
  if (op->prec != SPP_C128 && op->prec != SPP_C64_FRONTS) throw Error(SPP_EINVAL, "unknown precision");
  if (op->order != SPP_ORDER_OCTREE && op->order != SPP_ORDER_BISECT) throw Error(SPP_EINVAL, "unknown ordering");
  if (!(op->tol > 0) || op->max_iter < 1 || op->max_iter > 500) throw Error(SPP_EINVAL, "tol > 0 and 1 <= max_iter <= 500");
  if (op->restart < 0 || op->restart > 500) throw Error(SPP_EINVAL, "restart must be in [0, 500]");
  if (op->pattern != 0 && op->pattern != 1) throw Error(SPP_EINVAL, "spp_options::pattern must be 0 or 1");
  if ((op->alloc == nullptr) != (op->free == nullptr)) throw Error(SPP_EINVAL, "give both alloc and free, or neither");
  for (int i = 0; i < count; ++i) {
    validate_problem(&pbs[i]);
    if (pbs[i].dim != pbs[0].dim) throw Error(SPP_EINVAL, "all problems of a batch must have the same dimension");
    if (pbs[i].kind == SPP_MAXWELL && count > 1)
      throw Error(SPP_ENOTIMPL, "Maxwell problems are set up one at a time (spp_setup)");
  }
  const double t0 = now_ms();
  auto F = std::make_unique<spp_factor>();
  SPP_HIP(hipGetDevice(&F->device));
  SPP_HIP(hipEventCreateWithFlags(&F->resid_event, hipEventDisableTiming));
  F->opt = *op;
  F->csize = (op->prec == SPP_C128) ? sizeof(double2) : sizeof(float2);
  F->last_stream = st;
  if (op->flags & SPP_F_TIMING) F->timer = std::make_unique<KernelTimer>();
  TimerScope timer_scope(F.get());
  std::vector<Geom> geoms;
  for (int i = 0; i < count; ++i) {
    geoms.emplace_back(pbs[i].dim, pbs[i].n, pbs[i].b, op->order, op->pattern,
                       pbs[i].kind == SPP_MAXWELL ? pbs[i].dim : 1);
  }
  // Storage: every front resident unless asked for, or unless the resident
  // arena (sum of F^2 over all fronts) would not fit in 85% of what the
  // device has left.
  int storage = (op->flags & SPP_F_STREAMED) ? 1 : 0;
  if (!storage) {
    int64_t resident = 0;
    for (const Geom& g : geoms) resident += host_plan(g)->arena_elems;
    size_t freeb = 0, totalb = 0;
    SPP_HIP(hipMemGetInfo(&freeb, &totalb));
    size_t cached = 0;
    {
      std::lock_guard<std::mutex> lk(g_mem_mu);
      cached = g_mem_cached;
    }
    if ((double)resident * F->csize > 0.85 * (double)(freeb + cached)) storage = 1;
  }
  F->pd = get_plan(geoms, storage);
  F->planp = &F->pd->plan;
  const Plan& P = *F->planp;
  bool tune_fac = false;   // run the factorisation tuning pass (below)
  size_t spare_bytes = 0;  // device memory the memory plan leaves over (0: caller-owned memory)

  // Problems, and groups of consecutive problems with equal grids.
  int64_t Noff = 0;
  for (int i = 0; i < count; ++i) {
    SppInstance I;
    I.kind = pbs[i].kind; I.omega = pbs[i].omega; I.ell = pbs[i].ell; I.energy = pbs[i].energy;
    I.d = pbs[i].dim; I.n = pbs[i].n; I.b = pbs[i].b; I.m = I.n / I.b;
    I.bs = op->pattern == 1 ? 1 : I.b;
    I.nc = I.kind == SPP_MAXWELL ? I.d : 1;
    I.npts = (I.d == 2) ? (int64_t)I.n * I.n : (int64_t)I.n * I.n * I.n;
    I.N = I.nc * I.npts;
    I.Noff = Noff;
    I.plan = host_plan(geoms[i]);
    Noff += I.N;
    F->inst.push_back(std::move(I));
  }
  F->Ntot = Noff;
  for (int i = 0; i < count; ++i) {
    const SppInstance& I = F->inst[i];
    if (F->groups.empty() || F->groups.back().n != I.n) {
      SppGroup g;
      g.inst0 = i; g.d = I.d; g.n = I.n; g.nc = I.nc; g.N = I.N; g.Noff = I.Noff;
      F->groups.push_back(g);
    }
    F->groups.back().ninst += 1;
  }
  // Memory plan: every device block of the setup, known from the plan
  // alone, checked against what the device can still give before any launch.
  {
    size_t stencil_elems = 0;
    int64_t Nmax_ = 0;   // (Green symbols and kernels: nc^2 grids per problem)
    for (const SppInstance& I : F->inst) {
      size_t w = 0;
      const size_t c = I.nc;
      for (const SetType& T : I.plan->types)
        w += c * c * ((size_t)T.nG * T.nG + (size_t)T.nG * T.nB + (size_t)T.nB * (T.nB + T.nS) + 2 * (size_t)T.nS * T.nG);
      stencil_elems += w;
      Nmax_ = std::max<int64_t>(Nmax_, (int64_t)I.nc * I.nc * I.npts);
    }
    // Solve form and step schedule per level: the tuned choice where the
    // tuning table has one for the level's shape, else the heuristic.  A
    // tuning pass (SPP_F_AUTOTUNE, resident storage, some level untuned)
    // tries the forms on every level, so its inverse work is sized for all.
    tune_fac = (op->flags & SPP_F_AUTOTUNE) && P.storage == 0 && !(op->flags & SPP_F_PARTIAL_PIVOTING);
    bool untuned = false;
    int64_t xwork_all = 0;
    for (const Level& L : P.levels) {
      const int nf = L.end - L.begin;
      int form = mf_level_solve_form(nf, L.maxF, L.maxP, op->prec == SPP_C64_FRONTS, P.storage == 1);
      int var = mf_default_variant(nf);
      if (form != kFormBlocked && P.storage == 0) {
        const int tf = tune_get(form_tune_key(F->csize, L), -1);
        if (tf >= 0 && form_valid(tf, L, F->csize, op->flags)) form = tf;
        else untuned = true;
        const int tv = tune_get(var_tune_key(F->csize, L), -1);
        if (tv >= 0 && tv <= kVarAll) var = tv;
        else untuned = true;
      }
      if (form == kFormSide && (op->flags & SPP_F_NO_SIDE)) form = kFormInverse;
      F->level_form.push_back(form);
      F->level_var.push_back(var);
      int64_t xo = 0;
      for (int fi = L.begin; fi < L.end; ++fi) xo += 2LL * P.fronts[fi].p * P.fronts[fi].F;
      if (form == kFormInverse || form == kFormSide) F->xwork_elems = std::max(F->xwork_elems, xo);
      if (form != kFormBlocked) xwork_all = std::max(xwork_all, xo);
    }
    tune_fac = tune_fac && untuned;
    const size_t cs = F->csize;
    auto need_bytes = [&](int64_t xwork) {
      return ((size_t)P.arena_elems + (size_t)P.fstore_elems) * cs + (size_t)xwork * cs * 3 / 2 +
             (size_t)2 * 32 * 32 * F->pd->dblk_total * cs + sizeof(double2) * stencil_elems +
             sizeof(double) * 2 * (size_t)F->Ntot + sizeof(double2) * 4 * (size_t)Nmax_ +
             sizeof(int) * 3 * (size_t)F->pd->perm_total + sizeof(unsigned) * P.fronts.size();
    };
    size_t need = need_bytes(F->xwork_elems);
    F->stats.device_bytes = (int64_t)need;
    if (!op->alloc) {
      size_t freeb = 0, totalb = 0;
      SPP_HIP(hipMemGetInfo(&freeb, &totalb));
      size_t cached = 0;
      {
        std::lock_guard<std::mutex> lk(g_mem_mu);
        cached = g_mem_cached;
      }
      spare_bytes = freeb + cached > need ? freeb + cached - need : 0;
      // (the tuning pass, with the inverse work of every level and its own
      // solve vectors, runs only where that fits besides the rest)
      const size_t tune_extra = (size_t)(2 * P.vec_elems + 2 * F->Ntot + (1 << 20)) * cs;
      if (tune_fac && need_bytes(std::max(F->xwork_elems, xwork_all)) + tune_extra > (freeb + cached) * 0.9)
        tune_fac = false;
      if (need > freeb + cached)
        throw Error(SPP_ENOMEM, "memory plan: the setup needs " + std::to_string(need >> 20) + " MiB, the device has " +
                                    std::to_string((freeb + cached) >> 20) + " MiB free");
    } else {
      tune_fac = false;   // (caller-owned memory: no extra blocks for tuning)
    }
    if (tune_fac) F->xwork_elems = std::max(F->xwork_elems, xwork_all);
  }
  const bool streamed = P.storage == 1;
  F->arena = F->big_alloc((size_t)P.arena_elems * F->csize);
  // A resident arena from the library's own memory (no pending user of it)
  // is zeroed on the side stream at once, before any other work of the setup
  // is queued, so that the fill runs beside the coefficient and stencil work.
  bool arena_zero_ahead = false;
  if (!streamed && !F->opt.alloc) {
    hipStream_t zs = side_stream();
    if (!F->zero_event) SPP_HIP(hipEventCreateWithFlags(&F->zero_event, hipEventDisableTiming));
    SPP_HIP(hipMemsetAsync(F->arena, 0, (size_t)P.arena_elems * F->csize, zs));
    SPP_HIP(hipEventRecord(F->zero_event, zs));
    arena_zero_ahead = true;
  }
  F->q = F->dalloc<double>(F->Ntot);
  F->sigma = F->dalloc<double>(F->Ntot);
  for (SppInstance& I : F->inst) {
    auto it = F->tw_by_n.find(I.n);
    if (it == F->tw_by_n.end()) {
      double2* tw = F->dalloc<double2>(I.n);
      fft_make_twiddles(tw, I.n, st);
      it = F->tw_by_n.emplace(I.n, tw).first;
    }
    I.tw = it->second;
  }
  for (SppGroup& g : F->groups) g.tw = F->inst[g.inst0].tw;

  int* info = F->dalloc<int>(64);
  SPP_HIP(hipMemsetAsync(info, 0, 64 * sizeof(int), st));
  size_t work_elems = 0;
  int64_t Nmax = 0, Gmax = 0;   // grid points; entries of the nc^2 Green kernels
  for (const SppInstance& I : F->inst) {
    Nmax = std::max(Nmax, I.npts);
    Gmax = std::max<int64_t>(Gmax, (int64_t)I.nc * I.nc * I.npts);
    size_t w = 0;
    const size_t c = I.nc;
    for (const SetType& T : I.plan->types)
      w += c * c * ((size_t)T.nG * T.nG + (size_t)T.nG * T.nB + (size_t)T.nB * (T.nB + T.nS));
    work_elems = std::max(work_elems, w);
  }
  double2* swork = F->dalloc<double2>(work_elems);
  const int nblk_max = coeff_reduce_blocks(Nmax);
  double* red = F->dalloc<double>(2 * nblk_max + 2);
  double* red_out = red + 2 * nblk_max;
  double2* sig_c = F->dalloc<double2>(Gmax);
  double2* sig2_c = F->dalloc<double2>(Gmax);
  double2* g = F->dalloc<double2>(Gmax);
  double2* g2 = F->dalloc<double2>(Gmax);
  // Device descriptors of the instances and their stencil buffers, uploaded
  // before any work is queued, so that the host goes from queuing the
  // stencil work straight to the factorisation.
  std::vector<InstDev> idev(count);
  for (int i = 0; i < count; ++i) {
    SppInstance& I = F->inst[i];
    InstDev& D = idev[i];
    // (the device side indexes stencil sets: boxes of the set width bs)
    D.d = I.d; D.n = I.n; D.b = I.bs; D.m = I.n / I.bs; D.N = I.N; D.Noff = I.Noff; D.q = F->q + I.Noff;
    D.nc = I.nc;
    D.npts = I.npts;
    const size_t ntypes = I.plan->types.size();
    for (size_t t = 0; t < ntypes; ++t) {
      const SetType& T = I.plan->types[t];
      StencilDev& S = I.sten[t];
      // (sizes in unknowns: nc per point, point-major; offsets per point)
      S.nS = T.nS * I.nc; S.nB = T.nB * I.nc; S.nG = T.nG * I.nc;
      S.off = F->pd->type_off[i * ntypes + t];
      S.T = F->dalloc<double2>((size_t)S.nS * S.nB);
      S.C = F->dalloc<double2>((size_t)S.nS * S.nG);
      S.Tt = F->dalloc<double2>((size_t)S.nS * S.nB);
      S.Ct = F->dalloc<double2>((size_t)S.nS * S.nG);
      // (complex64 fronts: the Q apply, whose output is complex64, reads T_S
      // rounded to complex64, half the bytes per entry)
      float2* tt32 = op->prec == SPP_C64_FRONTS ? F->dalloc<float2>((size_t)S.nS * S.nB) : nullptr;
      D.types[t] = TypeDev{S.nS, S.nB, S.nG, S.off, S.T, S.C, S.Tt, S.Ct, tt32};
    }
  }
  F->inst_dev = F->dalloc<InstDev>(count);
  SPP_HIP(hipMemcpyAsync(F->inst_dev, idev.data(), sizeof(InstDev) * count, hipMemcpyHostToDevice, st));
  MfDev& mf = F->mf;
  mf.perm = F->dalloc<int>(F->pd->perm_total);
  mf.ipiv = F->dalloc<int>(F->pd->perm_total);
  mf.prow = F->dalloc<int>(F->pd->perm_total);
  mf.fnorm = F->dalloc<unsigned>(P.fronts.size());
  mf.pstat = F->dalloc<unsigned>(2);
  for (int i = 0; i < count; ++i) {
    SppInstance& I = F->inst[i];
    const spp_problem& pb = pbs[i];
    // a1: shift and potential (eq. Dsq).
    // (per-problem block count: the same summation order as a batch of one)
    coeff_reduce(st, pb.kind, pb.coeff, I.npts, pb.omega, pb.ell, red, coeff_reduce_blocks(I.npts), red_out);
    double hred[2];
    SPP_HIP(hipMemcpyAsync(hred, red_out, sizeof(hred), hipMemcpyDeviceToHost, st));
    SPP_HIP(hipStreamSynchronize(st));
    if (hred[1] != 0)
      throw Error(SPP_EINVAL, "coeff has non-finite (or, for Helmholtz and Maxwell, non-positive) entries");
    const double mean_w = hred[0] / (double)I.npts;
    double s = (pb.kind == SPP_SCHRODINGER) ? pb.ell * pb.ell * pb.energy - mean_w : mean_w;
    int moves = 0;
    const bool vec = I.nc > 1;
    while (shift_gap(I.d, I.n, s, vec) < 1e-6) {
      if (moves == 10) throw Error(SPP_ESINGULAR_SHIFT, "L - s stays singular after 10 perturbations");
      s += 4.0 * M_PI * M_PI * 1e-3;
      ++moves;
    }
    I.s = s;
    I.moves = moves;
    // (q for every kind; the scalar symbol arrays are overwritten below for
    // a vector problem, whose q vector offset is 0: one problem per factor)
    coeff_finish(st, pb.kind, pb.coeff, I.npts, I.d, I.n, pb.omega, pb.ell, pb.energy, s, F->q + I.Noff,
                 F->sigma + I.Noff, sig_c, sig2_c);
    // a2: kernels of G and G G^H (vector problems: the nc^2 component pairs).
    if (vec) maxwell_symbols(st, I.d, I.n, s, sig_c, sig2_c);
    for (int ab = 0; ab < I.nc * I.nc; ++ab) {
      fft_inverse_all(st, sig_c + ab * I.npts, g + ab * I.npts, I.tw, I.d, I.n);
      fft_inverse_all(st, sig2_c + ab * I.npts, g2 + ab * I.npts, I.tw, I.d, I.n);
    }
    // a3-a4: stencils per set type.
    stencil_build(st, I.d, I.n, g, g2, I.sten, (int)I.plan->types.size(), swork, info + 1, I.nc);
    for (size_t t = 0; t < I.plan->types.size(); ++t)
      if (idev[i].types[t].Tt32 && (int64_t)I.sten[t].nS * I.sten[t].nB > 0)
        cast_vectors<float>(st, I.sten[t].Tt, const_cast<float2*>(idev[i].types[t].Tt32),
                            (int64_t)I.sten[t].nS * I.sten[t].nB, 0);
  }

  // a5-a6: assembly and factorisation on the shared plan.
  mf.fronts = F->pd->fronts;
  mf.blocks = F->pd->blocks;
  mf.pos = F->pd->pos;
  mf.idx = F->pd->idx;
  mf.map = F->pd->map;
  mf.gptr = F->pd->gptr;
  mf.gsrc = F->pd->gsrc;
  mf.info = info;
  mf.piv_tol = 1e3f * (float)std::numeric_limits<double>::epsilon();
  mf.piv_warn = 1e3f * (op->prec == SPP_C128 ? (float)std::numeric_limits<double>::epsilon()
                                              : std::numeric_limits<float>::epsilon());
  mf.inst = F->inst_dev;
  mf.ninst = count;
  mf.d = pbs[0].dim;
  mf.anchors_max = 0;
  mf.Ntot = F->Ntot;
  for (int t = 0; t < 8; ++t) mf.nB_max[t] = 0;
  for (const SppInstance& I : F->inst) {
    int64_t a = 1;
    for (int x = 0; x < I.d; ++x) a *= I.n / I.bs;
    mf.anchors_max = std::max(mf.anchors_max, a);
    for (size_t t = 0; t < I.plan->types.size(); ++t)
      mf.nB_max[t] = std::max(mf.nB_max[t], I.plan->types[t].nB * I.nc);   // (unknowns)
  }
  for (const Level& L : P.levels) {
    F->level_begin.push_back(L.begin);
    F->level_maxF.push_back(L.maxF);
    F->level_maxK.push_back(L.maxK);
    F->level_maxP.push_back(L.maxP);
  }
  F->level_begin.push_back(static_cast<int>(P.fronts.size()));
  bool any_blocked = false;
  for (int form : F->level_form) any_blocked = any_blocked || form == kFormBlocked;
  const bool partial_pivoting = (F->opt.flags & SPP_F_PARTIAL_PIVOTING) != 0;

  if (streamed) F->fstore = F->big_alloc((size_t)P.fstore_elems * F->csize);
  F->fac = streamed ? F->fstore : F->arena;
  void* xwork = F->dalloc<char>((size_t)F->xwork_elems * F->csize);
  void* tbuf = F->dalloc<char>((size_t)(F->xwork_elems / 2) * F->csize);
  void* dinv = F->dalloc<char>((size_t)2 * 32 * 32 * F->pd->dblk_total * F->csize);
  int64_t tp_ints = 1;
  for (size_t l = 0; l < P.levels.size(); ++l)
    if (F->level_form[l] == kFormBlocked)
      tp_ints = std::max(tp_ints, mf_tournament_ints(P.levels[l].end - P.levels[l].begin, P.levels[l].maxP));
  int* tpbuf = F->dalloc<int>(tp_ints);
  if (any_blocked) {
    F->dkeep = dinv;
    mf.dkeep = dinv;
  }
  // The coefficient and Green buffers go back to the cache once the stream
  // has drained: before a tuning pass (whose buffers may reuse them), else
  // after the factorisation, so the host queues it behind the stencils.
  bool setup_bufs_freed = false;
  auto free_setup_bufs = [&] {
    if (setup_bufs_freed) return;
    // (only the stencil work on st used them: a device-wide drain here would
    // also wait for the last level's inverses on the side stream)
    SPP_HIP(hipStreamSynchronize(st));
    for (void* p : {(void*)red, (void*)sig_c, (void*)sig2_c, (void*)g, (void*)g2}) F->dfree(p, true);
    setup_bufs_freed = true;
  };
  const int nl = static_cast<int>(P.levels.size());
  // Assembly and factorisation of every level with the given solve forms and
  // step schedules; fev (optional) gets two events per level around it.
  // defer_inverses: the final factorisation leaves its last inverses running
  // on the side stream (see factor_ready).
  bool defer_inverses = false;
  auto factor_all = [&](const std::vector<int>& forms, const std::vector<int>& vars, hipEvent_t* fev) {
    // (breakdown front, small pivots, fatal flag, pivot statistics and the
    // fronts' largest entries, in one launch)
    mf_reset_status(st, mf, static_cast<int>(P.fronts.size()));
    if (arena_zero_ahead) {
      SPP_HIP(hipStreamWaitEvent(st, F->zero_event, 0));
      arena_zero_ahead = false;
    } else if (!streamed) {
      SPP_HIP(hipMemsetAsync(F->arena, 0, (size_t)P.arena_elems * F->csize, st));
    }
    // Resident storage, untimed: each level's inverses run on the side
    // stream beside the next level's LU (joined below).
    const bool overlap = !fev && !streamed && !F->timer && !partial_pivoting;
    hipStream_t inv_st = nullptr;
    if (overlap) {
      inv_st = side_stream();
      for (hipEvent_t& e : F->inv_event)
        if (!e) SPP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    for (int l = 0; l < nl; ++l) {
      const Level& L = P.levels[l];
      const int* hF = F->pd->level_F[l].data();
      const int* hP = F->pd->level_p[l].data();
      if (fev) SPP_HIP(hipEventRecord(fev[2 * l], st));
      // Streamed storage: this level's arena range held fronts two levels
      // down, whose Schur complements the level below has already added.
      if (streamed)
        SPP_HIP(hipMemsetAsync(static_cast<char*>(F->arena) + (size_t)L.arena_lo * F->csize, 0,
                               (size_t)(L.arena_hi - L.arena_lo) * F->csize, st));
      // Large pivot blocks choose their pivots over all their fully-summed
      // rows (by tournament): pivots chosen inside 32-row blocks let the
      // multipliers below the block, and with them the growth of the Schur
      // updates, grow with the front.
      const int piv = partial_pivoting ? kPivotPartial
                      : forms[l] == kFormBlocked ? kPivotTournament : kPivotBlockLocal;
      // (the side stream's work for the earlier levels ends here)
      if (overlap && l == nl - 1) SPP_HIP(hipEventRecord(F->inv_event[2], inv_st));
      if (F->opt.prec == SPP_C128)
        mf_factor_level<double>(st, mf, F->arena, xwork, tbuf, dinv, tpbuf, L.begin, L.end, L.maxF, L.maxP,
                                L.blk_begin, L.blk_end, L.max_children, forms[l], piv, vars[l], hF, hP, inv_st,
                                F->inv_event[0]);
      else
        mf_factor_level<float>(st, mf, F->arena, xwork, tbuf, dinv, tpbuf, L.begin, L.end, L.maxF, L.maxP,
                               L.blk_begin, L.blk_end, L.max_children, forms[l], piv, vars[l], hF, hP, inv_st,
                               F->inv_event[0]);
      if (streamed) {
        if (F->opt.prec == SPP_C128)
          mf_store_factors<double>(st, mf, F->arena, F->fstore, L.begin, L.end - L.begin, L.maxF);
        else
          mf_store_factors<float>(st, mf, F->arena, F->fstore, L.begin, L.end - L.begin, L.maxF);
      }
      if (fev) SPP_HIP(hipEventRecord(fev[2 * l + 1], st));
    }
    if (overlap) {   // (the factor is complete once the last inverses are)
      SPP_HIP(hipEventRecord(F->inv_event[1], inv_st));
      if (defer_inverses) F->inv_pending = true;
      else SPP_HIP(hipStreamWaitEvent(st, F->inv_event[1], 0));
    }
  };
  if (tune_fac) {
    free_setup_bufs();
    tune_factorisation(F.get(), factor_all, st);
  }
  // (the factorisation's own time between two events: the stencils may
  // still be running when the host has queued it)
  struct FactorEvents {
    hipEvent_t e[2] = {nullptr, nullptr};
    ~FactorEvents() {
      for (hipEvent_t x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } fe;
  for (hipEvent_t& x : fe.e) SPP_HIP(hipEventCreate(&x));
  SPP_HIP(hipEventRecord(fe.e[0], st));
  defer_inverses = true;
  factor_all(F->level_form, F->level_var, nullptr);
  SPP_HIP(hipEventRecord(fe.e[1], st));
  // The buffers of a one-right-hand-side solve are set up while the GPU
  // factors (host work that would otherwise stall the start of the first
  // solve), when they are small against the free memory.
  {
    const int maxit = F->opt.max_iter;
    const int cycle_len = F->opt.restart > 0 ? std::min(F->opt.restart, maxit) : maxit;
    const size_t vec = (size_t)F->Ntot * sizeof(double2);
    const size_t est = vec * (2 * (size_t)cycle_len + 10) + ((size_t)1 << 20) * F->csize +
                       (size_t)2 * P.vec_elems * F->csize;
    if (est <= ((size_t)4 << 30) && est <= spare_bytes / 8) ensure_solve_buffers(F.get(), 1, cycle_len);
  }
  int hinfo[16];
  unsigned hpstat[2];
  SPP_HIP(hipMemcpyAsync(hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost, st));
  SPP_HIP(hipMemcpyAsync(hpstat, mf.pstat, sizeof(hpstat), hipMemcpyDeviceToHost, st));
  SPP_HIP(hipStreamSynchronize(st));
  float factor_ms = 0.f;
  SPP_HIP(hipEventElapsedTime(&factor_ms, fe.e[0], fe.e[1]));
  free_setup_bufs();
  if (F->inv_pending) {   // (still in use by the last inverses)
    F->inv_buffers = {xwork, tbuf};
    if (!any_blocked) F->inv_buffers.push_back(dinv);
  } else {   // (the inverses, if any, were joined to st, which has drained)
    F->dfree(xwork, true);
    F->dfree(tbuf, true);
    if (!any_blocked) F->dfree(dinv, true);
  }
  F->dfree(tpbuf, true);   // (used on st only)
  F->dfree(swork, true);
  if (streamed) {   // the substitution reads the factor store only
    F->big_free(F->arena);
    F->arena = nullptr;
  }
  for (int t = 0; t < 8; ++t)
    if (hinfo[1 + t]) throw Error(SPP_EBREAKDOWN, "singular Gram matrix in the stencil least-squares problem");
  F->stats.breakdown_front = hinfo[0] ? hinfo[0] - 1 : -1;
  F->stats.s = F->inst[0].s;
  F->stats.shift_moves = F->inst[0].moves;
  F->stats.n_fronts = static_cast<int>(P.fronts.size());
  F->stats.n_levels = static_cast<int>(P.levels.size());
  F->stats.max_front = P.max_front;
  F->stats.factor_entries = P.factor_entries;
  F->stats.factor_bytes = P.factor_entries * (int64_t)F->csize;
  F->stats.factor_flops = P.factor_flops;
  F->stats.t_factor_ms = factor_ms;
  F->stats.t_setup_ms = now_ms() - t0;
  F->stats.last_iters = 0;
  F->stats.last_cycles = 0;
  F->stats.storage = P.storage;
  {
    float g, mp;
    std::memcpy(&g, &hpstat[0], sizeof(float));
    std::memcpy(&mp, &hpstat[1], sizeof(float));
    F->stats.pivot_growth = g;
    F->stats.min_pivot = mp;
    F->stats.small_pivots = hinfo[9];
  }
  if (hinfo[0]) {
    g_last_error = std::string(hinfo[10] ? "pivot below 1e3 FP64 eps times the largest front entry"
                                         : "zero or non-finite pivot") +
                   " in front " + std::to_string(hinfo[0] - 1);
    *out = F.release();
    return SPP_EBREAKDOWN;
  }
  *out = F.release();
  return SPP_OK;
}

int do_solve(spp_factor* F, const void* fv, int nrhs, void* uv, int32_t* iters, double* relres, hipStream_t st) {
  if (!F || !fv || !uv || !iters || !relres || nrhs < 1) throw Error(SPP_EINVAL, "null argument or nrhs < 1");
  const double t0 = now_ms();
  F->last_stream = st;
  TimerScope timer_scope(F);
  const int maxit = F->opt.max_iter;
  // Krylov vectors per cycle: the restart length, or the whole iteration
  // budget without restarts.
  const int cycle_len = F->opt.restart > 0 ? std::min(F->opt.restart, maxit) : maxit;
  ensure_solve_buffers(F, nrhs, cycle_len);
  if ((F->opt.flags & SPP_F_AUTOTUNE) && F->tuned_nrhs != nrhs) do_autotune(F, nrhs, st);
  const int64_t vstride = (int64_t)nrhs * F->Ntot;   // one Krylov vector of the whole batch
  const int ld = F->cap_iter + 1;                     // Hessenberg column stride, per-column vector stride
  const int hrhs = ld * F->cap_iter;                  // Hessenberg stride between columns
  const int cols = total_cols(F, nrhs);               // (problem, right-hand side) pairs
  const double2* f = static_cast<const double2*>(fv);
  double2* u = static_cast<double2*>(uv);
  const bool precond = !(F->opt.flags & SPP_F_UNPRECONDITIONED);

  // a7: g = G f; beta0 = ||g|| per column (the reference of every stopping test).
  apply_green(F, f, F->g0, nrhs, st);
  for (const SppGroup& g : F->groups) {
    const int c0 = g.inst0 * nrhs, nc = g.ninst * nrhs;
    kr_norms(st, F->g0 + g.Noff * nrhs, nc, g.N, F->rpart, F->norms + c0);
  }
  const bool learned = F->cnn != nullptr && precond;
  const bool use_graph = (F->opt.flags & SPP_F_GRAPHS) && !F->timer && !learned;
  if (use_graph) {   // (no event waits inside a capture: the factor is made complete first)
    factor_ready(F, st);
    factor_settled(F);
  }
  // The first cycle starts from r = g: its first basis vector, and in eager
  // iterations the preconditioner head on it, go out before the host waits
  // for beta0.
  for (const SppGroup& g : F->groups) {
    const int c0 = g.inst0 * nrhs, nc = g.ninst * nrhs;
    const int64_t o = g.Noff * nrhs;
    kr_scale_init(st, F->g0 + o, F->V + o, F->norms + c0, nc, g.N, F->gv + (int64_t)c0 * ld, ld);
  }
  const bool early_head = precond && !learned && !use_graph;
  if (early_head) precond_head(F, F->V, nrhs, st);
  std::vector<double> beta0(cols);
  SPP_HIP(hipMemcpyAsync(beta0.data(), F->norms, sizeof(double) * cols, hipMemcpyDeviceToHost, st));
  SPP_HIP(hipStreamSynchronize(st));
  std::vector<int> k(cols, 0), total(cols, 0);
  std::vector<bool> conv(cols, false), fin(cols, false);
  for (int c = 0; c < cols; ++c) fin[c] = !(beta0[c] > 0);
  std::vector<double> beta(cols), rn(cols, 0.0);
  int done = 0;
  // One Arnoldi step with z_j already in Z: w = A z_j, CGS2, Givens; returns
  // the residual estimates in F->h_resid.
  // head_next: after the step, run the next iteration's preconditioner head
  // on v_{j+1} while the host waits for the residual estimates.
  bool head_ready = false;
  auto arnoldi_step = [&](int j, bool head_next = false) {
    double2* zj = F->Z + (int64_t)j * vstride;
    // a8: w = (I + G q) z_j
    apply_operator(F, zj, F->wk, nrhs, st);
    // CGS2 against v_0 .. v_j; H(:, j) per column.
    for (const SppGroup& g : F->groups) {
      const int c0 = g.inst0 * nrhs, nc = g.ninst * nrhs;
      const int64_t o = g.Noff * nrhs;
      double2* hcol = F->H + (int64_t)c0 * hrhs + (int64_t)j * ld;
      double2* h2 = F->h2 + (int64_t)c0 * ld;
      kr_dots(st, F->V + o, vstride, j + 1, F->wk + o, nc, g.N, F->dpart, hcol, hrhs, 0, nullptr, 0);
      // (the first update, the second projection, the second update and the
      // norm's partial sums in two sweeps over V)
      kr_cgs2_second(st, F->V + o, vstride, j + 1, F->wk + o, nc, g.N, hcol, hrhs, F->dpart, h2, ld, hcol, hrhs,
                     F->rpart);
      // a10: the Givens update of the least-squares problem goes with the
      // normalisation of v_{j+1} (one launch per group).
      KrGivens gv;
      gv.H = F->H; gv.hcol = ld; gv.hrhs = hrhs; gv.cs = F->cs; gv.sn = F->sn; gv.g = F->gv;
      gv.j = j; gv.ldg = ld; gv.resid = F->resid; gv.resid_host = F->h_resid_dev; gv.c0 = c0;
      kr_normalize(st, F->wk + o, F->V + (int64_t)(j + 1) * vstride + o, nc, g.N, F->rpart, hcol + (j + 1), hrhs, gv);
    }
    if (head_next) {
      SPP_HIP(hipEventRecord(F->resid_event, st));
      precond_head(F, F->V + (int64_t)(j + 1) * vstride, nrhs, st);
      head_ready = true;
      SPP_HIP(hipEventSynchronize(F->resid_event));
    } else {
      SPP_HIP(hipStreamSynchronize(st));
    }
  };
  // The same step for graph replays: every launch reads j from F->dj, the
  // vectors go through fixed buffers, and the residual estimates are copied
  // to pinned memory inside the graph.
  auto graph_body = [&](hipStream_t s) {
    const int* dj = F->dj;
    kr_copy_j(s, F->V, vstride, F->vfix, 0, vstride, dj);
    if (precond) apply_precond(F, F->vfix, F->zfix, nrhs, s, false);
    else kr_copy_j(s, F->V, vstride, F->zfix, 0, vstride, dj);
    kr_copy_j(s, F->zfix, 0, F->Z, vstride, vstride, dj);
    apply_operator(F, F->zfix, F->wk, nrhs, s);
    for (const SppGroup& g : F->groups) {
      const int c0 = g.inst0 * nrhs, nc = g.ninst * nrhs;
      const int64_t o = g.Noff * nrhs;
      double2* hbase = F->H + (int64_t)c0 * hrhs;
      double2* h2 = F->h2 + (int64_t)c0 * ld;
      kr_dots(s, F->V + o, vstride, ld, F->wk + o, nc, g.N, F->dpart, hbase, hrhs, 0, nullptr, 0, dj, ld, 0);
      kr_update(s, F->V + o, vstride, ld, F->wk + o, nc, g.N, hbase, hrhs, dj, ld);
      kr_dots(s, F->V + o, vstride, ld, F->wk + o, nc, g.N, F->dpart, h2, ld, 0, hbase, hrhs, dj, 0, ld);
      kr_update(s, F->V + o, vstride, ld, F->wk + o, nc, g.N, h2, ld, dj, 0);
      KrGivens gv;
      gv.H = F->H; gv.hcol = ld; gv.hrhs = hrhs; gv.cs = F->cs; gv.sn = F->sn; gv.g = F->gv;
      gv.j = 0; gv.ldg = ld; gv.resid = F->resid; gv.c0 = c0;
      kr_norm_scale(s, F->wk + o, F->V + vstride + o, nc, g.N, F->rpart, hbase + 1, hrhs, dj, vstride, ld + 1, gv);
    }
    SPP_HIP(hipMemcpyAsync(F->h_resid, F->resid, sizeof(double) * cols, hipMemcpyDeviceToHost, s));
    kr_set_counter(s, F->dj, 1, true);
  };
  if (use_graph && (!F->graph_exec || F->graph_nrhs != nrhs || F->graph_precond != precond)) {
    F->drop_graph();
    if (!F->gstream) SPP_HIP(hipStreamCreateWithFlags(&F->gstream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    SPP_HIP(hipStreamBeginCapture(F->gstream, hipStreamCaptureModeThreadLocal));
    try {
      graph_body(F->gstream);
    } catch (...) {
      (void)hipStreamEndCapture(F->gstream, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      throw;
    }
    SPP_HIP(hipStreamEndCapture(F->gstream, &graph));
    const hipError_t ie = hipGraphInstantiate(&F->graph_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
      F->graph_exec = nullptr;
      throw_hip(ie, "hipGraphInstantiate", __FILE__, __LINE__);
    }
    F->graph_nrhs = nrhs;
    F->graph_precond = precond;
  }
  F->cnn_accepted = F->cnn_rejected = 0;
  int reject_run = 0;
  const double sN = std::sqrt((double)F->Ntot);
  const double tol = F->opt.tol;
  // a10-a11: cycles of FGMRES.  Each cycle starts from the current residual
  // r (g itself in the first cycle, x0 = 0), runs until every column's
  // residual estimate is <= tol ||g|| or the cycle length or iteration budget
  // is spent, adds its correction to u, and recomputes the true residual
  // ||g - (I + G q) u||.  A column whose true residual is still above
  // tol ||g|| (restarts, or an estimate that drifted from the truth) goes on
  // with another cycle while iterations remain.
  const double2* r = F->g0;
  int used = 0, j = 0, cycles = 0;
  bool all_ok = false;
  for (;;) {
    for (const SppGroup& g : F->groups) {
      if (cycles == 0) break;   // (queued before the wait for beta0)
      const int c0 = g.inst0 * nrhs, nc = g.ninst * nrhs;
      const int64_t o = g.Noff * nrhs;
      kr_norms(st, r + o, nc, g.N, F->rpart, F->norms + c0);
      kr_scale_init(st, r + o, F->V + o, F->norms + c0, nc, g.N, F->gv + (int64_t)c0 * ld, ld);
    }
    if (cycles == 0) {
      beta = beta0;
    } else {
      SPP_HIP(hipMemcpyAsync(beta.data(), F->norms, sizeof(double) * cols, hipMemcpyDeviceToHost, st));
      SPP_HIP(hipStreamSynchronize(st));
    }
    done = 0;
    for (int c = 0; c < cols; ++c) {
      k[c] = 0;
      conv[c] = fin[c] || !(beta[c] > tol * beta0[c]);
      if (conv[c]) ++done;
    }
    if (use_graph) kr_set_counter(st, F->dj, 0, false);
    std::vector<double> prev(beta);
    head_ready = cycles == 0 && early_head;
    const int jmax = std::min(cycle_len, maxit - used);
    for (j = 0; j < jmax && done < cols; ++j) {
      double2* vj = F->V + (int64_t)j * vstride;
      double2* zj = F->Z + (int64_t)j * vstride;
      bool have = false;
      if (use_graph) {
        SPP_HIP(hipGraphLaunch(F->graph_exec, st));
        SPP_HIP(hipStreamSynchronize(st));
        have = true;
      } else if (learned && reject_run < 3) {
        // Learned stage: z_j = net(v_j), kept only if every column's residual
        // estimate drops to rho times its previous value.
        SPP_HIP(hipMemcpyAsync(F->gsave, F->gv, sizeof(double2) * ld * cols, hipMemcpyDeviceToDevice, st));
        cnn_apply(F->cnn, vj, zj, cols, sN, 1.0 / sN, st);
        arnoldi_step(j);
        bool ok = true;
        for (int c = 0; c < cols; ++c)
          if (!conv[c] && !(F->h_resid[c] <= F->cnn_rho * prev[c])) ok = false;
        if (ok) {
          ++F->cnn_accepted;
          reject_run = 0;
          have = true;
        } else {
          ++F->cnn_rejected;
          ++reject_run;
          SPP_HIP(hipMemcpyAsync(F->gv, F->gsave, sizeof(double2) * ld * cols, hipMemcpyDeviceToDevice, st));
        }
      }
      if (!have) {
        // a9: z_j = M v_j (its head may already have run behind the previous
        // step's residual check)
        if (precond) {
          if (!head_ready) precond_head(F, vj, nrhs, st);
          precond_tail(F, zj, nrhs, st, true);
        } else {
          SPP_HIP(hipMemcpyAsync(zj, vj, sizeof(double2) * vstride, hipMemcpyDeviceToDevice, st));
        }
        head_ready = false;
        arnoldi_step(j, precond && !learned && j + 1 < jmax);
      }
      for (int c = 0; c < cols; ++c) prev[c] = F->h_resid[c];
      for (int c = 0; c < cols; ++c) {
        if (conv[c]) continue;
        if (!(F->h_resid[c] > tol * beta0[c])) {
          conv[c] = true;
          k[c] = j + 1;
          ++done;
        }
      }
    }
    for (int c = 0; c < cols; ++c)
      if (!conv[c]) k[c] = j;
      else if (fin[c]) k[c] = 0;
    // a11: u (+)= Z y, then the true residual ||g - (I + G q) u|| / ||g||.
    SPP_HIP(hipMemcpyAsync(F->kvec, k.data(), sizeof(int) * cols, hipMemcpyHostToDevice, st));
    kr_backsolve(st, F->H, ld, hrhs, F->gv, ld, F->y, 0, cols, F->kvec);
    const int kmax_all = std::max(1, *std::max_element(k.begin(), k.end()));
    for (const SppGroup& g : F->groups) {
      const int c0 = g.inst0 * nrhs, nc = g.ninst * nrhs;
      const int64_t o = g.Noff * nrhs;
      kr_combine(st, F->Z + o, vstride, kmax_all, F->y + (int64_t)c0 * ld, ld, u + o, nc, g.N, F->kvec + c0,
                 cycles > 0);
    }
    apply_operator(F, u, F->wk, nrhs, st);
    kr_sub(st, F->g0, F->wk, F->wk, vstride);
    for (const SppGroup& g : F->groups) {
      const int c0 = g.inst0 * nrhs, nc = g.ninst * nrhs;
      kr_norms(st, F->wk + g.Noff * nrhs, nc, g.N, F->rpart, F->norms + c0);
    }
    SPP_HIP(hipMemcpyAsync(rn.data(), F->norms, sizeof(double) * cols, hipMemcpyDeviceToHost, st));
    SPP_HIP(hipStreamSynchronize(st));
    used += j;
    ++cycles;
    all_ok = true;
    for (int c = 0; c < cols; ++c) {
      total[c] += k[c];
      if (!(beta0[c] > 0) || rn[c] <= tol * beta0[c]) fin[c] = true;
      else all_ok = false;
    }
    if (all_ok || used >= maxit || j == 0) break;
    r = F->wk;   // the next cycle starts from the true residual
  }
  int kmax = 0;
  for (int c = 0; c < cols; ++c) {
    iters[c] = total[c];
    relres[c] = beta0[c] > 0 ? rn[c] / beta0[c] : 0.0;
    kmax = std::max(kmax, total[c]);
  }
  F->stats.last_iters = kmax;
  F->stats.last_cycles = cycles;
  F->stats.t_solve_ms = now_ms() - t0;
  F->last_iters_all = j;
  F->last_nrhs = nrhs;
  factor_settled(F);   // (the last inverses are done by now: their buffers go back)
  if (!all_ok) {
    g_last_error = "GMRES reached max_iter before the true residual met the tolerance";
    return SPP_NOT_CONVERGED;
  }
  return SPP_OK;
}

// Per-problem right-hand sides: packed into the batch layout with the
// largest count per problem (missing columns are zero and converge at once),
// solved in lock step, unpacked.
int do_solve_batch(spp_factor* F, const void* const* f, const int32_t* nrhs, void* const* u, int32_t* iters,
                   double* relres, hipStream_t st) {
  if (!F || !f || !nrhs || !u || !iters || !relres) throw Error(SPP_EINVAL, "null argument");
  const int np = static_cast<int>(F->inst.size());
  int R = 0;
  for (int i = 0; i < np; ++i) {
    if (nrhs[i] < 0 || nrhs[i] > 64) throw Error(SPP_EINVAL, "nrhs[i] must be in [0, 64]");
    if (nrhs[i] > 0 && (!f[i] || !u[i])) throw Error(SPP_EINVAL, "null f[i] or u[i] with nrhs[i] > 0");
    R = std::max(R, (int)nrhs[i]);
  }
  if (R == 0) return SPP_OK;
  const int64_t need = (int64_t)R * F->Ntot;
  if (need > F->pack_cap) {
    F->dfree(F->pack_f);
    F->dfree(F->pack_u);
    F->pack_f = F->dalloc<double2>(need);
    F->pack_u = F->dalloc<double2>(need);
    F->pack_cap = need;
  }
  SPP_HIP(hipMemsetAsync(F->pack_f, 0, sizeof(double2) * need, st));
  for (int i = 0; i < np; ++i)
    if (nrhs[i] > 0)
      SPP_HIP(hipMemcpyAsync(F->pack_f + F->inst[i].Noff * R, f[i], sizeof(double2) * nrhs[i] * F->inst[i].N,
                             hipMemcpyDeviceToDevice, st));
  std::vector<int32_t> it((size_t)np * R);
  std::vector<double> rr((size_t)np * R);
  const int code = do_solve(F, F->pack_f, R, F->pack_u, it.data(), rr.data(), st);
  int o = 0;
  for (int i = 0; i < np; ++i) {
    if (nrhs[i] > 0)
      SPP_HIP(hipMemcpyAsync(u[i], F->pack_u + F->inst[i].Noff * R, sizeof(double2) * nrhs[i] * F->inst[i].N,
                             hipMemcpyDeviceToDevice, st));
    for (int c = 0; c < nrhs[i]; ++c, ++o) {
      iters[o] = it[(size_t)i * R + c];
      relres[o] = rr[(size_t)i * R + c];
    }
  }
  return code;
}

}  // namespace

extern "C" {

int spp_setup(const spp_problem* problem, const spp_options* options, spp_stream_t stream, spp_factor** out) {
  return guarded([&] { return do_setup(problem, 1, options, reinterpret_cast<hipStream_t>(stream), out); });
}

int spp_setup_batch(const spp_problem* problems, int32_t count, const spp_options* options, spp_stream_t stream,
                    spp_factor** out) {
  return guarded([&] { return do_setup(problems, count, options, reinterpret_cast<hipStream_t>(stream), out); });
}

int spp_solve(spp_factor* factor, const void* f, int32_t nrhs, void* u, int32_t* iters, double* relres,
              spp_stream_t stream) {
  return guarded([&] { return do_solve(factor, f, nrhs, u, iters, relres, reinterpret_cast<hipStream_t>(stream)); });
}

int spp_solve_batch(spp_factor* factor, const void* const* f, const int32_t* nrhs, void* const* u, int32_t* iters,
                    double* relres, spp_stream_t stream) {
  return guarded(
      [&] { return do_solve_batch(factor, f, nrhs, u, iters, relres, reinterpret_cast<hipStream_t>(stream)); });
}

int spp_autotune(spp_factor* factor, int32_t nrhs, spp_stream_t stream) {
  return guarded([&] {
    if (!factor || nrhs < 1) throw Error(SPP_EINVAL, "null factor or nrhs < 1");
    do_autotune(factor, nrhs, reinterpret_cast<hipStream_t>(stream));
    return SPP_OK;
  });
}

int spp_tune_set(const char* key, int32_t value) {
  return guarded([&] {
    if (!key || !*key) throw Error(SPP_EINVAL, "null or empty tuning key");
    tune_set(key, value);
    return SPP_OK;
  });
}

int spp_tune_get(const char* key, int32_t* value) {
  return guarded([&] {
    if (!key || !value) throw Error(SPP_EINVAL, "null tuning key or value");
    if (!tune_has(key)) throw Error(SPP_EINVAL, std::string("no tuning entry ") + key);
    *value = tune_get(key, -1);
    return SPP_OK;
  });
}

int spp_apply_operator(spp_factor* factor, const void* z, void* w, int32_t nrhs, spp_stream_t stream) {
  return guarded([&] {
    if (!factor || !z || !w || nrhs < 1) throw Error(SPP_EINVAL, "null argument or nrhs < 1");
    ensure_solve_buffers(factor, nrhs, factor->opt.max_iter);
    TimerScope timer_scope(factor);
    apply_operator(factor, static_cast<const double2*>(z), static_cast<double2*>(w), nrhs,
                   reinterpret_cast<hipStream_t>(stream));
    return SPP_OK;
  });
}

int spp_apply_operator_noalloc(spp_factor* factor, const void* z, void* w, int32_t nrhs, spp_stream_t stream) {
  return guarded([&] {
    if (!factor || !z || !w || nrhs < 1) throw Error(SPP_EINVAL, "null argument or nrhs < 1");
    const size_t need = sizeof(double2) * (size_t)nrhs * (size_t)factor->Ntot;
    if (need > kNoAllocScratchBytes)
      throw Error(SPP_EINVAL, "spp_apply_operator_noalloc: nrhs * N * 16 = " + std::to_string(need) +
                                  " bytes exceeds the scratch of " + std::to_string(kNoAllocScratchBytes) + " bytes");
    // The FFT intermediate goes to the library's static device scratch; no
    // buffer of the factor is grown and no kernel timer is recorded.
    double2* tmp = static_cast<double2*>(noalloc_scratch());
    KernelTimer* saved = g_timer;
    g_timer = nullptr;
    const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const double2* zz = static_cast<const double2*>(z);
    double2* ww = static_cast<double2*>(w);
    apply_operator_to(factor, zz, ww, tmp, nrhs, st);
    g_timer = saved;
    return SPP_OK;
  });
}

int spp_apply_green(spp_factor* factor, const void* f, void* g, int32_t nrhs, spp_stream_t stream) {
  return guarded([&] {
    if (!factor || !f || !g || nrhs < 1) throw Error(SPP_EINVAL, "null argument or nrhs < 1");
    ensure_solve_buffers(factor, nrhs, factor->opt.max_iter);
    TimerScope timer_scope(factor);
    apply_green(factor, static_cast<const double2*>(f), static_cast<double2*>(g), nrhs,
                reinterpret_cast<hipStream_t>(stream));
    return SPP_OK;
  });
}

int spp_apply_q(spp_factor* factor, const void* r, void* y, int32_t nrhs, spp_stream_t stream) {
  return guarded([&] {
    if (!factor || !r || !y || nrhs < 1) throw Error(SPP_EINVAL, "null argument or nrhs < 1");
    if (r == y) throw Error(SPP_EINVAL, "spp_apply_q: r and y must not alias");
    TimerScope timer_scope(factor);
    q_apply(reinterpret_cast<hipStream_t>(stream), factor->mf, static_cast<const double2*>(r),
            static_cast<double2*>(y), nrhs);
    return SPP_OK;
  });
}

int spp_apply_precond(spp_factor* factor, const void* r, void* z, int32_t nrhs, spp_stream_t stream) {
  return guarded([&] {
    if (!factor || !r || !z || nrhs < 1) throw Error(SPP_EINVAL, "null argument or nrhs < 1");
    ensure_solve_buffers(factor, nrhs, factor->opt.max_iter);
    TimerScope timer_scope(factor);
    apply_precond(factor, static_cast<const double2*>(r), static_cast<double2*>(z), nrhs,
                  reinterpret_cast<hipStream_t>(stream));
    return SPP_OK;
  });
}

int spp_get_coefficients(const spp_factor* factor, double* s, double* q) {
  return guarded([&] {
    if (!factor) throw Error(SPP_EINVAL, "null factor");
    if (s) *s = factor->inst[0].s;
    int64_t pts = 0;   // q lives per grid point (every field component shares it)
    for (const SppInstance& I : factor->inst) pts += I.npts;
    if (q) SPP_HIP(hipMemcpy(q, factor->q, sizeof(double) * pts, hipMemcpyDeviceToDevice));
    return SPP_OK;
  });
}

int spp_get_shift(const spp_factor* factor, int32_t problem, double* s, int32_t* moves) {
  return guarded([&] {
    if (!factor) throw Error(SPP_EINVAL, "null factor");
    if (problem < 0 || problem >= (int)factor->inst.size()) throw Error(SPP_EINVAL, "problem index out of range");
    if (s) *s = factor->inst[problem].s;
    if (moves) *moves = factor->inst[problem].moves;
    return SPP_OK;
  });
}

int spp_get_stencil(const spp_factor* factor, int32_t type, int32_t* nS, int32_t* nB, int32_t* offsets, void* T,
                    void* C) {
  return guarded([&] {
    if (!factor) throw Error(SPP_EINVAL, "null factor");
    const SppInstance& I = factor->inst[0];
    if (type < 0 || type >= (1 << I.d)) throw Error(SPP_EINVAL, "set type out of range");
    const SetType& ST = I.plan->types[type];
    const StencilDev& S = I.sten[type];
    if (nS) *nS = S.nS;
    if (nB) *nB = S.nB;
    if (offsets) std::memcpy(offsets, ST.off.data(), ST.off.size() * sizeof(int));
    if (T) SPP_HIP(hipMemcpy(T, S.T, sizeof(double2) * S.nS * S.nB, hipMemcpyDeviceToHost));
    if (C) SPP_HIP(hipMemcpy(C, S.C, sizeof(double2) * S.nS * S.nG, hipMemcpyDeviceToHost));
    return SPP_OK;
  });
}

int spp_attach_cnn(spp_factor* factor, spp_cnn* net, double rho) {
  return guarded([&] {
    if (net && !(rho > 0 && rho < 1)) throw Error(SPP_EINVAL, "rho must be in (0, 1)");
    if (!factor) throw Error(SPP_EINVAL, "null factor");
    if (!net) {
      factor->cnn = nullptr;
      return SPP_OK;
    }
    if (factor->inst.size() != 1 || factor->inst[0].d != 2 || factor->inst[0].n != cnn_grid(net))
      throw Error(SPP_EINVAL, "the learned stage needs a single 2D problem on the network's grid");
    if (factor->inst[0].nc != 1) throw Error(SPP_ENOTIMPL, "the learned stage takes scalar fields only");
    factor->cnn = net;
    factor->cnn_rho = rho;
    return SPP_OK;
  });
}

int spp_learned_stats(const spp_factor* factor, int32_t* accepted, int32_t* rejected) {
  return guarded([&] {
    if (!factor) throw Error(SPP_EINVAL, "null factor");
    if (accepted) *accepted = factor->cnn_accepted;
    if (rejected) *rejected = factor->cnn_rejected;
    return SPP_OK;
  });
}

int spp_get_krylov(const spp_factor* factor, int32_t j, void* v, void* z) {
  return guarded([&] {
    if (!factor) throw Error(SPP_EINVAL, "null factor");
    if (j < 0 || j >= factor->last_iters_all) throw Error(SPP_EINVAL, "j must be below the last solve's iterations");
    const size_t bytes = sizeof(double2) * (size_t)factor->last_nrhs * factor->Ntot;
    const int64_t vstride = (int64_t)factor->last_nrhs * factor->Ntot;
    if (v) SPP_HIP(hipMemcpy(v, factor->V + (int64_t)j * vstride, bytes, hipMemcpyDeviceToDevice));
    if (z) SPP_HIP(hipMemcpy(z, factor->Z + (int64_t)j * vstride, bytes, hipMemcpyDeviceToDevice));
    return SPP_OK;
  });
}

int spp_stats(const spp_factor* factor, spp_stats_t* out) {
  return guarded([&] {
    if (!factor || !out) throw Error(SPP_EINVAL, "null argument");
    *out = factor->stats;
    return SPP_OK;
  });
}

int spp_kernel_timing(const spp_factor* factor, int32_t kclass, double* total_ms, int64_t* launches, double* bytes,
                      double* flops) {
  return guarded([&] {
    if (!factor) throw Error(SPP_EINVAL, "null factor");
    if (kclass < 0 || kclass >= KC_COUNT) throw Error(SPP_EINVAL, "kernel class out of range");
    double ms = 0;
    int64_t n = 0;
    double by = 0, fl = 0;
    if (factor->timer) {
      KernelTimer& T = *factor->timer;
      for (auto& pr : T.ev[kclass]) {
        SPP_HIP(hipEventSynchronize(pr.second));
        float t = 0;
        SPP_HIP(hipEventElapsedTime(&t, pr.first, pr.second));
        ms += t;
      }
      n = T.launches[kclass];
      by = T.bytes[kclass];
      fl = T.flops[kclass];
    }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = n;
    if (bytes) *bytes = by;
    if (flops) *flops = fl;
    return SPP_OK;
  });
}

int spp_kernel_timing_reset(spp_factor* factor) {
  return guarded([&] {
    if (!factor) throw Error(SPP_EINVAL, "null factor");
    if (factor->timer) factor->timer = std::make_unique<KernelTimer>();
    return SPP_OK;
  });
}

void spp_destroy(spp_factor* factor) {
  if (!factor) return;
  if (factor->last_stream) (void)hipStreamSynchronize(factor->last_stream);
  else (void)hipDeviceSynchronize();
  delete factor;
}

const char* spp_error_string(int code) {
  switch (code) {
    case SPP_OK: return "success";
    case SPP_EINVAL: return "invalid argument";
    case SPP_ESINGULAR_SHIFT: return "L - s is singular and could not be perturbed away";
    case SPP_EBREAKDOWN: return "pivot breakdown in a frontal matrix";
    case SPP_NOT_CONVERGED: return "GMRES did not reach the tolerance";
    case SPP_ENOMEM: return "out of device memory";
    case SPP_EHIP: return "HIP runtime error";
    case SPP_ENOTIMPL: return "not implemented";
    default: return "unknown error";
  }
}

const char* spp_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
