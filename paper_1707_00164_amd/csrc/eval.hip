// GPU evaluation of K~ W on MI355X (gfx950).
//
// Every step of Alg. "Evaluate" (Sec. 2.2) is a list of gather-GEMM tasks
// (see pack.cpp); one kernel template runs a list level by level:
//
//   out[m x r] (=|+=) A[m x k] B[k x r]
//
// A is a packed operator block (P, P^T, coupling K(b~, a~) or near K(b, a)),
// B's rows are gathered by row code from the caller's W or from the skeleton
// workspace, and out's rows are scattered the same way (the permutation is
// folded into the codes).  Work item = one BM x BN output tile.  The k loop
// stages a BM x 32 slab of A and a 32 x BN slab of B through LDS (B is
// transposed on the way in so both operands are read k-contiguous), with the
// next slab's global loads in flight while the matrix cores work on the
// current one.  Matrix-core instructions (64-wide waves, 4 waves per block):
//
//   FP32    v_mfma_f32_32x32x2_f32   (A, B in FP32)
//   BF16    v_mfma_f32_32x32x16_bf16 (A stored BF16, B rounded to BF16)
//   BF16X3  three v_mfma_f32_32x32x16_bf16 per step on split operands,
//           a_hi b_hi + a_hi b_lo + a_lo b_hi, with x = hi + lo, hi = bf16(x),
//           lo = bf16(x - hi): about 16 significant bits per operand.
//
// Accumulation is FP32 in the matrix-core accumulators.  This file holds the
// host side: device buffers, work-item lists and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "kernels.hpp"

namespace gofmm {

// ------------------------------------------------------------------ configurations
using dev::Cfg;
using dev::KernelFn;
using dev::kCfgs;
using dev::kNumCfg;
using dev::kNumFamily;

// family: 0 upward pass, 1 far field, 2 downward pass (accumulating),
// 3 leaf output, 4 leaf output accumulating
static int family_of(const LaunchDesc& l) {
  if (l.kind == 0 || l.kind == 1) return 0;
  if (l.kind == 2) return 1;
  if (l.kind == 6) return 2;
  return l.accumulate ? 4 : 3;
}

// [vec][precision]: vec = 1 when every row of W, U and the workspace is
// 16-byte aligned and r % 4 == 0
struct Tables {
  KernelFn k[2][3][kNumCfg * kNumFamily];
  dev::BatchedFn b[2][3][kNumCfg];
  Tables() {
    dev::kernels_f32_vec(k[1][PREC_F32], b[1][PREC_F32]);
    dev::kernels_f32_any(k[0][PREC_F32], b[0][PREC_F32]);
    dev::kernels_bf16_vec(k[1][PREC_BF16], b[1][PREC_BF16]);
    dev::kernels_bf16_any(k[0][PREC_BF16], b[0][PREC_BF16]);
    dev::kernels_x3_vec(k[1][PREC_BF16X3], b[1][PREC_BF16X3]);
    dev::kernels_x3_any(k[0][PREC_BF16X3], b[0][PREC_BF16X3]);
  }
};
static const Tables& tables() {
  static Tables t;
  return t;
}

static KernelFn kernel_for(const LaunchDesc& l, int cfg, bool vec) {
  return tables().k[vec ? 1 : 0][l.prec][cfg * kNumFamily + family_of(l)];
}

// ------------------------------------------------------------------ device state
struct DeviceState {
  int device = -1;
  float* a_f32 = nullptr;
  uint16_t* a_b16 = nullptr;
  uint16_t* a_x3 = nullptr;
  i64 x3_plane = 0;
  TaskDesc* tasks = nullptr;
  i32* rows = nullptr;
  float* ws = nullptr;
  i64 ws_cols = 0;                  // floats per workspace row allocated
  // work-item lists per (launch, configuration, column tiles)
  std::map<std::tuple<int, int, int>, std::pair<int2*, int>> items;
  std::map<std::pair<int, i64>, int> tuned;   // (launch, r) -> configuration
  i64 op_bytes = 0;
  // per-launch timing (HIP events around every launch while enabled)
  bool profiling = false;
  int prof_only = -1;       // >= 0: record only this launch
  std::vector<hipEvent_t> events;
  size_t ev_used = 0;
  struct Rec { int launch; hipEvent_t a, b; };
  std::vector<Rec> pending;
};

#define HIP_OK(expr)                                                                 \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      fail(e_ == hipErrorOutOfMemory ? GOFMM_ENOMEM : GOFMM_EHIP,                    \
           std::string(#expr) + ": " + hipGetErrorString(e_));                       \
  } while (0)

void device_state_free(DeviceState* d) {
  if (!d) return;
  int cur = -1;
  (void)hipGetDevice(&cur);
  if (d->device >= 0) (void)hipSetDevice(d->device);
  (void)hipFree(d->a_f32);
  (void)hipFree(d->a_b16);
  (void)hipFree(d->a_x3);
  (void)hipFree(d->tasks);
  (void)hipFree(d->rows);
  (void)hipFree(d->ws);
  for (auto& kv : d->items) (void)hipFree(kv.second.first);
  for (auto& ev : d->events) (void)hipEventDestroy(ev);
  if (cur >= 0) (void)hipSetDevice(cur);
  delete d;
}

template <class T>
static void upload(T** dst, const std::vector<T>& src, i64& bytes) {
  if (src.empty()) return;
  HIP_OK(hipMalloc((void**)dst, src.size() * sizeof(T)));
  HIP_OK(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  bytes += (i64)(src.size() * sizeof(T));
}

static i64 ws_cols_for(i64 r) { return std::max<i64>(4, (r + 3) / 4 * 4); }

void device_prepare(Compression& c, i64 r_max) {
  if (r_max < 1) r_max = 1;
  int cur;
  HIP_OK(hipGetDevice(&cur));
  if (c.dev && c.dev->device != cur) fail(GOFMM_EINVAL, "compression was prepared on another device");
  if (!c.dev) {
    DeviceState* d = new DeviceState;
    d->device = cur;
    try {
      const HostPlan& pl = c.plan;
      upload(&d->a_f32, pl.a_f32, d->op_bytes);
      upload(&d->a_b16, pl.a_b16, d->op_bytes);
      if (!pl.a_x3.empty()) {
        d->x3_plane = pl.x3_plane;
        upload(&d->a_x3, pl.a_x3, d->op_bytes);
      }
      upload(&d->tasks, pl.tasks, d->op_bytes);
      upload(&d->rows, pl.rows, d->op_bytes);
    } catch (...) {
      device_state_free(d);
      throw;
    }
    c.dev = d;
  }
  DeviceState* d = c.dev;
  const i64 cols = ws_cols_for(r_max);
  if (cols > d->ws_cols) {
    HIP_OK(hipDeviceSynchronize());
    (void)hipFree(d->ws);
    d->ws = nullptr;
    d->ws_cols = 0;
    const i64 rows = std::max<i64>(1, c.plan.ws_rows);
    HIP_OK(hipMalloc((void**)&d->ws, (size_t)rows * cols * sizeof(float)));
    d->ws_cols = cols;
  }
}

constexpr int kXcds = 8;   // MI355X: blocks are dealt to the 8 XCDs round-robin by id

// Work items of launch li for tile configuration cfg and ntn column tiles:
// the (task, row tile) groups sorted by k (longest first) are assigned to the
// least-loaded XCD; each group's ntn column tiles stay on that XCD (they
// share the A rows), and block id b runs item b % 8's queue entry b / 8.
static std::vector<int2> build_items(const HostPlan& pl, const LaunchDesc& l, int bm, int ntn) {
  struct G { i32 task, mt; i64 cost; };
  std::vector<G> groups;
  for (i32 k = l.t_begin; k < l.t_end; ++k)
    for (int mt = 0; mt * bm < pl.tasks[k].m; ++mt)
      groups.push_back({k, mt, (i64)std::max(pl.tasks[k].lda, 32)});
  std::stable_sort(groups.begin(), groups.end(), [](const G& x, const G& y) { return x.cost > y.cost; });
  std::vector<std::vector<int2>> q(kXcds);
  std::vector<i64> load(kXcds, 0);
  for (const G& g : groups) {
    int best = 0;
    for (int x = 1; x < kXcds; ++x)
      if (load[x] < load[best]) best = x;
    load[best] += g.cost * ntn;
    for (int nt = 0; nt < ntn; ++nt) q[best].push_back(make_int2(g.task, (g.mt << 16) | nt));
  }
  size_t len = 0;
  for (auto& v : q) len = std::max(len, v.size());
  std::vector<int2> items(len * kXcds, make_int2(-1, 0));
  for (int x = 0; x < kXcds; ++x)
    for (size_t j = 0; j < q[x].size(); ++j) items[j * kXcds + x] = q[x][j];
  return items;
}

static std::pair<int2*, int> items_for(Compression& c, int li, int cfg, int ntn) {
  DeviceState* d = c.dev;
  const auto key = std::make_tuple(li, cfg, ntn);
  auto it = d->items.find(key);
  if (it != d->items.end()) return it->second;
  if (ntn >= (1 << 16)) fail(GOFMM_ELIMIT, "too many column tiles");
  const LaunchDesc& l = c.plan.launches[li];
  for (i32 k = l.t_begin; k < l.t_end; ++k)
    if ((c.plan.tasks[k].m + kCfgs[cfg].bm - 1) / kCfgs[cfg].bm >= (1 << 15)) fail(GOFMM_ELIMIT, "too many row tiles");
  std::vector<int2> v = build_items(c.plan, l, kCfgs[cfg].bm, ntn);
  int2* dp = nullptr;
  if (!v.empty()) {
    HIP_OK(hipMalloc((void**)&dp, v.size() * sizeof(int2)));
    HIP_OK(hipMemcpy(dp, v.data(), v.size() * sizeof(int2), hipMemcpyHostToDevice));
  }
  d->items[key] = {dp, (int)v.size()};
  return d->items[key];
}

// Padded-work model: tile count x tile area x k, plus a per-tile overhead.
static int choose_cfg(const Compression& c, int li, i64 r) {
  const LaunchDesc& l = c.plan.launches[li];
  double best = 1e300;
  int bc = 0;
  for (int q = 0; q < kNumCfg; ++q) {
    const Cfg& g = kCfgs[q];
    const double nt = (double)((r + g.bn - 1) / g.bn);
    double cost = 0.0, tiles = 0.0;
    for (i32 k = l.t_begin; k < l.t_end; ++k) {
      const TaskDesc& t = c.plan.tasks[k];
      const double mt = (double)((t.m + g.bm - 1) / g.bm);
      cost += mt * nt * g.bm * g.bn * (double)std::max(t.lda, 32);
      tiles += mt * nt;
    }
    const double fill = std::min(1.0, tiles / 256.0);
    cost = cost / fill + tiles * 32.0 * 128 * 128;
    if (cost < best) { best = cost; bc = q; }
  }
  return bc;
}

struct EvalArgs {
  i64 r;
  const float* W;
  i64 ldw;
  float* U;
  i64 ldu;
  hipStream_t stream;
};

static bool make_args(Compression& c, int li, int cfg, const EvalArgs& e, dev::KArgs& a, int& grid) {
  DeviceState* d = c.dev;
  const LaunchDesc& l = c.plan.launches[li];
  const Cfg& g = kCfgs[cfg];
  const int ntn = (int)((e.r + g.bn - 1) / g.bn);
  auto it = items_for(c, li, cfg, ntn);
  if (it.second == 0) return false;
  a.tasks = d->tasks;
  a.items = it.first;
  a.A = l.prec == PREC_F32 ? (const void*)d->a_f32 : l.prec == PREC_BF16 ? (const void*)d->a_b16 : (const void*)d->a_x3;
  a.plane = d->x3_plane;
  a.rows = d->rows;
  a.W = e.W;
  a.ldw = e.ldw;
  a.U = e.U;
  a.ldu = e.ldu;
  a.WS = d->ws;
  a.ldws = ws_cols_for(e.r);
  a.r = (int)e.r;
  a.vec = ((uintptr_t)e.W % 16 == 0) && ((uintptr_t)e.U % 16 == 0) && e.ldw % 4 == 0 && e.ldu % 4 == 0 && e.r % 4 == 0;
  grid = it.second;
  return true;
}

// GOFMM_TILE=<index> forces one tile shape for every launch (testing aid).
static int forced_tile() {
  const char* e = std::getenv("GOFMM_TILE");
  if (!e || !*e) return -1;
  const int v = std::atoi(e);
  return (v >= 0 && v < kNumCfg) ? v : -1;
}

static int cfg_for(Compression& c, int li, i64 r) {
  const int f = forced_tile();
  if (f >= 0) return f;
  auto it = c.dev->tuned.find({li, r});
  return it != c.dev->tuned.end() ? it->second : choose_cfg(c, li, r);
}

static void launch_all(Compression& c, const EvalArgs& e) {
  DeviceState* d = c.dev;
  for (int li = 0; li < (int)c.plan.launches.size(); ++li) {
    const LaunchDesc& l = c.plan.launches[li];
    const int cfg = cfg_for(c, li, e.r);
    dev::KArgs a;
    int grid = 0;
    if (!make_args(c, li, cfg, e, a, grid)) continue;
    KernelFn fn = kernel_for(l, cfg, a.vec != 0);
    if (d->profiling && (d->prof_only < 0 || d->prof_only == li)) {
      hipEvent_t ev[2];
      for (int q = 0; q < 2; ++q) {
        if (d->ev_used >= d->events.size()) {
          hipEvent_t x;
          HIP_OK(hipEventCreate(&x));
          d->events.push_back(x);
        }
        ev[q] = d->events[d->ev_used++];
      }
      HIP_OK(hipEventRecord(ev[0], e.stream));
      hipLaunchKernelGGL(fn, dim3(grid), dim3(dev::NT), 0, e.stream, a);
      HIP_OK(hipGetLastError());
      HIP_OK(hipEventRecord(ev[1], e.stream));
      d->pending.push_back({li, ev[0], ev[1]});
    } else {
      hipLaunchKernelGGL(fn, dim3(grid), dim3(dev::NT), 0, e.stream, a);
      HIP_OK(hipGetLastError());
    }
  }
}

void device_evaluate(Compression& c, i64 r, const float* W, i64 ldw, float* U, i64 ldu, void* stream) {
  if (!c.dev || ws_cols_for(r) > c.dev->ws_cols) device_prepare(c, r);
  int cur;
  HIP_OK(hipGetDevice(&cur));
  if (c.dev->device != cur) fail(GOFMM_EINVAL, "current device differs from the compression's device");
  if (r > INT32_MAX / 2) fail(GOFMM_ELIMIT, "r too large");
  launch_all(c, EvalArgs{r, W, ldw, U, ldu, (hipStream_t)stream});
}

// Time every configuration of every launch for this r and keep the fastest.
void device_autotune(Compression& c, i64 r, const float* W, i64 ldw, float* U, i64 ldu, void* stream,
                     int reps) {
  device_evaluate(c, r, W, ldw, U, ldu, stream);          // prepares and warms up
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  const EvalArgs e{r, W, ldw, U, ldu, st};
  const bool prof = c.dev->profiling;
  c.dev->profiling = false;
  for (int li = 0; li < (int)c.plan.launches.size(); ++li) {
    float best = 1e30f;
    int bc = choose_cfg(c, li, r);
    for (int q = 0; q < kNumCfg; ++q) {
      dev::KArgs a;
      int grid = 0;
      if (!make_args(c, li, q, e, a, grid)) continue;
      // accumulating launches would change their output; time them overwriting
      LaunchDesc lo = c.plan.launches[li];
      if (lo.kind == 6) lo.kind = 1;
      lo.accumulate = 0;
      KernelFn fn = kernel_for(lo, q, a.vec != 0);
      hipLaunchKernelGGL(fn, dim3(grid), dim3(dev::NT), 0, st, a);
      HIP_OK(hipEventRecord(e0, st));
      for (int t = 0; t < reps; ++t) hipLaunchKernelGGL(fn, dim3(grid), dim3(dev::NT), 0, st, a);
      HIP_OK(hipEventRecord(e1, st));
      HIP_OK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_OK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) { best = ms; bc = q; }
      if (std::getenv("GOFMM_TUNE_LOG"))
        std::fprintf(stderr, "tune %s r=%lld cfg %dx%d: %.4f ms\n", c.plan.launches[li].name.c_str(),
                     (long long)r, kCfgs[q].bm, kCfgs[q].bn, ms / reps);
    }
    c.dev->tuned[{li, r}] = bc;
  }
  c.dev->profiling = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // the timing runs overwrote intermediate rows: recompute a clean result
  device_evaluate(c, r, W, ldw, U, ldu, stream);
}

void device_profile(Compression& c, int mode) {
  if (!c.dev) device_prepare(c, 1);
  c.dev->profiling = mode != 0;
  c.dev->prof_only = mode >= 2 ? mode - 2 : -1;
}

// Sum of recorded launch times (ms) and record counts per launch; clears the records.
void device_profile_read(Compression& c, int n, float* total_ms, int* calls) {
  for (int i = 0; i < n; ++i) { total_ms[i] = 0.f; calls[i] = 0; }
  if (!c.dev) return;
  DeviceState* d = c.dev;
  for (auto& r : d->pending) {
    HIP_OK(hipEventSynchronize(r.b));
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, r.a, r.b));
    if (r.launch < n) { total_ms[r.launch] += ms; calls[r.launch] += 1; }
  }
  d->pending.clear();
  d->ev_used = 0;
}

i64 device_footprint(const Compression& c, i64 r_max) {
  const HostPlan& pl = c.plan;
  i64 b = (i64)(pl.a_f32.size() * 4 + pl.a_b16.size() * 2 + pl.a_x3.size() * 2 +
                pl.tasks.size() * sizeof(TaskDesc) + pl.rows.size() * 4);
  b += std::max<i64>(1, pl.ws_rows) * ws_cols_for(r_max) * 4;
  // work-item lists: one entry per 32 rows x 32 columns of every task, plus XCD padding
  i64 entries = 0;
  for (const auto& t : pl.tasks) entries += (t.m + 31) / 32;
  b += (entries * ((r_max + 31) / 32) + (i64)pl.launches.size() * kXcds) * 8;
  return b;
}

// ------------------------------------------------------------------ batched launch
static long long& spin_limit_ref() {
  static long long v = 1ll << 21;
  return v;
}
void device_set_spin_limit(long long v) { spin_limit_ref() = v > 0 ? v : (1ll << 21); }

static int batch_prec(int k, Compression* const* c) {
  int prec = -1;
  for (int i = 0; i < k; ++i)
    for (const LaunchDesc& l : c[i]->plan.launches) {
      if (prec < 0) prec = l.prec;
      else if (prec != l.prec)
        fail(GOFMM_EINVAL, "a batched launch needs one storage precision for every step of every compression");
    }
  return prec < 0 ? PREC_F32 : prec;
}

int device_batch_precision(Compression& c) {
  Compression* p = &c;
  return batch_prec(1, &p);
}

// Stage-major queue: stage j of every instance precedes stage j + 1 of any;
// within a stage position, tiles are ordered longest-k first.  need[s] is the
// tile count of stage s's predecessor.
static void build_batch_tables(int k, Compression* const* c, const i64* r, int cfg, std::vector<dev::BItem>& items,
                               std::vector<int>& prev, std::vector<int>& need, std::vector<int>& acc) {
  const Cfg& g = kCfgs[cfg];
  items.clear();
  prev.clear();
  need.clear();
  acc.clear();
  std::vector<int> own;
  std::vector<int> last(k, -1);
  size_t max_l = 0;
  for (int i = 0; i < k; ++i) max_l = std::max(max_l, c[i]->plan.launches.size());
  struct T { dev::BItem it; i64 cost; };
  std::vector<T> pos;
  for (size_t j = 0; j < max_l; ++j) {
    pos.clear();
    for (int i = 0; i < k; ++i) {
      const HostPlan& pl = c[i]->plan;
      if (j >= pl.launches.size()) continue;
      const LaunchDesc& l = pl.launches[j];
      const int sid = (int)prev.size();
      const int ntn = (int)((r[i] + g.bn - 1) / g.bn);
      int count = 0;
      for (i32 t = l.t_begin; t < l.t_end; ++t)
        for (int mt = 0; mt * g.bm < pl.tasks[t].m; ++mt)
          for (int nt = 0; nt < ntn; ++nt) {
            pos.push_back({{i, sid, t, (mt << 16) | nt}, (i64)std::max(pl.tasks[t].lda, 32)});
            ++count;
          }
      prev.push_back(last[i]);
      own.push_back(count);
      acc.push_back(l.accumulate);
      last[i] = sid;
    }
    std::stable_sort(pos.begin(), pos.end(), [](const T& x, const T& y) { return x.cost > y.cost; });
    for (auto& t : pos) items.push_back(t.it);
  }
  need.resize(prev.size());
  for (size_t s2 = 0; s2 < prev.size(); ++s2) need[s2] = prev[s2] < 0 ? 0 : own[prev[s2]];
}

static int batch_cfg_model(int k, Compression* const* c, const i64* r) {
  double best = 1e300;
  int bc = 0;
  for (int q = 0; q < kNumCfg; ++q) {
    const Cfg& g = kCfgs[q];
    double cost = 0.0;
    for (int i = 0; i < k; ++i) {
      const double nt = (double)((r[i] + g.bn - 1) / g.bn);
      for (const TaskDesc& t : c[i]->plan.tasks)
        cost += (double)((t.m + g.bm - 1) / g.bm) * nt * (g.bm * g.bn * (double)std::max(t.lda, 32) + 32.0 * 128 * 128);
    }
    if (cost < best) { best = cost; bc = q; }
  }
  return bc;
}

static int batch_grid_cap(int prec, int cfg) {
  static std::map<std::pair<int, int>, int> cache;
  static std::mutex mu;
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find({prec, cfg});
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0, devid = 0;
  HIP_OK(hipGetDevice(&devid));
  HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, tables().b[1][prec][cfg], dev::NT, 0));
  HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, devid));
  const int cap = std::max(1, per_cu) * std::max(1, cus);
  cache[{prec, cfg}] = cap;
  return cap;
}

BatchRing::~BatchRing() {
  for (auto& s : slot) {
    if (s.ev) (void)hipEventSynchronize((hipEvent_t)s.ev);
    (void)hipFree(s.dev);
    (void)hipHostFree(s.host);
    if (s.ev) (void)hipEventDestroy((hipEvent_t)s.ev);
  }
}

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// One batched launch through a staging slot: the host tables go to pinned
// memory, one async copy moves them (with the zeroed counters) to the device,
// the kernel runs, and the error flag is copied back to pinned memory.
void ring_launch(BatchRing& ring, int k, Compression* const* c, const i64* r, const float* const* W,
                 const i64* ldw, float* const* U, const i64* ldu, hipStream_t st, int cfg) {
  const int prec = batch_prec(k, c);
  std::vector<dev::BItem> items;
  std::vector<int> prev, need, acc;
  build_batch_tables(k, c, r, cfg, items, prev, need, acc);
  const int ns = (int)prev.size();
  const size_t o_cnt = 0, n_cnt = (size_t)(ns + 2) * sizeof(int);
  const size_t o_tab = align256(o_cnt + n_cnt), n_tab = (size_t)3 * ns * sizeof(int);
  const size_t o_inst = align256(o_tab + n_tab), n_inst = (size_t)k * sizeof(dev::BInst);
  const size_t o_item = align256(o_inst + n_inst), n_item = items.size() * sizeof(dev::BItem);
  const size_t o_err = align256(o_item + n_item);
  const size_t total = o_err + 256;
  BatchRing::Slot& s = ring.slot[ring.next];
  const int si = ring.next;
  ring.next = (ring.next + 1) % BatchRing::NS;
  if (s.ev) {
    HIP_OK(hipEventSynchronize((hipEvent_t)s.ev));     // the slot's previous launch has ended
  } else {
    hipEvent_t ev;
    HIP_OK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    s.ev = ev;
  }
  if (total > s.cap) {
    (void)hipFree(s.dev);
    (void)hipHostFree(s.host);
    s.dev = nullptr;
    s.host = nullptr;
    s.cap = 0;
    const size_t cap = total + total / 2;
    HIP_OK(hipMalloc((void**)&s.dev, cap));
    HIP_OK(hipHostMalloc((void**)&s.host, cap, hipHostMallocDefault));
    s.cap = cap;
  }
  char* h = s.host;
  std::memset(h + o_cnt, 0, n_cnt);
  int* tab = reinterpret_cast<int*>(h + o_tab);
  for (int q = 0; q < ns; ++q) {
    tab[q] = prev[q];
    tab[ns + q] = need[q];
    tab[2 * ns + q] = acc[q];
  }
  dev::BInst* in = reinterpret_cast<dev::BInst*>(h + o_inst);
  bool all_vec = true;
  for (int i = 0; i < k; ++i) {
    DeviceState* d = c[i]->dev;
    in[i].tasks = d->tasks;
    in[i].rows = d->rows;
    in[i].A = prec == PREC_F32 ? (const void*)d->a_f32 : prec == PREC_BF16 ? (const void*)d->a_b16 : (const void*)d->a_x3;
    in[i].plane = d->x3_plane;
    in[i].W = W[i];
    in[i].ldw = ldw[i];
    in[i].U = U[i];
    in[i].ldu = ldu[i];
    in[i].WS = d->ws;
    in[i].ldws = ws_cols_for(r[i]);
    in[i].r = (int)r[i];
    in[i].vec = ((uintptr_t)W[i] % 16 == 0) && ((uintptr_t)U[i] % 16 == 0) && ldw[i] % 4 == 0 && ldu[i] % 4 == 0 && r[i] % 4 == 0;
    all_vec = all_vec && in[i].vec;
  }
  if (n_item) std::memcpy(h + o_item, items.data(), n_item);
  *reinterpret_cast<int*>(h + o_err) = 0;
  HIP_OK(hipMemcpyAsync(s.dev, h, o_err, hipMemcpyHostToDevice, st));
  if (!items.empty()) {
    dev::BArgs a;
    char* dv = s.dev;
    a.inst = reinterpret_cast<const dev::BInst*>(dv + o_inst);
    a.items = reinterpret_cast<const dev::BItem*>(dv + o_item);
    a.n_items = (int)items.size();
    a.stage_prev = reinterpret_cast<const int*>(dv + o_tab);
    a.stage_need = a.stage_prev + ns;
    a.stage_acc = a.stage_prev + 2 * ns;
    a.done = reinterpret_cast<int*>(dv + o_cnt);
    a.head = a.done + ns;
    a.error = a.done + ns + 1;
    a.spin_limit = spin_limit_ref();
    const int grid = std::max(1, std::min(a.n_items, batch_grid_cap(prec, cfg)));
    hipLaunchKernelGGL(tables().b[all_vec ? 1 : 0][prec][cfg], dim3(grid), dim3(dev::NT), 0, st, a);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(h + o_err, dv + o_cnt + (size_t)(ns + 1) * sizeof(int), sizeof(int), hipMemcpyDeviceToHost, st));
  }
  HIP_OK(hipEventRecord((hipEvent_t)s.ev, st));
  s.err_off = o_err;
  ring.last = si;
}

// Error flag of the ring's last launch (waits for it).
int ring_status(BatchRing& ring) {
  if (ring.last < 0) return 0;
  BatchRing::Slot& s = ring.slot[ring.last];
  HIP_OK(hipEventSynchronize((hipEvent_t)s.ev));
  return *reinterpret_cast<int*>(s.host + s.err_off);
}

void batch_prepare(int k, Compression* const* c, const i64* r) {
  int cur;
  HIP_OK(hipGetDevice(&cur));
  for (int i = 0; i < k; ++i) {
    if (r[i] < 1) fail(GOFMM_EINVAL, "every instance of a batch needs r >= 1");
    if (!c[i]->dev || ws_cols_for(r[i]) > c[i]->dev->ws_cols) device_prepare(*c[i], r[i]);
    if (c[i]->dev->device != cur) fail(GOFMM_EINVAL, "current device differs from a compression's device");
  }
}

static std::vector<uint64_t> batch_key(int k, Compression* const* c, const i64* r) {
  std::vector<uint64_t> key;
  for (int i = 0; i < k; ++i) {
    key.push_back(c[i]->uid);
    key.push_back((uint64_t)r[i]);
  }
  return key;
}

static std::mutex& api_mutex() {
  static std::mutex m;
  return m;
}
static BatchRing& api_ring() {
  static BatchRing* r = new BatchRing;   // lives until the process ends
  return *r;
}
static std::map<std::vector<uint64_t>, int>& batch_tuned() {
  static std::map<std::vector<uint64_t>, int> t;
  return t;
}

// All instances' steps in one persistent launch.
void device_evaluate_batched(int k, Compression* const* c, const i64* r, const float* const* W,
                             const i64* ldw, float* const* U, const i64* ldu, void* stream) {
  std::lock_guard<std::mutex> g(api_mutex());
  batch_prepare(k, c, r);
  auto it = batch_tuned().find(batch_key(k, c, r));
  int cfg = it != batch_tuned().end() ? it->second : batch_cfg_model(k, c, r);
  if (forced_tile() >= 0) cfg = forced_tile();
  ring_launch(api_ring(), k, c, r, W, ldw, U, ldu, (hipStream_t)stream, cfg);
}

// Time the whole batched launch with every tile configuration; keep the fastest.
void device_autotune_batched(int k, Compression* const* c, const i64* r, const float* const* W,
                             const i64* ldw, float* const* U, const i64* ldu, void* stream, int reps) {
  {
    std::lock_guard<std::mutex> g(api_mutex());
    batch_prepare(k, c, r);
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    float best = 1e30f;
    int bc = batch_cfg_model(k, c, r);
    for (int q = 0; q < kNumCfg; ++q) {
      ring_launch(api_ring(), k, c, r, W, ldw, U, ldu, st, q);
      HIP_OK(hipEventRecord(e0, st));
      for (int t = 0; t < reps; ++t) ring_launch(api_ring(), k, c, r, W, ldw, U, ldu, st, q);
      HIP_OK(hipEventRecord(e1, st));
      HIP_OK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_OK(hipEventElapsedTime(&ms, e0, e1));
      if (std::getenv("GOFMM_TUNE_LOG"))
        std::fprintf(stderr, "tune batched k=%d cfg %dx%d: %.4f ms\n", k, kCfgs[q].bm, kCfgs[q].bn, ms / reps);
      if (ms < best) { best = ms; bc = q; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    batch_tuned()[batch_key(k, c, r)] = bc;
  }
  device_evaluate_batched(k, c, r, W, ldw, U, ldu, stream);
}

// Waits for the last batched launch made through the API and reports its
// error flag (1 if a dependency wait hit its poll bound).
int device_batched_status() {
  std::lock_guard<std::mutex> g(api_mutex());
  return ring_status(api_ring());
}

int device_batch_cfg(int k, Compression* const* c, const i64* r) { return batch_cfg_model(k, c, r); }

}  // namespace gofmm
