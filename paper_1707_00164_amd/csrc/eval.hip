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

struct Tables {
  KernelFn k[3][kNumCfg * kNumFamily];
  dev::BatchedFn b[3][kNumCfg];
  Tables() {
    dev::kernels_f32(k[PREC_F32], b[PREC_F32]);
    dev::kernels_bf16(k[PREC_BF16], b[PREC_BF16]);
    dev::kernels_x3(k[PREC_BF16X3], b[PREC_BF16X3]);
  }
};
static const Tables& tables() {
  static Tables t;
  return t;
}

static KernelFn kernel_for(const LaunchDesc& l, int cfg) {
  return tables().k[l.prec][cfg * kNumFamily + family_of(l)];
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
      if (!pl.a_x3hi.empty()) {
        std::vector<uint16_t> both(pl.a_x3hi);
        both.insert(both.end(), pl.a_x3lo.begin(), pl.a_x3lo.end());
        d->x3_plane = (i64)pl.a_x3hi.size();
        upload(&d->a_x3, both, d->op_bytes);
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
  a.vec = ((uintptr_t)e.W % 16 == 0) && ((uintptr_t)e.U % 16 == 0) && e.ldw % 4 == 0 && e.ldu % 4 == 0;
  grid = it.second;
  return true;
}

static int cfg_for(Compression& c, int li, i64 r) {
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
    KernelFn fn = kernel_for(l, cfg);
    if (d->profiling) {
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
      KernelFn fn = kernel_for(lo, q);
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

void device_profile(Compression& c, int on) {
  if (!c.dev) device_prepare(c, 1);
  c.dev->profiling = on != 0;
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
  i64 b = (i64)(pl.a_f32.size() * 4 + pl.a_b16.size() * 2 + (pl.a_x3hi.size() + pl.a_x3lo.size()) * 2 +
                pl.tasks.size() * sizeof(TaskDesc) + pl.rows.size() * 4);
  b += std::max<i64>(1, pl.ws_rows) * ws_cols_for(r_max) * 4;
  // work-item lists: one entry per 32 rows x 32 columns of every task, plus XCD padding
  i64 entries = 0;
  for (const auto& t : pl.tasks) entries += (t.m + 31) / 32;
  b += (entries * ((r_max + 31) / 32) + (i64)pl.launches.size() * kXcds) * 8;
  return b;
}

// ------------------------------------------------------------------ batched launch
struct BatchPlan;
static BatchPlan*& last_batch() {
  static BatchPlan* p = nullptr;
  return p;
}
static long long& spin_limit_ref() {
  static long long v = 1ll << 21;
  return v;
}
static long long batch_spin_limit() { return spin_limit_ref(); }
void device_set_spin_limit(long long v) { spin_limit_ref() = v > 0 ? v : (1ll << 21); }

struct BatchPlan {
  std::vector<uint64_t> key;     // compression ids and r values, then the configuration
  int prec = 0, cfg = 0;
  dev::BItem* items = nullptr;
  int n_items = 0;
  int* stage_tab = nullptr;      // prev, need, acc (3 x n_stages)
  int n_stages = 0;
  int* counters = nullptr;       // done[n_stages], head, error
  dev::BInst* inst = nullptr;
  int k = 0;
  int grid = 0;
  ~BatchPlan() {
    (void)hipFree(items);
    (void)hipFree(stage_tab);
    (void)hipFree(counters);
    (void)hipFree(inst);
  }
};

static std::vector<std::unique_ptr<BatchPlan>>& batch_cache() {
  static std::vector<std::unique_ptr<BatchPlan>> c;   // most recent last
  return c;
}
static std::map<std::vector<uint64_t>, int>& batch_tuned() {
  static std::map<std::vector<uint64_t>, int> t;
  return t;
}

static std::vector<uint64_t> batch_key(int k, Compression* const* c, const i64* r) {
  std::vector<uint64_t> key;
  for (int i = 0; i < k; ++i) {
    key.push_back(c[i]->uid);
    key.push_back((uint64_t)r[i]);
  }
  return key;
}

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

// Stage-major queue: stage j of every instance precedes stage j + 1 of any;
// within a stage position, tiles are ordered longest-k first.
static BatchPlan* batch_plan(int k, Compression* const* c, const i64* r, int cfg) {
  std::vector<uint64_t> key = batch_key(k, c, r);
  key.push_back((uint64_t)cfg);
  auto& cache = batch_cache();
  for (size_t i = 0; i < cache.size(); ++i)
    if (cache[i]->key == key) {
      std::unique_ptr<BatchPlan> p = std::move(cache[i]);
      cache.erase(cache.begin() + i);
      cache.push_back(std::move(p));
      return cache.back().get();
    }
  std::unique_ptr<BatchPlan> bp(new BatchPlan);
  bp->key = key;
  bp->prec = batch_prec(k, c);
  bp->cfg = cfg;
  bp->k = k;
  const Cfg& g = kCfgs[cfg];
  std::vector<int> prev, need, acc;
  std::vector<std::vector<int>> stage_of(k);   // stage id of instance i's j-th launch
  size_t max_l = 0;
  for (int i = 0; i < k; ++i) max_l = std::max(max_l, c[i]->plan.launches.size());
  std::vector<dev::BItem> items;
  for (size_t j = 0; j < max_l; ++j) {
    struct T { dev::BItem it; i64 cost; };
    std::vector<T> pos;
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
      const int ps = j == 0 ? -1 : stage_of[i][j - 1];
      prev.push_back(ps);
      need.push_back(ps < 0 ? 0 : 0);
      acc.push_back(l.accumulate);
      stage_of[i].push_back(sid);
      // remember the tile count of this stage for its successor's wait
      need.back() = count;          // temporarily the stage's own count
    }
    std::stable_sort(pos.begin(), pos.end(), [](const T& x, const T& y) { return x.cost > y.cost; });
    for (auto& t : pos) items.push_back(t.it);
  }
  // need[s] must be the tile count of prev[s]; convert from own counts
  std::vector<int> own(need);
  for (size_t s2 = 0; s2 < prev.size(); ++s2) need[s2] = prev[s2] < 0 ? 0 : own[prev[s2]];
  bp->n_stages = (int)prev.size();
  bp->n_items = (int)items.size();
  std::vector<int> tab(prev);
  tab.insert(tab.end(), need.begin(), need.end());
  tab.insert(tab.end(), acc.begin(), acc.end());
  if (!items.empty()) {
    HIP_OK(hipMalloc((void**)&bp->items, items.size() * sizeof(dev::BItem)));
    HIP_OK(hipMemcpy(bp->items, items.data(), items.size() * sizeof(dev::BItem), hipMemcpyHostToDevice));
  }
  HIP_OK(hipMalloc((void**)&bp->stage_tab, std::max<size_t>(1, tab.size()) * sizeof(int)));
  if (!tab.empty()) HIP_OK(hipMemcpy(bp->stage_tab, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice));
  HIP_OK(hipMalloc((void**)&bp->counters, (bp->n_stages + 2) * sizeof(int)));
  HIP_OK(hipMalloc((void**)&bp->inst, k * sizeof(dev::BInst)));
  dev::BatchedFn fn = tables().b[bp->prec][cfg];
  int per_cu = 0, cus = 0, devid = 0;
  HIP_OK(hipGetDevice(&devid));
  HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, dev::NT, 0));
  HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, devid));
  bp->grid = std::max(1, std::min(bp->n_items, std::max(1, per_cu) * std::max(1, cus)));
  if (cache.size() >= 16) {
    if (last_batch() == cache.front().get()) last_batch() = nullptr;
    cache.erase(cache.begin());
  }
  cache.push_back(std::move(bp));
  return cache.back().get();
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

static void batch_launch(BatchPlan* bp, int k, Compression* const* c, const i64* r, const float* const* W,
                         const i64* ldw, float* const* U, const i64* ldu, hipStream_t st) {
  std::vector<dev::BInst> in(k);
  for (int i = 0; i < k; ++i) {
    DeviceState* d = c[i]->dev;
    const int prec = bp->prec;
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
    in[i].vec = ((uintptr_t)W[i] % 16 == 0) && ((uintptr_t)U[i] % 16 == 0) && ldw[i] % 4 == 0 && ldu[i] % 4 == 0;
  }
  HIP_OK(hipMemcpyAsync(bp->inst, in.data(), k * sizeof(dev::BInst), hipMemcpyHostToDevice, st));
  HIP_OK(hipMemsetAsync(bp->counters, 0, (bp->n_stages + 2) * sizeof(int), st));
  if (bp->n_items == 0) return;
  dev::BArgs a;
  a.inst = bp->inst;
  a.items = bp->items;
  a.n_items = bp->n_items;
  a.stage_prev = bp->stage_tab;
  a.stage_need = bp->stage_tab + bp->n_stages;
  a.stage_acc = bp->stage_tab + 2 * bp->n_stages;
  a.done = bp->counters;
  a.head = bp->counters + bp->n_stages;
  a.error = bp->counters + bp->n_stages + 1;
  a.spin_limit = batch_spin_limit();
  hipLaunchKernelGGL(tables().b[bp->prec][bp->cfg], dim3(bp->grid), dim3(dev::NT), 0, st, a);
  HIP_OK(hipGetLastError());
  last_batch() = bp;
}

static void batch_prepare(int k, Compression* const* c, const i64* r) {
  int cur;
  HIP_OK(hipGetDevice(&cur));
  for (int i = 0; i < k; ++i) {
    if (r[i] < 1) fail(GOFMM_EINVAL, "every instance of a batch needs r >= 1");
    if (!c[i]->dev || ws_cols_for(r[i]) > c[i]->dev->ws_cols) device_prepare(*c[i], r[i]);
    if (c[i]->dev->device != cur) fail(GOFMM_EINVAL, "current device differs from a compression's device");
  }
}

// All instances' steps in one persistent launch.
void device_evaluate_batched(int k, Compression* const* c, const i64* r, const float* const* W,
                             const i64* ldw, float* const* U, const i64* ldu, void* stream) {
  batch_prepare(k, c, r);
  auto it = batch_tuned().find(batch_key(k, c, r));
  const int cfg = it != batch_tuned().end() ? it->second : batch_cfg_model(k, c, r);
  BatchPlan* bp = batch_plan(k, c, r, cfg);
  batch_launch(bp, k, c, r, W, ldw, U, ldu, (hipStream_t)stream);
}

// Time the whole batched launch with every tile configuration; keep the fastest.
void device_autotune_batched(int k, Compression* const* c, const i64* r, const float* const* W,
                             const i64* ldw, float* const* U, const i64* ldu, void* stream, int reps) {
  batch_prepare(k, c, r);
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  float best = 1e30f;
  int bc = batch_cfg_model(k, c, r);
  for (int q = 0; q < kNumCfg; ++q) {
    BatchPlan* bp = batch_plan(k, c, r, q);
    batch_launch(bp, k, c, r, W, ldw, U, ldu, st);
    HIP_OK(hipEventRecord(e0, st));
    for (int t = 0; t < reps; ++t) batch_launch(bp, k, c, r, W, ldw, U, ldu, st);
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
  device_evaluate_batched(k, c, r, W, ldw, U, ldu, stream);
}

// Waits for the device, then reports and clears the error flag of the last
// batched launch (1 if a dependency wait hit its spin limit).
int device_batched_status() {
  BatchPlan* bp = last_batch();
  if (!bp) return 0;
  HIP_OK(hipDeviceSynchronize());
  int flag = 0;
  HIP_OK(hipMemcpy(&flag, bp->counters + bp->n_stages + 1, sizeof(int), hipMemcpyDeviceToHost));
  return flag;
}

}  // namespace gofmm
