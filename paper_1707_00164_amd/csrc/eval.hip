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
  if (l.kind == 4 && !l.accumulate) return 5;
  return l.accumulate ? 4 : 3;
}

// [vec][precision]: vec = 1 when every row of W, U and the workspace is
// 16-byte aligned and r % 4 == 0
struct Tables {
  KernelFn k[2][3][kNumCfg * kNumFamily];
  dev::BatchedFn b[2][3][kNumCfg * 2];   // [cfg * 2]: batched, [cfg * 2 + 1]: tree pass
  KernelFn geo[2][3 * kNumCfg];          // [kernel kind * kNumCfg + cfg]: L2L from points
  Tables() {
    dev::kernels_geo_vec(geo[1]);
    dev::kernels_geo_any(geo[0]);
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

static KernelFn kernel_for(const Compression& c, const LaunchDesc& l, int cfg, bool vec) {
  if (l.kind == 7) return tables().geo[vec ? 1 : 0][c.geo.kind * kNumCfg + cfg];
  return tables().k[vec ? 1 : 0][l.prec][cfg * kNumFamily + family_of(l)];
}

// ------------------------------------------------------------------ device state
struct DeviceState {
  int device = -1;
  float* a_f32 = nullptr;
  uint16_t* a_b16 = nullptr;
  uint16_t* a_x3 = nullptr;
  i64 x3_plane = 0;
  float* geo_cols = nullptr;        // geometric mode: column entries per L2L task
  float* geo_pts = nullptr;         // and the point entries of every index
  TaskDesc* tasks = nullptr;
  i32* rows = nullptr;
  float* ws = nullptr;
  i64 ws_cols = 0;                  // floats per workspace row allocated
  // work-item lists per (launch, configuration, column tiles)
  std::map<std::tuple<int, int, int>, std::pair<int2*, int>> items;
  std::map<std::pair<int, i64>, int> tuned;   // (launch, r) -> configuration; pass segments use -(first + 1)
  // persistent tree passes: device tables per (first launch, configuration, r)
  struct Pass {
    dev::BItem* items = nullptr;
    int* stage_acc = nullptr;
    int* ctr_total = nullptr;
    unsigned long long* ctr = nullptr;    // counters, then the queue head
    int* error = nullptr;
    int n_items = 0, n_ctr = 0, grid = 0;
    unsigned long long epoch = 0, head_base = 0;
  };
  std::map<std::tuple<int, int, i64>, Pass> passes;
  // allocation-free evaluate: per (r, configuration of every launch), the
  // work items of all launches back to back in host memory (never modified
  // once built, so an asynchronous copy may read them), with each launch's
  // (offset, count)
  struct FixedItems {
    std::vector<int2> items;
    std::vector<std::pair<size_t, int>> at;
  };
  std::map<std::vector<i64>, FixedItems> fixed;
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
  for (auto& kv : d->passes) {
    (void)hipFree(kv.second.items);
    (void)hipFree(kv.second.stage_acc);
    (void)hipFree(kv.second.ctr_total);
    (void)hipFree(kv.second.ctr);
    (void)hipFree(kv.second.error);
  }
  (void)hipFree(d->a_f32);
  (void)hipFree(d->a_b16);
  (void)hipFree(d->a_x3);
  (void)hipFree(d->geo_cols);
  (void)hipFree(d->geo_pts);
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
      if (c.geo.kind >= 0) {
        upload(&d->geo_cols, pl.geo_cols, d->op_bytes);
        upload(&d->geo_pts, c.geo.pts, d->op_bytes);
      }
    } catch (...) {
      device_state_free(d);
      throw;
    }
    c.dev = d;
  }
  DeviceState* d = c.dev;
  const i64 cols = ws_cols_for(r_max);
  if (cols > d->ws_cols) {
    // work in flight may still use the old workspace (a fresh state has none)
    if (d->ws) HIP_OK(hipDeviceSynchronize());
    (void)hipFree(d->ws);
    d->ws = nullptr;
    d->ws_cols = 0;
    const i64 rows = std::max<i64>(1, c.plan.ws_rows);
    HIP_OK(hipMalloc((void**)&d->ws, (size_t)rows * cols * sizeof(float)));
    d->ws_cols = cols;
  }
}

constexpr int kXcds = 8;   // MI355X: blocks are dealt to the 8 XCDs round-robin by id

// Work items of launch li for tile configuration cfg and ntn column tiles;
// block id b runs XCD b % 8's queue entry b / 8.  FP32 launches: the (task,
// row tile) groups sorted by k (longest first) are assigned to the
// least-loaded XCD, and each group's ntn column tiles stay on that XCD (they
// share the A rows in its L2).  BF16 and split-BF16 launches, which stream
// their operands two to three times as fast: whole tasks are assigned that
// way, column tile by column tile with the row tiles of each column tile side
// by side, so that the tiles running together on one XCD share both the A
// rows and the gathered B rows, and both reach its L2 about once per task.
static std::vector<int2> build_items(const HostPlan& pl, const LaunchDesc& l, int bm, int ntn) {
  const bool together = l.prec != PREC_F32;
  struct G { i32 task, mt, nmt; i64 cost; };
  std::vector<G> groups;
  for (i32 k = l.t_begin; k < l.t_end; ++k) {
    const int nmt = (int)((pl.tasks[k].m + bm - 1) / bm);
    const i64 kc = (i64)std::max(pl.tasks[k].lda, 32);
    if (nmt == 0) continue;
    if (together)
      groups.push_back({k, 0, nmt, kc * nmt});
    else
      for (int mt = 0; mt * bm < pl.tasks[k].m; ++mt) groups.push_back({k, mt, 1, kc});
  }
  std::stable_sort(groups.begin(), groups.end(), [](const G& x, const G& y) { return x.cost > y.cost; });
  std::vector<std::vector<int2>> q(kXcds);
  std::vector<i64> load(kXcds, 0);
  for (const G& g : groups) {
    int best = 0;
    for (int x = 1; x < kXcds; ++x)
      if (load[x] < load[best]) best = x;
    load[best] += g.cost * ntn;
    for (int nt = 0; nt < ntn; ++nt)
      for (int mt = g.mt; mt < g.mt + g.nmt; ++mt) q[best].push_back(make_int2(g.task, (mt << 16) | nt));
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
    const hipError_t e = hipMemcpy(dp, v.data(), v.size() * sizeof(int2), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(dp);
      fail(GOFMM_EHIP, std::string("hipMemcpy of work items: ") + hipGetErrorString(e));
    }
  }
  d->items[key] = {dp, (int)v.size()};
  return d->items[key];
}

// Cost of one tile in the padded-work model: matrix-core work (weighted by
// the precision: split BF16 issues three BF16 products, which together are
// still cheaper than one FP32 product), operand staging (A and B slabs of the
// tile) and a fixed per-tile latency.
static double tile_cost(const Cfg& g, int prec, double lda) {
  const double w = prec == PREC_F32 ? 1.0 : prec == PREC_BF16X3 ? 1.0 / 3.0 : 1.0 / 8.0;
  return g.bm * g.bn * lda * w + 24.0 * (g.bm + g.bn) * lda + 32.0 * 128 * 128;
}

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
      cost += mt * nt * tile_cost(g, l.prec, (double)std::max(t.lda, 32));
      tiles += mt * nt;
    }
    const double fill = std::min(1.0, tiles / 256.0);
    cost = cost / fill;
    if (cost < best) { best = cost; bc = q; }
  }
  return bc;
}

// ------------------------------------------------------------------ persistent tables
// Node of task t of launch l, and back (the task order of each step is the
// one pack.cpp builds: leaves left to right, the nodes of a level left to
// right, every non-root node in heap order for S2S).
static i64 node_of(const Compression& c, const LaunchDesc& l, i32 t) {
  const i64 o = t - l.t_begin;
  switch (l.kind) {
    case 1: case 6: return ((i64)1 << l.level) - 1 + o;
    case 2: return 1 + o;
    default: return c.fl() + o;                   // leaf steps
  }
}
static i32 task_of(const Compression& c, const LaunchDesc& l, i64 node) {
  switch (l.kind) {
    case 1: case 6: return l.t_begin + (i32)(node - (((i64)1 << l.level) - 1));
    case 2: return l.t_begin + (i32)(node - 1);
    default: return l.t_begin + (i32)(node - c.fl());
  }
}
static int find_launch(const HostPlan& pl, int kind, int level) {
  for (int j = 0; j < (int)pl.launches.size(); ++j)
    if (pl.launches[j].kind == kind && (level < 0 || pl.launches[j].level == level)) return j;
  return -1;
}

// Work items of the launches [j0[i], j1[i]) of every instance i, in stage
// order (launch j of every instance before launch j + 1 of any; longest k
// first within that), with their dependencies:
//   N2S of a node     waits for the N2S tasks of its two children;
//   S2S               waits for the whole upward pass (its last stage: every
//                     task of a stage waited for its children, and every task
//                     has at least one tile since ranks are >= 1);
//   S2N of a node     waits for its own S2S task and for the task that
//                     finished its parent's potential (S2N, or S2S at level 1);
//   leaf output       waits for the task that finished the leaf's potential;
//   L2L (split leaf)  waits for the leaf's S2N-leaf task.
// Dependencies on launches outside the ranges are met by stream order.
// Counters: one per stage, then one per task.
static void build_pass_tables(int k, Compression* const* c, const i64* r, const int* j0, const int* j1, int cfg,
                              std::vector<dev::BItem>& items, std::vector<int>& stage_acc,
                              std::vector<int>& ctr_total) {
  const Cfg& g = kCfgs[cfg];
  items.clear();
  stage_acc.clear();
  ctr_total.clear();
  int max_l = 0;
  for (int i = 0; i < k; ++i) max_l = std::max(max_l, j1[i]);
  std::vector<std::vector<int>> sid(k);             // stage of launch j of instance i, or -1
  std::vector<int> tbase;                           // first task counter (relative) per stage
  std::vector<int> stage_tiles;
  int S = 0, T = 0;
  for (int j = 0; j < max_l; ++j)
    for (int i = 0; i < k; ++i) {
      if ((int)sid[i].size() < max_l) sid[i].assign(max_l, -1);
      if (j < j0[i] || j >= j1[i]) continue;
      const LaunchDesc& l = c[i]->plan.launches[j];
      sid[i][j] = S++;
      tbase.push_back(T);
      T += l.t_end - l.t_begin;
      stage_acc.push_back(l.accumulate);
    }
  ctr_total.assign(S + T, 0);
  auto tiles_of = [&](int i, i32 t) {
    const int ntn = (int)((r[i] + g.bn - 1) / g.bn);
    return (int)((c[i]->plan.tasks[t].m + g.bm - 1) / g.bm) * ntn;
  };
  // tile counts per stage and per task
  for (int i = 0; i < k; ++i)
    for (int j = j0[i]; j < j1[i]; ++j) {
      const LaunchDesc& l = c[i]->plan.launches[j];
      for (i32 t = l.t_begin; t < l.t_end; ++t) {
        const int n = tiles_of(i, t);
        ctr_total[sid[i][j]] += n;
        ctr_total[S + tbase[sid[i][j]] + (t - l.t_begin)] += n;
      }
    }
  auto task_ctr = [&](int i, int j, i32 t) {
    const LaunchDesc& l = c[i]->plan.launches[j];
    return S + tbase[sid[i][j]] + (t - l.t_begin);
  };
  auto in_range = [&](int i, int j) { return j >= 0 && j >= j0[i] && j < j1[i]; };
  struct T2 { dev::BItem it; i64 cost; };
  std::vector<T2> pos;
  for (int j = 0; j < max_l; ++j) {
    pos.clear();
    for (int i = 0; i < k; ++i) {
      if (j < j0[i] || j >= j1[i]) continue;
      const Compression& cc = *c[i];
      const HostPlan& pl = cc.plan;
      const LaunchDesc& l = pl.launches[j];
      const int D = cc.depth;
      const int ntn = (int)((r[i] + g.bn - 1) / g.bn);
      const int j_s2s = find_launch(pl, 2, -1);
      for (i32 t = l.t_begin; t < l.t_end; ++t) {
        int dep[2] = {-1, -1}, need[2] = {0, 0}, nd = 0;
        auto add_task = [&](int jj, i64 node) {
          if (!in_range(i, jj)) return;
          const i32 tt = task_of(cc, pl.launches[jj], node);
          dep[nd] = task_ctr(i, jj, tt);
          need[nd] = tiles_of(i, tt);
          ++nd;
        };
        const i64 h = node_of(cc, l, t);
        if (l.kind == 1) {                          // N2S of a node: its children
          for (i64 ch : {2 * h + 1, 2 * h + 2})
            add_task(l.level + 1 == D ? find_launch(pl, 0, -1) : find_launch(pl, 1, l.level + 1), ch);
        } else if (l.kind == 2) {                   // S2S: the whole upward pass
          const int ju = D >= 2 ? find_launch(pl, 1, 1) : find_launch(pl, 0, -1);
          if (in_range(i, ju)) {
            dep[0] = sid[i][ju];
            need[0] = ctr_total[sid[i][ju]];
            nd = 1;
          }
        } else if (l.kind == 6) {                   // S2N of node h at level >= 2
          add_task(j_s2s, h);
          const i64 p = (h - 1) / 2;
          add_task(l.level >= 3 ? find_launch(pl, 6, l.level - 1) : j_s2s, p);
        } else if (l.kind == 3 || l.kind == 4) {    // leaf output / S2N at the leaf
          if (D >= 2) add_task(find_launch(pl, 6, D), h);
          else if (D == 1) add_task(j_s2s, h);
        } else if (l.kind == 5) {                   // L2L after the leaf's S2N
          add_task(find_launch(pl, 4, -1), h);
        }
        const int tc = task_ctr(i, j, t);
        for (int mt = 0; mt * g.bm < pl.tasks[t].m; ++mt)
          for (int nt = 0; nt < ntn; ++nt) {
            dev::BItem it;
            it.inst = i;
            it.stage = sid[i][j];
            it.task = t;
            it.tile = (mt << 16) | nt;
            it.tctr = tc;
            it.dep[0] = dep[0];
            it.dep[1] = dep[1];
            it.need[0] = need[0];
            it.need[1] = need[1];
            pos.push_back({it, (i64)std::max(pl.tasks[t].lda, 32)});
          }
      }
    }
    std::stable_sort(pos.begin(), pos.end(), [](const T2& x, const T2& y) { return x.cost > y.cost; });
    for (auto& t2 : pos) items.push_back(t2.it);
  }
}

struct EvalArgs {
  i64 r;
  const float* W;
  i64 ldw;
  float* U;
  i64 ldu;
  hipStream_t stream;
};

// Kernel arguments of launch li; `fixed_items` and `fixed_ws` replace the
// library-allocated work items and workspace (the allocation-free evaluate).

// The kernels form a B row's offset as one 32 x 32 -> 64-bit product of the
// row index and the leading dimension, so W's leading dimension must fit 32
// bits (the workspace's is r plus padding).
static void check_ldw(i64 ldw) {
  if (ldw > (i64)UINT32_MAX) fail(GOFMM_ELIMIT, "leading dimension of W above 2^32 - 1");
}
static bool make_args(Compression& c, int li, int cfg, const EvalArgs& e, dev::KArgs& a, int& grid,
                      const std::pair<int2*, int>* fixed_items = nullptr, float* fixed_ws = nullptr) {
  DeviceState* d = c.dev;
  const LaunchDesc& l = c.plan.launches[li];
  const Cfg& g = kCfgs[cfg];
  const int ntn = (int)((e.r + g.bn - 1) / g.bn);
  auto it = fixed_items ? *fixed_items : items_for(c, li, cfg, ntn);
  if (it.second == 0) return false;
  a.tasks = d->tasks;
  a.items = it.first;
  a.A = l.prec == PREC_F32 ? (const void*)d->a_f32 : l.prec == PREC_BF16 ? (const void*)d->a_b16 : (const void*)d->a_x3;
  a.plane = d->x3_plane;
  a.gpts = nullptr;
  a.gh2inv = a.gshift = 0.f;
  a.gacc = l.accumulate;
  if (l.kind == 7) {
    a.A = d->geo_cols;
    a.gpts = d->geo_pts;
    a.gh2inv = c.geo.h2inv;
    a.gshift = c.geo.shift;
  }
  a.rows = d->rows;
  a.W = e.W;
  check_ldw(e.ldw);
  a.ldw = e.ldw;
  a.U = e.U;
  a.ldu = e.ldu;
  a.WS = fixed_ws ? fixed_ws : d->ws;
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

static bool rows_vec(const float* W, i64 ldw, const float* U, i64 ldu, i64 r) {
  return ((uintptr_t)W % 16 == 0) && ((uintptr_t)U % 16 == 0) && ldw % 4 == 0 && ldu % 4 == 0 && r % 4 == 0;
}

static dev::BInst make_inst(Compression& c, int prec, i64 r, const float* W, i64 ldw, float* U, i64 ldu) {
  check_ldw(ldw);
  DeviceState* d = c.dev;
  dev::BInst in;
  in.tasks = d->tasks;
  in.rows = d->rows;
  in.A = prec == PREC_F32 ? (const void*)d->a_f32 : prec == PREC_BF16 ? (const void*)d->a_b16 : (const void*)d->a_x3;
  in.plane = d->x3_plane;
  in.W = W;
  in.ldw = ldw;
  in.U = U;
  in.ldu = ldu;
  in.WS = d->ws;
  in.ldws = ws_cols_for(r);
  in.r = (int)r;
  in.vec = rows_vec(W, ldw, U, ldu, r);
  return in;
}

static long long& spin_limit_ref() {
  static long long lim = 1ll << 21;
  return lim;
}

static int persistent_cap(int prec, int cfg, int which) {
  static std::map<std::tuple<int, int, int>, int> cache;
  static std::mutex mu;
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find({prec, cfg, which});
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0, devid = 0;
  HIP_OK(hipGetDevice(&devid));
  HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, tables().b[1][prec][cfg * 2 + which], kCfgs[cfg].nt, 0));
  HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, devid));
  const int cap = std::max(1, per_cu) * std::max(1, cus);
  cache[{prec, cfg, which}] = cap;
  return cap;
}

// Segments of one evaluate.  By default every launch runs on its own.  With
// GOFMM_PASSES=1 the N2S launches (upward pass) and the S2N level launches
// (downward pass) each run as one persistent launch with per-task
// dependencies (when they hold two or more launches).  Measured on MI355X the
// separate launches are faster: the persistent passes pay device-coherent
// (L2-bypassing) accesses for every row they hand between tiles, while kernel
// boundaries pay one cache write-back per launch.
struct Seg { int j0, j1; bool pass; };
static std::vector<Seg> segments(const HostPlan& pl) {
  const char* ev = std::getenv("GOFMM_PASSES");
  const bool off = !(ev && ev[0] == '1');
  std::vector<Seg> out;
  const int n = (int)pl.launches.size();
  for (int j = 0; j < n;) {
    const int kind = pl.launches[j].kind;
    const int grp = (kind == 0 || kind == 1) ? 1 : kind == 6 ? 2 : 0;
    int e = j + 1;
    if (grp) {
      while (e < n) {
        const int k2 = pl.launches[e].kind;
        if (((k2 == 0 || k2 == 1) ? 1 : k2 == 6 ? 2 : 0) != grp) break;
        ++e;
      }
    }
    if (!off && grp && e - j >= 2) {
      out.push_back({j, e, true});
    } else {
      for (int q = j; q < e; ++q) out.push_back({q, q + 1, false});
    }
    j = e;
  }
  return out;
}

static DeviceState::Pass& pass_for(Compression& c, const Seg& sg, int cfg, i64 r) {
  DeviceState* d = c.dev;
  const auto key = std::make_tuple(sg.j0, cfg, r);
  auto it = d->passes.find(key);
  if (it != d->passes.end()) return it->second;
  Compression* cp = &c;
  std::vector<dev::BItem> items;
  std::vector<int> acc, tot;
  build_pass_tables(1, &cp, &r, &sg.j0, &sg.j1, cfg, items, acc, tot);
  DeviceState::Pass P;
  P.n_items = (int)items.size();
  P.n_ctr = (int)tot.size();
  P.grid = std::max(1, std::min(P.n_items, persistent_cap(c.plan.launches[sg.j0].prec, cfg, 1)));
  try {
    if (!items.empty()) {
      HIP_OK(hipMalloc((void**)&P.items, items.size() * sizeof(dev::BItem)));
      HIP_OK(hipMemcpy(P.items, items.data(), items.size() * sizeof(dev::BItem), hipMemcpyHostToDevice));
    }
    HIP_OK(hipMalloc((void**)&P.stage_acc, std::max<size_t>(1, acc.size()) * sizeof(int)));
    if (!acc.empty()) HIP_OK(hipMemcpy(P.stage_acc, acc.data(), acc.size() * sizeof(int), hipMemcpyHostToDevice));
    HIP_OK(hipMalloc((void**)&P.ctr_total, std::max<size_t>(1, tot.size()) * sizeof(int)));
    if (!tot.empty()) HIP_OK(hipMemcpy(P.ctr_total, tot.data(), tot.size() * sizeof(int), hipMemcpyHostToDevice));
    HIP_OK(hipMalloc((void**)&P.ctr, (tot.size() + 1) * sizeof(unsigned long long)));
    HIP_OK(hipMemset(P.ctr, 0, (tot.size() + 1) * sizeof(unsigned long long)));
    HIP_OK(hipMalloc((void**)&P.error, sizeof(int)));
    HIP_OK(hipMemset(P.error, 0, sizeof(int)));
    HIP_OK(hipDeviceSynchronize());
  } catch (...) {
    (void)hipFree(P.items);
    (void)hipFree(P.stage_acc);
    (void)hipFree(P.ctr_total);
    (void)hipFree(P.ctr);
    (void)hipFree(P.error);
    throw;
  }
  return d->passes[key] = P;
}

// One persistent launch of a pass segment.  Its counters only grow, so the
// launch waits for epoch * (tiles per launch) + need and nothing is cleared;
// launches of one compression must therefore run in the order they are made.
static void launch_pass(Compression& c, const Seg& sg, int cfg, const EvalArgs& e) {
  DeviceState::Pass& P = pass_for(c, sg, cfg, e.r);
  if (P.n_items == 0) return;
  const int prec = c.plan.launches[sg.j0].prec;
  dev::BArgs a;
  a.inst = nullptr;
  a.one = make_inst(c, prec, e.r, e.W, e.ldw, e.U, e.ldu);
  a.items = P.items;
  a.n_items = P.n_items;
  a.stage_acc = P.stage_acc;
  a.ctr_total = P.ctr_total;
  a.ctr = P.ctr;
  a.head = P.ctr + P.n_ctr;
  a.head_base = P.head_base;
  a.epoch = P.epoch;
  a.error = P.error;
  a.spin_limit = spin_limit_ref();
  hipLaunchKernelGGL(tables().b[a.one.vec ? 1 : 0][prec][cfg * 2 + 1], dim3(P.grid), dim3(kCfgs[cfg].nt), 0, e.stream, a);
  HIP_OK(hipGetLastError());
  P.epoch += 1;
  P.head_base += (unsigned long long)P.n_items + (unsigned long long)P.grid;
}

static int cfg_for_seg(Compression& c, const Seg& sg, i64 r) {
  if (!sg.pass) return cfg_for(c, sg.j0, r);
  const int f = forced_tile();
  if (f >= 0) return f;
  auto it = c.dev->tuned.find({-(sg.j0 + 1), r});
  return it != c.dev->tuned.end() ? it->second : choose_cfg(c, sg.j0, r);
}

static void launch_seg(Compression& c, const Seg& sg, int cfg, const EvalArgs& e, bool overwrite_only = false) {
  if (sg.pass) {
    launch_pass(c, sg, cfg, e);
    return;
  }
  dev::KArgs a;
  int grid = 0;
  if (!make_args(c, sg.j0, cfg, e, a, grid)) return;
  LaunchDesc lo = c.plan.launches[sg.j0];
  if (overwrite_only) {              // timing runs: accumulating launches would change their output
    if (lo.kind == 6) lo.kind = 1;
    lo.accumulate = 0;
  }
  a.gacc = lo.accumulate;
  hipLaunchKernelGGL(kernel_for(c, lo, cfg, a.vec != 0), dim3(grid), dim3(kCfgs[cfg].nt), 0, e.stream, a);
  HIP_OK(hipGetLastError());
}

static void launch_all(Compression& c, const EvalArgs& e) {
  DeviceState* d = c.dev;
  for (const Seg& sg : segments(c.plan)) {
    const int cfg = cfg_for_seg(c, sg, e.r);
    const bool rec = d->profiling && (d->prof_only < 0 || (d->prof_only >= sg.j0 && d->prof_only < sg.j1));
    if (!rec) {
      launch_seg(c, sg, cfg, e);
      continue;
    }
    // a pass segment is recorded under its first launch
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
    launch_seg(c, sg, cfg, e);
    HIP_OK(hipEventRecord(ev[1], e.stream));
    d->pending.push_back({sg.j0, ev[0], ev[1]});
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

// ------------------------------------------------------------------ allocation-free evaluate
// For callers that cannot allocate device memory (code under graph capture,
// tight serving loops): the skeleton workspace (w~ and u~ rows) and the work
// items of one evaluate live in `scratch`, a fixed array of every device the
// library runs on, instead of library allocations.  Each device keeps its copy
// until the process ends; every call on a device shares it and leaves its
// contents behind.  Nothing in it needs to start at zero: every workspace row
// is written (S2S, N2S) before it is read or accumulated into, and the work
// items are copied in by each call.
constexpr size_t kScratchBytes = (size_t)GOFMM_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on the current device, looked up once per
// device (each device holds its own copy of the array at its own address).
static unsigned char* scratch_on(int device) {
  static std::mutex mu;
  static std::map<int, unsigned char*> addr;
  std::lock_guard<std::mutex> g(mu);
  auto it = addr.find(device);
  if (it != addr.end()) return it->second;
  void* p = nullptr;
  HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) fail(GOFMM_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
  addr[device] = static_cast<unsigned char*>(p);
  return addr[device];
}

static size_t round256(size_t x) { return (x + 255) / 256 * 256; }

void device_evaluate_noalloc(Compression& c, i64 r, const float* W, i64 ldw, float* U, i64 ldu, void* stream) {
  if (!c.dev) fail(GOFMM_EINVAL, "the compression is not on the device: call gofmm_prepare first");
  int cur;
  HIP_OK(hipGetDevice(&cur));
  if (c.dev->device != cur) fail(GOFMM_EINVAL, "current device differs from the compression's device");
  if (r > INT32_MAX / 2) fail(GOFMM_ELIMIT, "r too large");
  const HostPlan& pl = c.plan;
  const int nl = (int)pl.launches.size();
  std::vector<i64> key(nl + 1);
  key[0] = r;
  for (int li = 0; li < nl; ++li) key[li + 1] = cfg_for(c, li, r);
  DeviceState* d = c.dev;
  auto fit = d->fixed.find(key);
  if (fit == d->fixed.end()) {
    DeviceState::FixedItems f;
    for (int li = 0; li < nl; ++li) {
      const Cfg& g = kCfgs[key[li + 1]];
      const int ntn = (int)((r + g.bn - 1) / g.bn);
      if (ntn >= (1 << 16)) fail(GOFMM_ELIMIT, "too many column tiles");
      const LaunchDesc& l = pl.launches[li];
      for (i32 k = l.t_begin; k < l.t_end; ++k)
        if ((pl.tasks[k].m + g.bm - 1) / g.bm >= (1 << 15)) fail(GOFMM_ELIMIT, "too many row tiles");
      std::vector<int2> v = build_items(pl, l, g.bm, ntn);
      f.at.push_back({f.items.size(), (int)v.size()});
      f.items.insert(f.items.end(), v.begin(), v.end());
    }
    fit = d->fixed.emplace(key, std::move(f)).first;
  }
  const DeviceState::FixedItems& f = fit->second;
  const size_t ws_bytes = round256((size_t)std::max<i64>(1, pl.ws_rows) * (size_t)ws_cols_for(r) * sizeof(float));
  const size_t it_bytes = f.items.size() * sizeof(int2);
  if (ws_bytes + it_bytes > kScratchBytes)
    fail(GOFMM_ELIMIT, "this evaluate needs " + std::to_string(ws_bytes + it_bytes) +
                           " bytes of scratch; the fixed array holds " + std::to_string(kScratchBytes) +
                           " (use a smaller r, or gofmm_evaluate)");
  unsigned char* base = scratch_on(cur);
  float* ws = reinterpret_cast<float*>(base);
  int2* items = reinterpret_cast<int2*>(base + ws_bytes);
  const hipStream_t st = (hipStream_t)stream;
  if (it_bytes) HIP_OK(hipMemcpyAsync(items, f.items.data(), it_bytes, hipMemcpyHostToDevice, st));
  const EvalArgs e{r, W, ldw, U, ldu, st};
  for (int li = 0; li < nl; ++li) {
    const int cfg = (int)key[li + 1];
    const std::pair<int2*, int> fi{items + f.at[li].first, f.at[li].second};
    dev::KArgs a;
    int grid = 0;
    if (!make_args(c, li, cfg, e, a, grid, &fi, ws)) continue;
    hipLaunchKernelGGL(kernel_for(c, pl.launches[li], cfg, a.vec != 0), dim3(grid), dim3(kCfgs[cfg].nt), 0, st, a);
    HIP_OK(hipGetLastError());
  }
}

// Time every configuration of every segment for this r and keep the fastest.
// Two timing events, destroyed on every exit path.
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  EventPair() {
    HIP_OK(hipEventCreate(&a));
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      fail(GOFMM_EHIP, "hipEventCreate failed");
    }
  }
  ~EventPair() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
  EventPair(const EventPair&) = delete;
  EventPair& operator=(const EventPair&) = delete;
};

// A shape replaces the fastest one timed so far only if it is faster by 4%:
// timings within the noise (and within what a profiler's own overhead shifts)
// keep the earlier (simpler) shape, so the choice is stable from run to run.
constexpr float kTuneMargin = 0.96f;

void device_profile_read(Compression& c, int n, float* total_ms, int* calls);

// Tile shape per launch, timed in context: for each launch in turn and each
// shape, `reps` whole evaluates run with that launch on that shape and HIP
// events around that launch alone, so every shape is timed with the caches,
// the accumulation and the clock the launch meets inside an evaluate (a
// launch repeated on its own keeps its operands cached and, for short
// launches, measures something else).  Launches not yet tuned use the cost
// model's shape.  When that many evaluates would take more than
// kInContextBudgetMs (large problems, whose launches are long enough to time
// alone), and for the persistent tree passes (opt-in), each shape is timed by
// repeating the launch on its own.
constexpr double kInContextBudgetMs = 5000.0;

void device_autotune(Compression& c, i64 r, const float* W, i64 ldw, float* U, i64 ldu, void* stream,
                     int reps) {
  device_evaluate(c, r, W, ldw, U, ldu, stream);          // prepares and warms up
  hipStream_t st = (hipStream_t)stream;
  EventPair ev;
  hipEvent_t e0 = ev.a, e1 = ev.b;
  const EvalArgs e{r, W, ldw, U, ldu, st};
  float t_eval = 0.f;
  HIP_OK(hipEventRecord(e0, st));
  device_evaluate(c, r, W, ldw, U, ldu, stream);
  HIP_OK(hipEventRecord(e1, st));
  HIP_OK(hipEventSynchronize(e1));
  HIP_OK(hipEventElapsedTime(&t_eval, e0, e1));
  const bool in_context =
      (double)t_eval * (double)c.plan.launches.size() * kNumCfg * (reps + 1) <= kInContextBudgetMs;
  // the caller's profiling state is restored on every exit path
  struct ProfRestore {
    DeviceState* d;
    bool was;
    int only;
    ~ProfRestore() {
      d->profiling = was;
      d->prof_only = only;
    }
  } restore{c.dev, c.dev->profiling, c.dev->prof_only};
  c.dev->profiling = false;
  const int nl = (int)c.plan.launches.size();
  std::vector<float> ms(nl);
  std::vector<int> calls(nl);
  device_profile_read(c, nl, ms.data(), calls.data());   // drop earlier records
  for (const Seg& sg : segments(c.plan)) {
    float best = 1e30f;
    int bc = choose_cfg(c, sg.j0, r);
    for (int q = 0; q < kNumCfg; ++q) {
      float t = 0.f;
      if (sg.pass || !in_context) {
        launch_seg(c, sg, q, e, true);
        HIP_OK(hipEventRecord(e0, st));
        for (int k = 0; k < reps; ++k) launch_seg(c, sg, q, e, true);
        HIP_OK(hipEventRecord(e1, st));
        HIP_OK(hipEventSynchronize(e1));
        HIP_OK(hipEventElapsedTime(&t, e0, e1));
        t /= reps;
      } else {
        c.dev->tuned[{sg.j0, r}] = q;
        device_evaluate(c, r, W, ldw, U, ldu, stream);  // item lists for this shape, warm
        c.dev->profiling = true;
        c.dev->prof_only = sg.j0;
        for (int k = 0; k < reps; ++k) device_evaluate(c, r, W, ldw, U, ldu, stream);
        c.dev->profiling = false;
        device_profile_read(c, nl, ms.data(), calls.data());
        t = ms[sg.j0] / std::max(1, calls[sg.j0]);
      }
      if (t < kTuneMargin * best) { best = t; bc = q; }
      if (std::getenv("GOFMM_TUNE_LOG"))
        std::fprintf(stderr, "tune %s%s r=%lld cfg %dx%dx%d: %.4f ms\n", c.plan.launches[sg.j0].name.c_str(),
                     sg.pass ? " (pass)" : "", (long long)r, kCfgs[q].bm, kCfgs[q].bn, kCfgs[q].nt, t);
    }
    c.dev->tuned[{sg.pass ? -(sg.j0 + 1) : sg.j0, r}] = bc;
  }
  // timing runs on their own overwrote intermediate rows: a clean result
  device_evaluate(c, r, W, ldw, U, ldu, stream);
}

// Error flags of the compression's persistent passes (1 if a dependency wait
// hit its poll bound since the last call); waits for the device.
int device_pass_status(Compression& c) {
  if (!c.dev) return 0;
  HIP_OK(hipDeviceSynchronize());
  int any = 0;
  for (auto& kv : c.dev->passes) {
    int f = 0;
    HIP_OK(hipMemcpy(&f, kv.second.error, sizeof(int), hipMemcpyDeviceToHost));
    if (f) {
      any = 1;
      HIP_OK(hipMemset(kv.second.error, 0, sizeof(int)));
    }
  }
  return any;
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
  if (c.geo.kind >= 0) b += (i64)(pl.geo_cols.size() + c.geo.pts.size()) * 4;
  b += std::max<i64>(1, pl.ws_rows) * ws_cols_for(r_max) * 4;
  // work-item lists: one entry per 32 rows x 32 columns of every task, plus XCD padding
  i64 entries = 0;
  for (const auto& t : pl.tasks) entries += (t.m + 31) / 32;
  b += (entries * ((r_max + 31) / 32) + (i64)pl.launches.size() * kXcds) * 8;
  return b;
}

// ------------------------------------------------------------------ batched launch
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

static int batch_cfg_model(int k, Compression* const* c, const i64* r) {
  double best = 1e300;
  int bc = 0;
  for (int q = 0; q < kNumCfg; ++q) {
    const Cfg& g = kCfgs[q];
    double cost = 0.0;
    for (int i = 0; i < k; ++i) {
      const double nt = (double)((r[i] + g.bn - 1) / g.bn);
      for (const LaunchDesc& l : c[i]->plan.launches)
        for (i32 t = l.t_begin; t < l.t_end; ++t) {
          const TaskDesc& td = c[i]->plan.tasks[t];
          cost += (double)((td.m + g.bm - 1) / g.bm) * nt * tile_cost(g, l.prec, (double)std::max(td.lda, 32));
        }
    }
    if (cost < best) { best = cost; bc = q; }
  }
  return bc;
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
// memory, one async copy moves them (with zeroed counters) to the device, the
// kernel runs, and the error flag is copied back to pinned memory.
void ring_launch(BatchRing& ring, int k, Compression* const* c, const i64* r, const float* const* W,
                 const i64* ldw, float* const* U, const i64* ldu, hipStream_t st, int cfg) {
  const int prec = batch_prec(k, c);
  std::vector<dev::BItem> items;
  std::vector<int> acc, tot;
  std::vector<int> j0(k, 0), j1(k);
  for (int i = 0; i < k; ++i) j1[i] = (int)c[i]->plan.launches.size();
  build_pass_tables(k, c, r, j0.data(), j1.data(), cfg, items, acc, tot);
  const int ns = (int)acc.size(), nc = (int)tot.size();
  const size_t o_cnt = 0, n_cnt = (size_t)(nc + 1) * sizeof(unsigned long long);
  const size_t o_tab = align256(o_cnt + n_cnt), n_tab = (size_t)(ns + nc) * sizeof(int);
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
  for (int q = 0; q < ns; ++q) tab[q] = acc[q];
  for (int q = 0; q < nc; ++q) tab[ns + q] = tot[q];
  dev::BInst* in = reinterpret_cast<dev::BInst*>(h + o_inst);
  bool all_vec = true;
  for (int i = 0; i < k; ++i) {
    in[i] = make_inst(*c[i], prec, r[i], W[i], ldw[i], U[i], ldu[i]);
    all_vec = all_vec && in[i].vec;
  }
  if (n_item) std::memcpy(h + o_item, items.data(), n_item);
  *reinterpret_cast<int*>(h + o_err) = 0;
  HIP_OK(hipMemcpyAsync(s.dev, h, o_err + sizeof(int), hipMemcpyHostToDevice, st));
  if (!items.empty()) {
    dev::BArgs a;
    char* dv = s.dev;
    a.inst = reinterpret_cast<const dev::BInst*>(dv + o_inst);
    a.one = in[0];
    a.items = reinterpret_cast<const dev::BItem*>(dv + o_item);
    a.n_items = (int)items.size();
    a.stage_acc = reinterpret_cast<const int*>(dv + o_tab);
    a.ctr_total = a.stage_acc + ns;
    a.ctr = reinterpret_cast<unsigned long long*>(dv + o_cnt);
    a.head = a.ctr + nc;
    a.head_base = 0;
    a.epoch = 0;
    a.error = reinterpret_cast<int*>(dv + o_err);
    a.spin_limit = spin_limit_ref();
    const int grid = std::max(1, std::min(a.n_items, persistent_cap(prec, cfg, 0)));
    hipLaunchKernelGGL(tables().b[all_vec ? 1 : 0][prec][cfg * 2], dim3(grid), dim3(kCfgs[cfg].nt), 0, st, a);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(h + o_err, dv + o_err, sizeof(int), hipMemcpyDeviceToHost, st));
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
    if (c[i]->geo.kind >= 0) fail(GOFMM_EINVAL, "compressions with device-computed near blocks are evaluated one at a time");
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
    EventPair ev;
    hipEvent_t e0 = ev.a, e1 = ev.b;
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
        std::fprintf(stderr, "tune batched k=%d cfg %dx%dx%d: %.4f ms\n", k, kCfgs[q].bm, kCfgs[q].bn, kCfgs[q].nt, ms / reps);
      if (ms < kTuneMargin * best) { best = ms; bc = q; }
    }
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
