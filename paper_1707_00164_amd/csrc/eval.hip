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
// Accumulation is FP32 in the matrix-core accumulators.  Block ids are
// remapped so that consecutive tiles (same A rows, neighbouring columns) run
// on the same XCD and share its L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "internal.hpp"

namespace gofmm {

// ------------------------------------------------------------------ device code
namespace dev {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int BK = 32;
constexpr int NT = 256;

struct KArgs {
  const TaskDesc* tasks;
  const int2* tiles;    // (task, m-tile) entries
  int total;            // entries * ntn work items
  int ntn;              // column tiles
  const void* A;
  long long plane;      // offset of the lo plane (split BF16)
  const int* rows;
  const float* W;
  long long ldw;
  float* U;
  long long ldu;
  float* WS;
  long long ldws;
  int r;
  int vec;              // rows of W, U, WS are 16-byte aligned
};

__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned int u = __builtin_bit_cast(unsigned int, f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_val(unsigned short h) {
  return __builtin_bit_cast(float, (unsigned int)h << 16);
}

template <int PREC, int BM, int BN, int WM, int WN, bool ACC>
__global__ __launch_bounds__(NT) void gemm_tiles(KArgs a) {
  constexpr int WTM = BM / WM, WTN = BN / WN, TM = WTM / 32, TN = WTN / 32;
  static_assert(WM * WN == 4 && TM >= 1 && TN >= 1, "tile shape");
  constexpr bool F32 = PREC == PREC_F32;
  constexpr bool X3 = PREC == PREC_BF16X3;
  constexpr int NPL = X3 ? 2 : 1;                    // planes per operand
  constexpr int LDK = F32 ? BK + 4 : BK + 8;         // LDS row stride (elements)
  using E = typename std::conditional<F32, float, unsigned short>::type;
  __shared__ __attribute__((aligned(16))) E sA[NPL * BM * LDK];
  __shared__ __attribute__((aligned(16))) E sB[NPL * BN * LDK];
  __shared__ int sOut[BM];

  const int G = gridDim.x;                           // a multiple of 8
  const int lid = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  if (lid >= a.total) return;
  const int2 tl = a.tiles[lid / a.ntn];
  const int n0 = (lid % a.ntn) * BN;
  const TaskDesc td = a.tasks[tl.x];
  const int m0 = tl.y * BM;
  const int tid = threadIdx.x;
  const int* codes = a.rows + td.idx_off;
  for (int i = tid; i < BM; i += NT) sOut[i] = (m0 + i < td.m) ? codes[td.lda + m0 + i] : ROW_ZERO;

  constexpr int EPU = F32 ? 4 : 8;                   // A elements per 16-byte unit
  constexpr int AU = BM * BK / EPU, AUT = (AU + NT - 1) / NT;
  constexpr int BU = BK * BN / 4, BUT = (BU + NT - 1) / NT;
  uint4 ra[NPL][AUT];
  f32x4 rb[BUT];
  const E* Ab = reinterpret_cast<const E*>(a.A);

  auto gload = [&](int k0) {
#pragma unroll
    for (int t = 0; t < AUT; ++t) {
      const int u = tid + t * NT;
      if (u < AU) {
        const int row = u / (BK / EPU), c = u % (BK / EPU);
        if (m0 + row < td.m) {
          const long long off = td.a_off + (long long)(m0 + row) * td.lda + k0 + c * EPU;
          ra[0][t] = *reinterpret_cast<const uint4*>(Ab + off);
          if constexpr (X3) ra[NPL - 1][t] = *reinterpret_cast<const uint4*>(Ab + a.plane + off);
        } else {
#pragma unroll
          for (int p = 0; p < NPL; ++p) ra[p][t] = make_uint4(0, 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < BUT; ++t) {
      const int u = tid + t * NT;
      if (u < BU) {
        const int krow = u / (BN / 4), c4 = u % (BN / 4);
        const int code = codes[k0 + krow];
        const int col = n0 + 4 * c4;
        f32x4 v = {0.f, 0.f, 0.f, 0.f};
        if (code != ROW_ZERO) {
          const float* p = code >= 0 ? a.W + (long long)code * a.ldw
                                     : a.WS + (long long)(-(code + 1)) * a.ldws;
          if (a.vec && col + 3 < a.r) {
            v = *reinterpret_cast<const f32x4*>(p + col);
          } else {
            if (col < a.r) v[0] = p[col];
            if (col + 1 < a.r) v[1] = p[col + 1];
            if (col + 2 < a.r) v[2] = p[col + 2];
            if (col + 3 < a.r) v[3] = p[col + 3];
          }
        }
        rb[t] = v;
      }
    }
  };

  auto lstore = [&]() {
#pragma unroll
    for (int t = 0; t < AUT; ++t) {
      const int u = tid + t * NT;
      if (u < AU) {
        const int row = u / (BK / EPU), c = u % (BK / EPU);
#pragma unroll
        for (int p = 0; p < NPL; ++p)
          *reinterpret_cast<uint4*>(&sA[p * BM * LDK + row * LDK + c * EPU]) = ra[p][t];
      }
    }
#pragma unroll
    for (int t = 0; t < BUT; ++t) {
      const int u = tid + t * NT;
      if (u < BU) {
        const int krow = u / (BN / 4), c4 = u % (BN / 4);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int idx = (4 * c4 + e) * LDK + krow;
          if constexpr (F32) {
            sB[idx] = rb[t][e];
          } else {
            const unsigned short hi = bf16_rne(rb[t][e]);
            sB[idx] = hi;
            if constexpr (X3) sB[BN * LDK + idx] = bf16_rne(rb[t][e] - bf16_val(hi));
          }
        }
      }
    }
  };

  const int lane = tid & 63, li = lane & 31, lh = lane >> 5;
  const int wid = tid >> 6, wr = wid / WN, wc = wid % WN;
  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  auto compute = [&]() {
    if constexpr (F32) {
      // lane (li, lh) feeds k = lh * 16 + 4u + q: the two halves of the wave
      // cover k 0..15 and 16..31 of the slab, matching A and B.
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        f32x4 av[TM], bv[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
          av[i] = *reinterpret_cast<const f32x4*>(&sA[(wr * WTM + i * 32 + li) * LDK + lh * 16 + 4 * u]);
#pragma unroll
        for (int j = 0; j < TN; ++j)
          bv[j] = *reinterpret_cast<const f32x4*>(&sB[(wc * WTN + j * 32 + li) * LDK + lh * 16 + 4 * u]);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i][q], bv[j][q], acc[i][j], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        bf16x8 ah[TM], bh[TN], al[TM], bl[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          const int o = (wr * WTM + i * 32 + li) * LDK + 16 * s + 8 * lh;
          ah[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&sA[o]));
          if constexpr (X3) al[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&sA[BM * LDK + o]));
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int o = (wc * WTN + j * 32 + li) * LDK + 16 * s + 8 * lh;
          bh[j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&sB[o]));
          if constexpr (X3) bl[j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&sB[BN * LDK + o]));
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            if constexpr (X3) {
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
            }
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
          }
      }
    }
  };

  const int nk = td.lda / BK;
  if (nk > 0) gload(0);
  for (int kt = 0; kt < nk; ++kt) {
    __syncthreads();
    lstore();
    __syncthreads();
    if (kt + 1 < nk) gload((kt + 1) * BK);
    compute();
  }
  __syncthreads();

  // epilogue: accumulator (i, j, v) of lane (li, lh) is row 8(v/4) + 4 lh + v%4,
  // column li of the 32 x 32 block
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int row = wr * WTM + i * 32 + (v >> 2) * 8 + lh * 4 + (v & 3);
      if (m0 + row >= td.m) continue;
      const int code = sOut[row];
      float* p = code >= 0 ? a.U + (long long)code * a.ldu : a.WS + (long long)(-(code + 1)) * a.ldws;
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int col = n0 + wc * WTN + j * 32 + li;
        if (col < a.r) {
          if constexpr (ACC) p[col] += acc[i][j][v];
          else p[col] = acc[i][j][v];
        }
      }
    }
}

}  // namespace dev

// ------------------------------------------------------------------ configurations
struct Cfg { int bm, bn; };
static const Cfg kCfgs[] = {{128, 128}, {128, 64}, {64, 128}, {64, 64}, {128, 32}, {32, 128}};
constexpr int kNumCfg = sizeof(kCfgs) / sizeof(kCfgs[0]);

typedef void (*KernelFn)(dev::KArgs);

template <int PREC, bool ACC>
static KernelFn pick(int cfg) {
  switch (cfg) {
    case 0: return dev::gemm_tiles<PREC, 128, 128, 2, 2, ACC>;
    case 1: return dev::gemm_tiles<PREC, 128, 64, 2, 2, ACC>;
    case 2: return dev::gemm_tiles<PREC, 64, 128, 2, 2, ACC>;
    case 3: return dev::gemm_tiles<PREC, 64, 64, 2, 2, ACC>;
    case 4: return dev::gemm_tiles<PREC, 128, 32, 4, 1, ACC>;
    default: return dev::gemm_tiles<PREC, 32, 128, 1, 4, ACC>;
  }
}

static KernelFn kernel_for(int prec, bool acc, int cfg) {
  if (prec == PREC_F32) return acc ? pick<PREC_F32, true>(cfg) : pick<PREC_F32, false>(cfg);
  if (prec == PREC_BF16) return acc ? pick<PREC_BF16, true>(cfg) : pick<PREC_BF16, false>(cfg);
  return acc ? pick<PREC_BF16X3, true>(cfg) : pick<PREC_BF16X3, false>(cfg);
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
  std::map<int, std::pair<int2*, int>> tiles;   // key launch * 256 + bm
  std::map<long long, int> tuned;   // (launch, r) -> configuration
  i64 op_bytes = 0;
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
  for (auto& kv : d->tiles) (void)hipFree(kv.second.first);
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

static std::pair<int2*, int> tiles_for(Compression& c, int li, int bm) {
  DeviceState* d = c.dev;
  const int key = li * 256 + bm;
  auto it = d->tiles.find(key);
  if (it != d->tiles.end()) return it->second;
  const LaunchDesc& l = c.plan.launches[li];
  std::vector<int2> t;
  for (i32 k = l.t_begin; k < l.t_end; ++k)
    for (int mt = 0; mt * bm < c.plan.tasks[k].m; ++mt) t.push_back(make_int2(k, mt));
  int2* dp = nullptr;
  if (!t.empty()) {
    HIP_OK(hipMalloc((void**)&dp, t.size() * sizeof(int2)));
    HIP_OK(hipMemcpy(dp, t.data(), t.size() * sizeof(int2), hipMemcpyHostToDevice));
  }
  d->tiles[key] = {dp, (int)t.size()};
  return d->tiles[key];
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
    // fewer work items than compute units leaves the chip idle
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

static void launch_all(Compression& c, const EvalArgs& e, int forced_cfg) {
  DeviceState* d = c.dev;
  const i64 ldws = ws_cols_for(e.r);
  const bool vec = ((uintptr_t)e.W % 16 == 0) && ((uintptr_t)e.U % 16 == 0) && e.ldw % 4 == 0 &&
                   e.ldu % 4 == 0;
  for (int li = 0; li < (int)c.plan.launches.size(); ++li) {
    const LaunchDesc& l = c.plan.launches[li];
    int cfg = forced_cfg;
    if (cfg < 0) {
      auto it = d->tuned.find((long long)li * (1ll << 32) + e.r);
      cfg = it != d->tuned.end() ? it->second : choose_cfg(c, li, e.r);
    }
    const Cfg& g = kCfgs[cfg];
    auto tl = tiles_for(c, li, g.bm);
    if (tl.second == 0) continue;
    dev::KArgs a;
    a.tasks = d->tasks;
    a.tiles = tl.first;
    a.ntn = (int)((e.r + g.bn - 1) / g.bn);
    a.total = tl.second * a.ntn;
    a.A = l.prec == PREC_F32 ? (const void*)d->a_f32 : l.prec == PREC_BF16 ? (const void*)d->a_b16 : (const void*)d->a_x3;
    a.plane = d->x3_plane;
    a.rows = d->rows;
    a.W = e.W;
    a.ldw = e.ldw;
    a.U = e.U;
    a.ldu = e.ldu;
    a.WS = d->ws;
    a.ldws = ldws;
    a.r = (int)e.r;
    a.vec = vec ? 1 : 0;
    const int grid = (a.total + 7) / 8 * 8;
    hipLaunchKernelGGL(kernel_for(l.prec, l.accumulate != 0, cfg), dim3(grid), dim3(dev::NT), 0, e.stream, a);
    HIP_OK(hipGetLastError());
  }
}

void device_evaluate(Compression& c, i64 r, const float* W, i64 ldw, float* U, i64 ldu, void* stream) {
  if (!c.dev || ws_cols_for(r) > c.dev->ws_cols) device_prepare(c, r);
  int cur;
  HIP_OK(hipGetDevice(&cur));
  if (c.dev->device != cur) fail(GOFMM_EINVAL, "current device differs from the compression's device");
  if (r > INT32_MAX / 2) fail(GOFMM_ELIMIT, "r too large");
  launch_all(c, EvalArgs{r, W, ldw, U, ldu, (hipStream_t)stream}, -1);
}

// Time every configuration of every launch for this r and keep the fastest.
void device_autotune(Compression& c, i64 r, const float* W, i64 ldw, float* U, i64 ldu, void* stream,
                     int reps) {
  device_evaluate(c, r, W, ldw, U, ldu, stream);          // prepares and warms up
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  DeviceState* d = c.dev;
  const i64 ldws = ws_cols_for(r);
  const bool vec = ((uintptr_t)W % 16 == 0) && ((uintptr_t)U % 16 == 0) && ldw % 4 == 0 && ldu % 4 == 0;
  for (int li = 0; li < (int)c.plan.launches.size(); ++li) {
    const LaunchDesc& l = c.plan.launches[li];
    float best = 1e30f;
    int bc = choose_cfg(c, li, r);
    for (int q = 0; q < kNumCfg; ++q) {
      const Cfg& g = kCfgs[q];
      auto tl = tiles_for(c, li, g.bm);
      if (tl.second == 0) continue;
      dev::KArgs a;
      a.tasks = d->tasks;
      a.tiles = tl.first;
      a.ntn = (int)((r + g.bn - 1) / g.bn);
      a.total = tl.second * a.ntn;
      a.A = l.prec == PREC_F32 ? (const void*)d->a_f32 : l.prec == PREC_BF16 ? (const void*)d->a_b16 : (const void*)d->a_x3;
      a.plane = d->x3_plane;
      a.rows = d->rows;
      a.W = W;
      a.ldw = ldw;
      a.U = U;
      a.ldu = ldu;
      a.WS = d->ws;
      a.ldws = ldws;
      a.r = (int)r;
      a.vec = vec ? 1 : 0;
      const int grid = (a.total + 7) / 8 * 8;
      // accumulate-mode launches would change U; time them in overwrite mode
      KernelFn fn = kernel_for(l.prec, false, q);
      hipLaunchKernelGGL(fn, dim3(grid), dim3(dev::NT), 0, st, a);
      HIP_OK(hipEventRecord(e0, st));
      for (int t = 0; t < reps; ++t) hipLaunchKernelGGL(fn, dim3(grid), dim3(dev::NT), 0, st, a);
      HIP_OK(hipEventRecord(e1, st));
      HIP_OK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_OK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) { best = ms; bc = q; }
    }
    d->tuned[(long long)li * (1ll << 32) + r] = bc;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // the timing runs overwrote intermediate rows: recompute a clean result
  device_evaluate(c, r, W, ldw, U, ldu, stream);
}

i64 device_footprint(const Compression& c, i64 r_max) {
  const HostPlan& pl = c.plan;
  i64 b = (i64)(pl.a_f32.size() * 4 + pl.a_b16.size() * 2 + (pl.a_x3hi.size() + pl.a_x3lo.size()) * 2 +
                pl.tasks.size() * sizeof(TaskDesc) + pl.rows.size() * 4);
  b += std::max<i64>(1, pl.ws_rows) * ws_cols_for(r_max) * 4;
  // tile lists: at most one entry per 32 rows of every task, per configuration height
  i64 entries = 0;
  for (const auto& t : pl.tasks) entries += (t.m + 31) / 32;
  b += entries * 8 * 3;
  return b;
}

}  // namespace gofmm

namespace gofmm {
// Independent products, one after another on the stream (the persistent
// single-launch form replaces this).
void device_evaluate_batched(int k, Compression* const* c, const i64* r, const float* const* W,
                             const i64* ldw, float* const* U, const i64* ldu, void* stream) {
  for (int i = 0; i < k; ++i)
    if (r[i] > 0) device_evaluate(*c[i], r[i], W[i], ldw[i], U[i], ldu[i], stream);
}
}  // namespace gofmm
