// Device code of the gather-GEMM evaluator (included by one translation unit
// per precision, which instantiates the kernels).
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
// Accumulation is FP32 in the matrix-core accumulators.  Each block reads its
// work item (task, row tile, column tile) from a host-built list; the host
// orders the list so that the longest tiles start first and the column tiles
// of one A block run on the same XCD (sharing its L2).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.hpp"

namespace gofmm {
// ------------------------------------------------------------------ device code
namespace dev {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int BK = 32;
constexpr int NT = 256;

struct KArgs {
  const TaskDesc* tasks;
  const int2* items;    // per block: (task, m-tile << 16 | n-tile), task < 0 = idle
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

// Pointers into device memory as global-address-space pointers, so loads and
// stores use the global (not generic flat) instructions even when the pointer
// itself was read from memory (the batched launch).
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned int u = __builtin_bit_cast(unsigned int, f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_val(unsigned short h) {
  return __builtin_bit_cast(float, (unsigned int)h << 16);
}

// LDS of one block: A and B slabs (two planes each for split BF16) and the
// output row codes of the tile.
template <int PREC, int BM, int BN>
struct Smem {
  static constexpr bool F32 = PREC == PREC_F32;
  static constexpr int NPL = PREC == PREC_BF16X3 ? 2 : 1;
  static constexpr int LDK = F32 ? BK + 4 : BK + 8;  // row stride (elements)
  using E = typename std::conditional<F32, float, unsigned short>::type;
  __attribute__((aligned(16))) E sA[NPL * BM * LDK];
  __attribute__((aligned(16))) E sB[NPL * BN * LDK];
  int sOut[BM];
};

// One BM x BN output tile of task td (rows m0.., columns n0..); acc adds the
// product to the output instead of overwriting it.
template <int PREC, int BM, int BN, int WM, int WN>
__device__ __forceinline__ void tile_body(const KArgs& a, const TaskDesc& td, int m0, int n0, bool accumulate,
                                          Smem<PREC, BM, BN>& sm) {
  constexpr int WTM = BM / WM, WTN = BN / WN, TM = WTM / 32, TN = WTN / 32;
  static_assert(WM * WN == 4 && TM >= 1 && TN >= 1, "tile shape");
  constexpr bool F32 = PREC == PREC_F32;
  constexpr bool X3 = PREC == PREC_BF16X3;
  constexpr int NPL = X3 ? 2 : 1;                    // planes per operand
  constexpr int LDK = Smem<PREC, BM, BN>::LDK;
  using E = typename Smem<PREC, BM, BN>::E;
  E* sA = sm.sA;
  E* sB = sm.sB;
  int* sOut = sm.sOut;
  const int tid = threadIdx.x;
  const auto codes = gmem(a.rows + td.idx_off);
  for (int i = tid; i < BM; i += NT) sOut[i] = (m0 + i < td.m) ? codes[td.lda + m0 + i] : ROW_ZERO;

  constexpr int EPU = F32 ? 4 : 8;                   // A elements per 16-byte unit
  constexpr int AU = BM * BK / EPU, AUT = (AU + NT - 1) / NT;
  // B is loaded in sub-blocks of KS rows x 4 columns and transposed in
  // registers, so that LDS receives k-contiguous 16-byte vectors per column.
  constexpr int KS = 4;
  constexpr int BSUB = (BK / KS) * (BN / 4), BST = (BSUB + NT - 1) / NT;
  u32x4 ra[NPL][AUT];
  f32x4 rb[BST][KS];
  const auto Ab = gmem(reinterpret_cast<const E*>(a.A));
  // Row codes of B are fetched one slab ahead of the B rows they address, so
  // that the address of a B load never waits on a code load.
  int nc[BST][KS];
  auto cload = [&](int k0) {
#pragma unroll
    for (int t = 0; t < BST; ++t) {
      const int sub = tid + t * NT;
      const int kq = sub / (BN / 4);
#pragma unroll
      for (int e = 0; e < KS; ++e)
        nc[t][e] = (sub < BSUB && k0 < td.lda) ? codes[k0 + kq * KS + e] : ROW_ZERO;
    }
  };

  auto gload = [&](int k0) {
#pragma unroll
    for (int t = 0; t < AUT; ++t) {
      const int u = tid + t * NT;
      if (u < AU) {
        const int row = u / (BK / EPU), c = u % (BK / EPU);
        if (m0 + row < td.m) {
          const long long off = td.a_off + (long long)(m0 + row) * td.lda + k0 + c * EPU;
          ra[0][t] = *(const __attribute__((address_space(1))) u32x4*)(Ab + off);
          if constexpr (X3) ra[NPL - 1][t] = *(const __attribute__((address_space(1))) u32x4*)(Ab + a.plane + off);
        } else {
#pragma unroll
          for (int p = 0; p < NPL; ++p) ra[p][t] = u32x4{0u, 0u, 0u, 0u};
        }
      }
    }
#pragma unroll
    for (int t = 0; t < BST; ++t) {
      const int sub = tid + t * NT;
      if (sub < BSUB) {
        const int cq = sub % (BN / 4), kq = sub / (BN / 4);
        const int col = n0 + 4 * cq;
#pragma unroll
        for (int e = 0; e < KS; ++e) {
          const int code = nc[t][e];
          f32x4 v = {0.f, 0.f, 0.f, 0.f};
          if (code != ROW_ZERO) {
            const auto p = gmem(code >= 0 ? a.W + (long long)code * a.ldw
                                          : a.WS + (long long)(-(code + 1)) * a.ldws);
            if (a.vec && col + 3 < a.r) {
              v = *(const __attribute__((address_space(1))) f32x4*)(p + col);
            } else {
              if (col < a.r) v[0] = p[col];
              if (col + 1 < a.r) v[1] = p[col + 1];
              if (col + 2 < a.r) v[2] = p[col + 2];
              if (col + 3 < a.r) v[3] = p[col + 3];
            }
          }
          rb[t][e] = v;
        }
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
          *reinterpret_cast<u32x4*>(&sA[p * BM * LDK + row * LDK + c * EPU]) = ra[p][t];
      }
    }
#pragma unroll
    for (int t = 0; t < BST; ++t) {
      const int sub = tid + t * NT;
      if (sub < BSUB) {
        const int cq = sub % (BN / 4), kq = sub / (BN / 4);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int idx = (4 * cq + j) * LDK + kq * KS;
          if constexpr (F32) {
            f32x4 v = {rb[t][0][j], rb[t][1][j], rb[t][2][j], rb[t][3][j]};
            *reinterpret_cast<f32x4*>(&sB[idx]) = v;
          } else {
            u16x4 hi, lo;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              hi[e] = bf16_rne(rb[t][e][j]);
              if constexpr (X3) lo[e] = bf16_rne(rb[t][e][j] - bf16_val(hi[e]));
            }
            *reinterpret_cast<u16x4*>(&sB[idx]) = hi;
            if constexpr (X3) *reinterpret_cast<u16x4*>(&sB[BN * LDK + idx]) = lo;
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
  if (nk > 0) {
    cload(0);
    gload(0);
    cload(BK);
  }
  for (int kt = 0; kt < nk; ++kt) {
    __syncthreads();
    lstore();
    __syncthreads();
    if (kt + 1 < nk) {
      gload((kt + 1) * BK);
      cload((kt + 2) * BK);
    }
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
      const auto p = gmem(code >= 0 ? a.U + (long long)code * a.ldu : a.WS + (long long)(-(code + 1)) * a.ldws);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int col = n0 + wc * WTN + j * 32 + li;
        if (col < a.r) {
          if (accumulate) p[col] += acc[i][j][v];
          else p[col] = acc[i][j][v];
        }
      }
    }
}

template <int PREC, int BM, int BN, int WM, int WN, bool ACC>
__device__ __forceinline__ void gemm_tiles(const KArgs& a) {
  __shared__ Smem<PREC, BM, BN> sm;
  const int2 it = a.items[blockIdx.x];
  if (it.x < 0) return;
  const TaskDesc td = a.tasks[it.x];
  tile_body<PREC, BM, BN, WM, WN>(a, td, (it.y >> 16) * BM, (it.y & 0xffff) * BN, ACC, sm);
}


// Entry points with the same body, so that profiles separate the upward pass,
// the far field, the downward pass and the leaf output.
template <int PREC, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(NT) void n2s_tiles(KArgs a) { gemm_tiles<PREC, BM, BN, WM, WN, false>(a); }
template <int PREC, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(NT) void s2s_tiles(KArgs a) { gemm_tiles<PREC, BM, BN, WM, WN, false>(a); }
template <int PREC, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(NT) void s2n_tiles(KArgs a) { gemm_tiles<PREC, BM, BN, WM, WN, true>(a); }
template <int PREC, int BM, int BN, int WM, int WN, bool ACC>
__global__ __launch_bounds__(NT) void leaf_tiles(KArgs a) { gemm_tiles<PREC, BM, BN, WM, WN, ACC>(a); }

typedef void (*KernelFn)(KArgs);

// ------------------------------------------------------------ batched launch
// Many compressions in one persistent launch.  Every (instance, step) pair is
// a stage; stages of one instance run in their evaluation order and stages of
// different instances are independent.  Work items (tiles) sit in one global
// queue in stage-major order; each resident block takes the next item, waits
// until the item's predecessor stage has finished all its tiles, runs the
// tile, and counts it as done.  Every item's predecessors precede it in the
// queue and are held by running blocks, so the waits always end; a spin limit
// still bounds each wait (the block then flags an error and skips the tile).
struct BInst {
  const TaskDesc* tasks;
  const int* rows;
  const void* A;
  long long plane;
  const float* W;
  long long ldw;
  float* U;
  long long ldu;
  float* WS;
  long long ldws;
  int r;
  int vec;
};

struct BItem { int inst, stage, task, tile; };   // tile = row tile << 16 | column tile

struct BArgs {
  const BInst* inst;
  const BItem* items;
  int n_items;
  const int* stage_prev;    // predecessor stage or -1
  const int* stage_need;    // tiles of the predecessor stage
  const int* stage_acc;     // 1: the stage accumulates into its output
  int* done;                // per stage: finished tiles (zero at launch)
  int* head;                // queue head (zero at launch)
  int* error;               // set to 1 if a wait exceeded the spin limit
  long long spin_limit;
};

template <int PREC, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(NT) void batched_tiles(BArgs b) {
  __shared__ Smem<PREC, BM, BN> sm;
  __shared__ int s_item;
  __shared__ int s_ok;
  // Lane 0's bookkeeping (publish the previous tile, take the next item, wait
  // for the item's predecessor stage) sits at the top of the iteration, each
  // part closed by a barrier, and the values it broadcasts are made
  // wave-uniform with readfirstlane: the loop's exit and back edge are then
  // uniform branches, so the compiler cannot split lane 0 from its wave.
  int last_stage = -1;
  while (true) {
    if (threadIdx.x == 0) {
      if (last_stage >= 0)
        __hip_atomic_fetch_add(&b.done[last_stage], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      s_item = atomicAdd(b.head, 1);
    }
    __syncthreads();
    const int idx = __builtin_amdgcn_readfirstlane(s_item);
    if (idx >= b.n_items) break;
    const BItem it = b.items[idx];
    const int stage = __builtin_amdgcn_readfirstlane(it.stage);
    if (threadIdx.x == 0) {
      int ok = 1;
      const int prev = b.stage_prev[stage];
      if (prev >= 0) {
        // Poll with relaxed loads (an acquire on every poll would invalidate
        // the L2 each time and starve the blocks doing the work), then one
        // acquire fence once the predecessor stage is complete.
        const int need = b.stage_need[stage];
        long long polls = 0;
        while (__hip_atomic_load(&b.done[prev], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
          __builtin_amdgcn_s_sleep(8);
          if (++polls > b.spin_limit) {
            atomicExch(b.error, 1);
            ok = 0;
            break;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      s_ok = ok;
    }
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(s_ok)) {
      const BInst& in = b.inst[__builtin_amdgcn_readfirstlane(it.inst)];
      KArgs a;
      a.tasks = in.tasks;
      a.items = nullptr;
      a.A = in.A;
      a.plane = in.plane;
      a.rows = in.rows;
      a.W = in.W;
      a.ldw = in.ldw;
      a.U = in.U;
      a.ldu = in.ldu;
      a.WS = in.WS;
      a.ldws = in.ldws;
      a.r = in.r;
      a.vec = in.vec;
      const TaskDesc td = in.tasks[__builtin_amdgcn_readfirstlane(it.task)];
      const int tile = __builtin_amdgcn_readfirstlane(it.tile);
      const int m0 = (tile >> 16) * BM, n0 = (tile & 0xffff) * BN;
      tile_body<PREC, BM, BN, WM, WN>(a, td, m0, n0, b.stage_acc[stage] != 0, sm);
    }
    last_stage = stage;
    __syncthreads();                      // every thread's stores issued, LDS free
  }
}

typedef void (*BatchedFn)(BArgs);
constexpr int kNumCfg = 8;
constexpr int kNumFamily = 5;   // n2s, s2s, s2n (accumulate), leaf, leaf accumulating
struct Cfg { int bm, bn; };
constexpr Cfg kCfgs[kNumCfg] = {{128, 128}, {128, 64}, {64, 128}, {64, 64},
                                {128, 32}, {32, 128}, {256, 128}, {128, 256}};

template <int PREC, int BM, int BN, int WM, int WN>
void fill_family(KernelFn* row, BatchedFn* brow) {
  *brow = batched_tiles<PREC, BM, BN, WM, WN>;
  row[0] = n2s_tiles<PREC, BM, BN, WM, WN>;
  row[1] = s2s_tiles<PREC, BM, BN, WM, WN>;
  row[2] = s2n_tiles<PREC, BM, BN, WM, WN>;
  row[3] = leaf_tiles<PREC, BM, BN, WM, WN, false>;
  row[4] = leaf_tiles<PREC, BM, BN, WM, WN, true>;
}

// table[cfg * kNumFamily + family], batched[cfg]
template <int PREC>
void fill_table(KernelFn* table, BatchedFn* batched) {
  fill_family<PREC, 128, 128, 2, 2>(table + 0 * kNumFamily, batched + 0);
  fill_family<PREC, 128, 64, 2, 2>(table + 1 * kNumFamily, batched + 1);
  fill_family<PREC, 64, 128, 2, 2>(table + 2 * kNumFamily, batched + 2);
  fill_family<PREC, 64, 64, 2, 2>(table + 3 * kNumFamily, batched + 3);
  fill_family<PREC, 128, 32, 4, 1>(table + 4 * kNumFamily, batched + 4);
  fill_family<PREC, 32, 128, 1, 4>(table + 5 * kNumFamily, batched + 5);
  fill_family<PREC, 256, 128, 2, 2>(table + 6 * kNumFamily, batched + 6);
  fill_family<PREC, 128, 256, 2, 2>(table + 7 * kNumFamily, batched + 7);
}

void kernels_f32(KernelFn* table, BatchedFn* batched);
void kernels_bf16(KernelFn* table, BatchedFn* batched);
void kernels_x3(KernelFn* table, BatchedFn* batched);

}  // namespace dev
}  // namespace gofmm
