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
// folded into the codes).  Work item = one BM x BN output tile.  FP32: the k
// loop stages a BM x 32 slab of A and a 32 x BN slab of B through LDS (B is
// transposed on the way in so both operands are read k-contiguous), with the
// next slab's global loads in flight while the matrix cores work on the
// current one.  BF16 forms: A is stored in matrix-core fragment order and read
// by each wave straight into registers; only B goes through LDS, double
// buffered in slabs of 64.  Matrix-core instructions (64-wide waves, 4 waves
// per block):
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
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));


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
  int vec;              // rows of W, U, WS are 16-byte aligned and r % 4 == 0
  // near blocks computed from points (l2l_geo_tiles): point entries of
  // kGeoStride floats per index (original order), kernel scale, diagonal
  // shift, and whether the launch accumulates into U
  const float* gpts;
  float gh2inv, gshift;
  int gacc;
};

// Radial kernel of the geometric mode on a squared distance (GEO = 1 + kind):
// Gaussian exp(-d2 h2inv / 2) = 2^(-d2 h2inv log2(e) / 2), inverse
// multiquadric 1 / sqrt(1 + d2 h2inv), Laplacian-like 1 / (sqrt(d2) + 0.05),
// each with the hardware's base-2 exponential, reciprocal square root, square
// root and reciprocal (about 1 ulp each; the entry's relative error stays
// near 1e-6 for exponents down to -20).
template <int GEO>
__device__ __forceinline__ float geo_kernel(float d2, float h2inv) {
  if constexpr (GEO == 1) return __builtin_amdgcn_exp2f(d2 * (h2inv * -0.72134752044448170f));
  else if constexpr (GEO == 2) return __builtin_amdgcn_rsqf(1.0f + d2 * h2inv);
  else return __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(d2) + 0.05f);
}

// Pointers into device memory as global-address-space pointers, so loads and
// stores use the global (not generic flat) instructions even when the pointer
// itself was read from memory (the batched launch).
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}


// Scheduling groups for one k step: N matrix-core instructions, each followed
// by at most one LDS read, one LDS write, one global load and VAL vector
// instructions (groups the step cannot fill stay empty).
template <int N, int VAL>
struct Interleave {
  static __device__ __forceinline__ void run() {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x002, VAL, 0);
    Interleave<N - 1, VAL>::run();
  }
};
template <int VAL>
struct Interleave<0, VAL> {
  static __device__ __forceinline__ void run() {}
};
template <int N, int VAL>
__device__ __forceinline__ void interleave() { Interleave<N, VAL>::run(); }

// LDS of one block: B only, double-buffered, one k slab per buffer (32 FP32 or
// 64 BF16 values = 128 bytes per column).  Column c occupies 36 words (the
// slab and 4 words of padding); its 16-byte chunk q sits at chunk position
// q ^ ((c >> 4) & 3).  With this stride and swizzle both the fragment reads
// (16 consecutive columns, one chunk) and the transposing writes (columns 4
// apart, consecutive chunks) touch 16 distinct 4-bank groups.
template <int PREC, int BM, int BN>
struct Smem {
  static constexpr int NPL = PREC == PREC_BF16X3 ? 2 : 1;
  static constexpr int CW = 36;
  __attribute__((aligned(16))) unsigned int sB[2][NPL][BN * CW];
  int sOut[BM];
};

__device__ __forceinline__ int swz(int c, int q) { return c * 36 + 4 * (q ^ ((c >> 4) & 3)); }

// Sixteen zero bytes in device memory: B elements that read as zero (rows
// coded ROW_ZERO, columns past r) are loaded from here, so their loads need
// neither a branch nor a mask.
static __device__ __attribute__((aligned(16))) float g_zero16[4];

// One BM x BN output tile of task td (rows m0.., columns n0..); accumulate adds
// the product to the output instead of overwriting it.
//
// A is stored in matrix-core fragment order: chunks of 32 rows, one 16-byte
// vector per lane (FP32: 4 values at k = 16h + 4s + q of a 32-slab, h the
// half-wave, s the step; BF16: 8 values at k = 16s + 8h + e of a 64-slab).
// Every wave loads its A fragments straight from global memory into
// registers, one slab (four steps) ahead of use, with one coalesced 1 KiB load
// per chunk and plane.  B rows are gathered two slabs ahead into registers
// (their row codes three slabs ahead), transposed (and rounded or split to
// BF16) into the LDS buffer that is not being read while the matrix cores
// work on the current slab, and read back as fragments one step ahead: one
// barrier per slab.  The k loop has no branch but the loop itself, and a
// scheduling fence per step keeps each step's loads, conversions and LDS
// traffic interleaved with its own matrix-core work.
//
// Per step and (row block, column block): FP32 four v_mfma_f32_32x32x2_f32
// (the two half-waves feed k 16h + 4s + q, q = 0..3); BF16 one
// v_mfma_f32_32x32x16_bf16; split BF16 three (lo*hi, hi*lo, hi*hi).  The k
// order of the products is the same for every tile shape, so every shape
// gives the same bits.
// COH (persistent launches): the tile's B rows, its output rows and the rows
// it accumulates into are read and written with device-coherent accesses
// (they bypass the per-XCD L2 caches, which the XCDs do not keep coherent
// with each other), so a tile can consume rows that a tile on another XCD
// produced in the same launch without cache write-backs or invalidations.
// GEO > 0: A is not loaded but computed, A(i, k) = kernel(|x_i - x_k|^2) plus
// the shift where the two indices are equal, from the row's point (held in
// registers) and the column's point entry (staged through LDS, sg, one slab
// of 32 columns ahead like B); FP32 only.
template <int PREC, int BM, int BN, int WM, int WN, bool VEC, bool COH = false, int GEO = 0>
__device__ __forceinline__ void tile_body(const KArgs& a, const TaskDesc& td, int m0, int n0, bool accumulate,
                                          Smem<PREC, BM, BN>& sm, f32x4* sg = nullptr) {
  constexpr int WTM = BM / WM, WTN = BN / WN, TM = WTM / 32, TN = WTN / 32;
  constexpr int NT = WM * WN * 64;                   // threads per block (4 or 8 waves)
  static_assert((WM * WN == 4 || WM * WN == 8) && TM >= 1 && TN >= 1, "tile shape");
  constexpr bool F32 = PREC == PREC_F32;
  constexpr bool X3 = PREC == PREC_BF16X3;
  constexpr int NPL = X3 ? 2 : 1;                    // planes per operand
  constexpr int KSLAB = F32 ? 32 : 64;               // k per slab
  constexpr int NS = 4;                              // steps per slab
  constexpr int EPU = F32 ? 4 : 8;                   // A elements per 16-byte unit
  constexpr int SBR = F32 ? 4 : 8;                   // B rows per sub-block (one 16-byte LDS chunk)
  const int tid = threadIdx.x;
  const int lane = tid & 63, li = lane & 31, lh = lane >> 5;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  // 8 waves: waves w and w + 4 are placed on one SIMD, so they get
  // complementary halves of the rows and of the columns; a tile whose last
  // rows or columns are empty then leaves one busy wave on every SIMD
  int wr, wc;
  if constexpr (WM * WN == 8) {
    const int p = wid & 3, h = wid >> 2;
    if constexpr (WM == 8) {
      wr = h ? 7 - p : p;
      wc = 0;
    } else if constexpr (WM == 4) {
      wr = h ? 3 - (p & 1) : (p & 1);
      wc = h ? 1 - (p >> 1) : (p >> 1);
    } else {
      wr = h;
      wc = h ? 3 - p : p;
    }
  } else {
    wr = wid / WN;
    wc = wid % WN;
  }
  const auto codes = gmem(a.rows + td.idx_off);
  for (int i = tid; i < BM; i += NT) sm.sOut[i] = (m0 + i < td.m) ? codes[td.lda + m0 + i] : ROW_ZERO;

  // A: ring of one slab of fragments per row block and plane.  Row blocks past
  // the stored ones and steps past the end read chunk 0 of the block (always
  // present); those products reach only rows that are never stored, or are
  // never issued.
  const int kch = td.lda / (KSLAB / NS);              // chunks per row block
  const int nrb = (td.m + 31) >> 5;                   // row blocks stored
  const int rb0 = (m0 + wr * WTM) >> 5;
  const auto Ab = gmem(reinterpret_cast<const u32x4*>(a.A));
  const long long abase = td.a_off / EPU;            // in 16-byte units
  const long long aplane = a.plane / EPU;
  // Prefetch depth in slabs: the large 4-wave BF16 tiles (their slabs are
  // short next to memory latency) and the 8-wave FP32 tiles (whose second
  // slab of registers still fits two waves per SIMD, as one block per CU
  // already holds) keep two slabs of A and of B rows in flight; the others one.
  constexpr int DEP = ((!F32 && WM * WN == 4 && BM == 256 && BN == 128) || (F32 && WM * WN == 8 && GEO == 0)) ? 2 : 1;
  u32x4 ra[DEP * NS][NPL][TM];
  // (TMA: the row blocks the wave computes, a compile-time count)
  auto aload = [&](int slot, int g, auto tmac) {
    constexpr int TMA = decltype(tmac)::value;
    if constexpr (GEO != 0) return;
#pragma unroll
    for (int i = 0; i < TMA; ++i) {
      const bool ok = rb0 + i < nrb && g < kch;
      // the chunk's start is wave-uniform (a scalar address); lanes add their
      // own 16-byte offset
      const auto Ac = Ab + (abase + (ok ? ((long long)(rb0 + i) * kch + g) * 64 : 0));
      ra[slot][0][i] = Ac[lane];
      if constexpr (X3) ra[slot][1][i] = Ac[aplane + lane];
    }
  };

  // B: sub-blocks of SBR rows x 4 columns per thread and slab.  Codes of slabs
  // past the end are clamped to the last k of the block: the rows they fetch
  // only reach LDS buffers that are never read again.  With more threads than
  // sub-blocks, whole waves sit out the B staging.
  constexpr int BSUB = (KSLAB / SBR) * (BN / 4), BST = (BSUB + NT - 1) / NT;
  static_assert(BSUB % 64 == 0, "sub-blocks per wave");
  const bool bwave = BSUB >= NT || wid * 64 < BSUB;
  int nc[BST][SBR];
  f32x4 rbv[DEP][BST][SBR];
  auto cload = [&](int k0) {
#pragma unroll
    for (int t = 0; t < BST; ++t) {
      const int kq = (tid + t * NT) / (BN / 4);
#pragma unroll
      for (int e = 0; e < SBR; ++e) nc[t][e] = codes[min(k0 + kq * SBR + e, td.lda - 1)];
    }
  };
  const auto Wg = gmem(a.W);
  const auto WSg = gmem(a.WS);
  const auto Zg = gmem(static_cast<const float*>(g_zero16));
  // Every load is issued unconditionally; B elements that read as zero (rows
  // coded ROW_ZERO, columns past r) come from the zero bytes above.  Nothing
  // waits for a B load before the slab is stored to LDS a slab later, and the
  // k loop stays free of branches.
  // coh: the slab holds workspace rows (produced by other tiles of a
  // persistent launch), read with device-coherent loads; rows of W are
  // read-only during a launch and take the cached path
  auto bload = [&](bool coh, int set, int e0, int e1) {
    if (!bwave) return;
#pragma unroll
    for (int t = 0; t < BST; ++t) {
      const int sub = tid + t * NT;
      const int col = n0 + 4 * (sub % (BN / 4));
      const auto rowp = [&](int e, bool& zr) {
        const int code = nc[t][e];
        zr = code == ROW_ZERO;
        const bool inw = code >= 0;
        // row index and leading dimension both fit 32 bits (checked on the
        // host), so the offset is one 32 x 32 -> 64-bit multiply
        const unsigned int idx = inw ? (unsigned int)code : (unsigned int)(-(code + 1));
        const unsigned int ld = inw ? (unsigned int)a.ldw : (unsigned int)a.ldws;
        return (inw ? Wg : WSg) + (unsigned long long)idx * ld;
      };
      // (the row address is made opaque before the select, so the compiler
      // cannot move its computation into a branch)
      if constexpr (VEC) {                            // rows 16-byte aligned, r % 4 == 0
        const bool zc = col >= a.r;
#pragma unroll
        for (int e = e0; e < e1; ++e) {
          bool zr;
          unsigned long long pa = (unsigned long long)(rowp(e, zr) + col);
          asm volatile("" : "+v"(pa));
          const auto q = (zr || zc) ? Zg : (const __attribute__((address_space(1))) float*)pa;
          if (COH && coh) {
            typedef unsigned long long u64 __attribute__((address_space(1)));
            const unsigned long long lo = __hip_atomic_load((u64*)q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned long long hi = __hip_atomic_load((u64*)q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            rbv[set][t][e] = f32x4{__builtin_bit_cast(float, (unsigned int)lo), __builtin_bit_cast(float, (unsigned int)(lo >> 32)),
                                   __builtin_bit_cast(float, (unsigned int)hi), __builtin_bit_cast(float, (unsigned int)(hi >> 32))};
          } else {
            rbv[set][t][e] = *(const __attribute__((address_space(1))) f32x4*)q;
          }
        }
      } else {
#pragma unroll
        for (int e = e0; e < e1; ++e) {
          bool zr;
          unsigned long long pa = (unsigned long long)(rowp(e, zr) + col);
          asm volatile("" : "+v"(pa));
          const auto p = (const __attribute__((address_space(1))) float*)pa;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const auto x = (zr || col + q >= a.r) ? Zg : p + q;
            if (COH && coh)
              rbv[set][t][e][q] = __hip_atomic_load((__attribute__((address_space(1))) float*)x, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
            else
              rbv[set][t][e][q] = *x;
          }
        }
      }
    }
  };
  // columns j0 .. j1-1 of each thread's sub-blocks, from register set `set`
  auto bstore = [&](int buf, int j0, int j1, int set) {
#pragma unroll
    for (int t = 0; t < BST; ++t) {
      const int sub = tid + t * NT;
      if (BSUB % NT == 0 || sub < BSUB) {
        const int cq = sub % (BN / 4), kq = sub / (BN / 4);
#pragma unroll
        for (int j = j0; j < j1; ++j) {
          const int w = swz(4 * cq + j, kq);
          if constexpr (F32) {
            const f32x4 v = {rbv[set][t][0][j], rbv[set][t][1][j], rbv[set][t][2][j], rbv[set][t][3][j]};
            *reinterpret_cast<f32x4*>(&sm.sB[buf][0][w]) = v;
          } else {
            u32x4 hi, lo;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const f32x2 x = {rbv[set][t][2 * e][j], rbv[set][t][2 * e + 1][j]};
              const bf16x2 h = __builtin_convertvector(x, bf16x2);
              hi[e] = __builtin_bit_cast(unsigned int, h);
              if constexpr (X3) {
                const f32x2 r = x - __builtin_convertvector(h, f32x2);
                lo[e] = __builtin_bit_cast(unsigned int, __builtin_convertvector(r, bf16x2));
              }
            }
            *reinterpret_cast<u32x4*>(&sm.sB[buf][0][w]) = hi;
            if constexpr (X3) *reinterpret_cast<u32x4*>(&sm.sB[buf][NPL - 1][w]) = lo;
          }
        }
      }
    }
  };

  f32x16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  u32x4 bfr[2][NPL][TN];
  auto bread = [&](int slot, int buf, int s) {
    const int q = F32 ? 4 * lh + s : 2 * s + lh;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int w = swz(wc * WTN + j * 32 + li, q);
#pragma unroll
      for (int p = 0; p < NPL; ++p) bfr[slot][p][j] = *reinterpret_cast<const u32x4*>(&sm.sB[buf][p][w]);
    }
  };
  // geometric mode: the lane's row points (rows of its row blocks), and the
  // column entries of one slab per LDS buffer (32 entries of 3 chunks)
  constexpr int GCH = KSLAB * 3;
  [[maybe_unused]] f32x4 xr[GEO ? TM : 1][2];
  [[maybe_unused]] unsigned int ridx[GEO ? TM : 1];
  [[maybe_unused]] f32x4 gq = {0.f, 0.f, 0.f, 0.f};
  [[maybe_unused]] f32x4 gav[2][GEO ? TM : 1];
  auto gload = [&](int slab) {
    if constexpr (GEO != 0) {
      const auto Gc = gmem(reinterpret_cast<const f32x4*>(a.A));
      if (tid < GCH) gq = Gc[td.a_off / 4 + (long long)min(slab, td.lda / KSLAB - 1) * GCH + tid];
    }
  };
  auto gstore = [&](int buf) {
    if constexpr (GEO != 0) {
      if (tid < GCH) sg[buf * GCH + tid] = gq;
    }
  };
  // A values of step s: columns 16 h + 4 s + q of the slab in buffer buf
  auto gcomp = [&](int slot, int buf, int s) {
    if constexpr (GEO != 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int col = 16 * lh + 4 * s + q;
        const f32x4 c0 = sg[buf * GCH + 3 * col], c1 = sg[buf * GCH + 3 * col + 1];
        const unsigned int cidx = __builtin_bit_cast(u32x4, sg[buf * GCH + 3 * col + 2])[0];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          const f32x4 d0 = xr[i][0] - c0, d1 = xr[i][1] - c1;
          const float d2 = ((d0[0] * d0[0] + d0[1] * d0[1]) + (d0[2] * d0[2] + d0[3] * d0[3])) +
                           ((d1[0] * d1[0] + d1[1] * d1[1]) + (d1[2] * d1[2] + d1[3] * d1[3]));
          float v = geo_kernel<GEO>(d2, a.gh2inv);
          if (ridx[i] == cidx) v += a.gshift;
          gav[slot][i][q] = v;
        }
      }
    }
  };
  auto mfma_step = [&](int s, int bs, auto tmac) {
    constexpr int TMA = decltype(tmac)::value;
    if constexpr (F32) {
      // (whole vectors are reinterpreted before indexing: a bit cast of a
      // single vector element reads element 0 with this compiler)
      f32x4 av[TM], bv[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        if constexpr (GEO != 0) av[i] = gav[bs][i];
        else av[i] = __builtin_bit_cast(f32x4, ra[s][0][i]);
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) bv[j] = __builtin_bit_cast(f32x4, bfr[bs][0][j]);
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < TMA; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i][q], bv[j][q], acc[i][j], 0, 0, 0);
    } else {
      // product-major order: consecutive matrix-core instructions update
      // different accumulators, so none waits for the previous result (each
      // element still receives lo*hi, hi*lo, hi*hi in that order)
      constexpr int NPROD = X3 ? 3 : 1;
#pragma unroll
      for (int pr = 0; pr < NPROD; ++pr)
#pragma unroll
        for (int i = 0; i < TMA; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            const int pa = (X3 && pr == 0) ? NPL - 1 : 0;    // lo*hi, hi*lo, hi*hi
            const int pb = (X3 && pr == 1) ? NPL - 1 : 0;
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, ra[s][pa][i]),
                                                                __builtin_bit_cast(bf16x8, bfr[bs][pb][j]),
                                                                acc[i][j], 0, 0, 0);
          }
    }
  };

  const int ns = td.lda / KSLAB;                     // k is padded to whole slabs
  // slab j's A fragments sit in ring slots (j % DEP) * NS + step, its B rows
  // in register set j % DEP
  // In the 8-wave shapes (two waves per SIMD) a wave computes only its row
  // blocks that hold rows of the task: one whose rows all lie past the
  // task's m, or whose columns all lie past r, has no products to form (it
  // still stages its share of B and meets every barrier, but loads no A and
  // issues no matrix-core work), and one whose last row block lies past m
  // skips that block's A loads and products; either way its SIMD partner
  // gets the matrix cores the more.  (The 4-wave shapes keep one k loop: a
  // second copy costs them registers, and an idle wave there would only
  // leave its SIMD idle.)
  constexpr bool IDLE = WM * WN == 8;
  const int tma = !IDLE ? TM
                        : __builtin_amdgcn_readfirstlane(n0 + wc * WTN < a.r ? max(0, min(TM, nrb - rb0)) : 0);
  const bool act = tma > 0;
  if constexpr (GEO != 0) {
    static_assert(F32 && DEP == 1, "geometric mode is FP32");
    const auto Pp = gmem(reinterpret_cast<const f32x4*>(a.gpts));
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int row = m0 + wr * WTM + i * 32 + li;
      if (row < td.m) {
        const long long code = codes[td.lda + row];      // a row of U: an original index
        xr[i][0] = Pp[code * 3];
        xr[i][1] = Pp[code * 3 + 1];
        ridx[i] = __builtin_bit_cast(u32x4, Pp[code * 3 + 2])[0];
      } else {
        xr[i][0] = f32x4{0.f, 0.f, 0.f, 0.f};
        xr[i][1] = f32x4{0.f, 0.f, 0.f, 0.f};
        ridx[i] = 0xffffffffu;
      }
    }
  }
  if (ns > 0) {
    cload(0);
    bload(0 < td.kws, 0, 0, SBR);
    if constexpr (DEP == 2) {
      cload(KSLAB);
      bload(KSLAB < td.kws, 1, 0, SBR);
    }
    cload(DEP * KSLAB);
    if (act) {
#pragma unroll
      for (int s = 0; s < DEP * NS; ++s) aload(s, s, std::integral_constant<int, TM>());
    }
    bstore(0, 0, 4, 0);
    bload(DEP * KSLAB < td.kws, 0, 0, SBR);
    cload((DEP + 1) * KSLAB);
    gload(0);
    gstore(0);
    gload(1);
  }
  __syncthreads();
  auto iter = [&](int kt, auto setc, auto tmac) {
    constexpr int SET = decltype(setc)::value;       // kt % DEP
    constexpr int NXT = DEP == 2 ? 1 - SET : 0;      // register set of slabs kt + 1 and kt + 1 + DEP
    constexpr int TMA = decltype(tmac)::value;       // row blocks computed
    constexpr bool ACT = TMA > 0;
    const int buf = kt & 1;
    if constexpr (ACT) {
      bread(0, buf, 0);
      gcomp(0, buf, 0);
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if constexpr (ACT) {
        if (s + 1 < NS) {
          bread((s + 1) & 1, buf, s + 1);
          gcomp((s + 1) & 1, buf, s + 1);
        }
        mfma_step(SET * NS + s, s & 1, tmac);
        aload(SET * NS + s, (kt + DEP) * NS + s, tmac);
      }
      // slab kt + 1 into the other buffer (no wave reads it before the
      // barrier below), then the B rows of slab kt + 1 + DEP and the codes of
      // the slab after; past the last slab these move data that nobody reads
      if constexpr (F32) {
        if (s == 0) {
          bstore(buf ^ 1, 0, 2, NXT);
          gstore(buf ^ 1);
        }
        if (s == 1) {
          bstore(buf ^ 1, 2, 4, NXT);
          bload((kt + 1 + DEP) * KSLAB < td.kws, NXT, 0, SBR);
          cload((kt + 2 + DEP) * KSLAB);
          gload(kt + 2);
        }
      } else {
        // BF16 conversions and row addressing spread over all four steps
        if (s == 0) bstore(buf ^ 1, 0, 2, NXT);
        if (s == 1) bstore(buf ^ 1, 2, 4, NXT);
        if (s == 2) bload((kt + 1 + DEP) * KSLAB < td.kws, NXT, 0, SBR / 2);
        if (s == 3) {
          bload((kt + 1 + DEP) * KSLAB < td.kws, NXT, SBR / 2, SBR);
          cload((kt + 2 + DEP) * KSLAB);
        }
      }
      // one matrix-core instruction at a time, with the step's LDS traffic,
      // global loads and vector work placed in its shadow
      if constexpr (F32 && ACT) interleave<TMA * TN * 4, 12>();
      if constexpr (!F32 && ACT) interleave<(X3 ? 3 : 1) * TMA * TN, 8>();
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
  };
  auto kloop = [&](auto tmac) {
    if constexpr (DEP == 1) {
      for (int kt = 0; kt < ns; ++kt) iter(kt, std::integral_constant<int, 0>(), tmac);
    } else {
      int kt = 0;
      for (; kt + 1 < ns; kt += 2) {
        iter(kt, std::integral_constant<int, 0>(), tmac);
        iter(kt + 1, std::integral_constant<int, 1>(), tmac);
      }
      if (kt < ns) iter(kt, std::integral_constant<int, 0>(), tmac);
    }
  };
  if constexpr (!IDLE) {
    kloop(std::integral_constant<int, TM>());
  } else {
    // (the persistent launches keep two copies of the loop: a third one
    // measured slower there: batched FP32 124 -> 140 ms)
    static_assert(TM <= 2, "8-wave shapes hold one or two row blocks per wave");
    if (tma >= TM || (COH && tma > 0)) kloop(std::integral_constant<int, TM>());
    else if (!COH && TM == 2 && tma == 1) kloop(std::integral_constant<int, 1>());
    else kloop(std::integral_constant<int, 0>());
  }

  // epilogue: accumulator (i, j, v) of lane (li, lh) is row 8(v/4) + 4 lh + v%4,
  // column li of the 32 x 32 block
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int row = wr * WTM + i * 32 + (v >> 2) * 8 + lh * 4 + (v & 3);
      if (m0 + row >= td.m) continue;
      const int code = sm.sOut[row];
      const auto p = gmem(code >= 0 ? a.U + (long long)code * a.ldu : a.WS + (long long)(-(code + 1)) * a.ldws);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int col = n0 + wc * WTN + j * 32 + li;
        if (col < a.r) {
          if constexpr (COH) {
            auto q = (__attribute__((address_space(1))) float*)(p + col);
            const float base = accumulate ? __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0.f;
            __hip_atomic_store(q, accumulate ? base + acc[i][j][v] : acc[i][j][v], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
          } else {
            if (accumulate) p[col] += acc[i][j][v];
            else p[col] = acc[i][j][v];
          }
        }
      }
    }
}

// VEC: every W, U and workspace row is 16-byte aligned and r % 4 == 0 (B rows
// are then loaded as 16-byte vectors)
template <int PREC, int BM, int BN, int WM, int WN, bool ACC, bool VEC>
__device__ __forceinline__ void gemm_tiles(const KArgs& a) {
  __shared__ Smem<PREC, BM, BN> sm;
  const int2 it = a.items[blockIdx.x];
  if (it.x < 0) return;
  const TaskDesc td = a.tasks[it.x];
  tile_body<PREC, BM, BN, WM, WN, VEC>(a, td, (it.y >> 16) * BM, (it.y & 0xffff) * BN, ACC, sm);
}


// Entry points with the same body, so that profiles separate the upward pass,
// the far field, the downward pass and the leaf output.
template <int PREC, int BM, int BN, int WM, int WN, bool VEC>
__global__ __launch_bounds__(WM * WN * 64) void n2s_tiles(KArgs a) { gemm_tiles<PREC, BM, BN, WM, WN, false, VEC>(a); }
template <int PREC, int BM, int BN, int WM, int WN, bool VEC>
__global__ __launch_bounds__(WM * WN * 64) void s2s_tiles(KArgs a) { gemm_tiles<PREC, BM, BN, WM, WN, false, VEC>(a); }
template <int PREC, int BM, int BN, int WM, int WN, bool VEC>
__global__ __launch_bounds__(WM * WN * 64) void s2n_tiles(KArgs a) { gemm_tiles<PREC, BM, BN, WM, WN, true, VEC>(a); }
template <int PREC, int BM, int BN, int WM, int WN, bool ACC, bool VEC>
__global__ __launch_bounds__(WM * WN * 64) void leaf_tiles(KArgs a) { gemm_tiles<PREC, BM, BN, WM, WN, ACC, VEC>(a); }
template <int PREC, int BM, int BN, int WM, int WN, bool VEC>
__global__ __launch_bounds__(WM * WN * 64) void s2n_leaf_tiles(KArgs a) { gemm_tiles<PREC, BM, BN, WM, WN, false, VEC>(a); }

typedef void (*KernelFn)(KArgs);

// L2L with the near blocks computed from the points (GEO = 1 + kernel kind);
// whether it accumulates into U comes with the arguments.
template <int BM, int BN, int WM, int WN, bool VEC, int GEO>
__global__ __launch_bounds__(WM * WN * 64) void l2l_geo_tiles(KArgs a) {
  __shared__ Smem<PREC_F32, BM, BN> sm;
  __shared__ f32x4 sg[2 * 32 * 3];
  const int2 it = a.items[blockIdx.x];
  if (it.x < 0) return;
  const TaskDesc td = a.tasks[it.x];
  tile_body<PREC_F32, BM, BN, WM, WN, VEC, false, GEO>(a, td, (it.y >> 16) * BM, (it.y & 0xffff) * BN,
                                                      a.gacc != 0, sm, sg);
}

// ------------------------------------------------------------ persistent launches
// Several steps (of one or of many compressions) in one persistent launch.
// Every (instance, step) pair is a stage.  Work items (tiles) sit in one
// global queue in stage order; each resident block takes the next item, waits
// until the item's dependencies are met, runs the tile, and counts it.  A
// dependency is a counter reaching a value: counters count finished tiles per
// stage and per task, so a tile can wait for a whole stage (S2S waits for the
// upward pass) or only for the tasks whose rows it reads (a node's N2S waits
// for its two children, a child's S2N for its parent).  Counters and the
// queue head only grow: a launch made after `epoch` earlier launches with the
// same tables waits for epoch * (tiles per launch) + need, so nothing has to
// be cleared between launches.  Every item's dependencies precede it in the
// queue and are held by running blocks, so the waits always end; a spin limit
// still bounds each wait (the block then flags an error and skips the tile,
// which still counts as finished).
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

struct BItem {
  int inst, stage, task, tile;   // tile = row tile << 16 | column tile
  int tctr;                      // the task's counter (the stage's counter is `stage`)
  int dep[2];                    // counters waited for (-1: none)
  int need[2];                   // finished tiles they must reach in this launch
};

struct BArgs {
  const BInst* inst;             // per instance, or nullptr: every item uses `one`
  BInst one;
  const BItem* items;
  int n_items;
  const int* stage_acc;          // 1: the stage accumulates into its output
  const int* ctr_total;          // tiles each counter receives per launch
  unsigned long long* ctr;       // stage counters, then task counters
  unsigned long long* head;      // queue head
  unsigned long long head_base;  // head value when this launch starts
  unsigned long long epoch;      // earlier launches with these counters
  int* error;                    // set to 1 if a wait exceeded the spin limit
  long long spin_limit;
};

template <int PREC, int BM, int BN, int WM, int WN, bool VEC>
__device__ __forceinline__ void persistent_tiles(const BArgs& b) {
  __shared__ Smem<PREC, BM, BN> sm;
  __shared__ int s_item;
  __shared__ int s_ok;
  // Lane 0's bookkeeping (publish the previous tile, take the next item, wait
  // for the item's dependencies) sits at the top of the iteration, each part
  // closed by a barrier, and the values it broadcasts are made wave-uniform
  // with readfirstlane: the loop's exit and back edge are then uniform
  // branches, so the compiler cannot split lane 0 from its wave.
  int last_s = -1, last_t = -1;
  while (true) {
    if (threadIdx.x == 0) {
      if (last_s >= 0) {
        // the tile's rows were written with device-coherent stores that every
        // thread waited for before the barrier: relaxed increments publish it
        __hip_atomic_fetch_add(&b.ctr[last_s], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&b.ctr[last_t], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      const unsigned long long h = atomicAdd(b.head, 1ull) - b.head_base;
      s_item = h < (unsigned long long)b.n_items ? (int)h : b.n_items;
    }
    __syncthreads();
    const int idx = __builtin_amdgcn_readfirstlane(s_item);
    if (idx >= b.n_items) break;
    const BItem it = b.items[idx];
    if (threadIdx.x == 0) {
      int ok = 1;
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const int c = it.dep[d];
        if (c >= 0 && ok) {
          // Relaxed polls, and no acquire fence after them: the rows this tile
          // reads from other tiles are loaded with device-coherent loads (an
          // acquire at device scope would invalidate this XCD's L2 and cost
          // every block on it its cached operands).
          const unsigned long long target = b.epoch * (unsigned long long)b.ctr_total[c] + (unsigned long long)it.need[d];
          long long polls = 0;
          while (__hip_atomic_load(&b.ctr[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(8);
            if (++polls > b.spin_limit) {
              atomicExch(b.error, 1);
              ok = 0;
              break;
            }
          }
        }
      }
      s_ok = ok;
    }
    __syncthreads();
    const int stage = __builtin_amdgcn_readfirstlane(it.stage);
    if (__builtin_amdgcn_readfirstlane(s_ok)) {
      const BInst& in = b.inst ? b.inst[__builtin_amdgcn_readfirstlane(it.inst)] : b.one;
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
      tile_body<PREC, BM, BN, WM, WN, VEC, true>(a, td, m0, n0, b.stage_acc[stage] != 0, sm);
    }
    last_s = stage;
    last_t = __builtin_amdgcn_readfirstlane(it.tctr);
    __builtin_amdgcn_s_waitcnt(0);        // this thread's stores have completed
    __syncthreads();                      // every thread's stores done, LDS free
  }
}

// Many compressions in one launch (all steps of each), and the tree passes of
// one compression (entry points with the same body, so profiles separate
// them).
template <int PREC, int BM, int BN, int WM, int WN, bool VEC>
__global__ __launch_bounds__(WM * WN * 64) void batched_tiles(BArgs b) { persistent_tiles<PREC, BM, BN, WM, WN, VEC>(b); }
template <int PREC, int BM, int BN, int WM, int WN, bool VEC>
__global__ __launch_bounds__(WM * WN * 64) void pass_tiles(BArgs b) { persistent_tiles<PREC, BM, BN, WM, WN, VEC>(b); }

typedef void (*BatchedFn)(BArgs);
constexpr int kNumCfg = 11;
constexpr int kNumFamily = 6;   // n2s, s2s, s2n (accumulate), leaf, leaf accumulating, s2n at the leaves
struct Cfg { int bm, bn, nt; };   // tile rows, tile columns, threads per block
constexpr Cfg kCfgs[kNumCfg] = {{128, 128, 256}, {128, 64, 256}, {64, 128, 256}, {64, 64, 256},
                                {128, 32, 256},  {32, 128, 256}, {256, 128, 256}, {128, 256, 256},
                                {256, 128, 512}, {128, 256, 512}, {256, 128, 512}};

template <int PREC, int BM, int BN, int WM, int WN, bool VEC>
void fill_family(KernelFn* row, BatchedFn* brow) {
  brow[0] = batched_tiles<PREC, BM, BN, WM, WN, VEC>;
  brow[1] = pass_tiles<PREC, BM, BN, WM, WN, VEC>;
  row[0] = n2s_tiles<PREC, BM, BN, WM, WN, VEC>;
  row[1] = s2s_tiles<PREC, BM, BN, WM, WN, VEC>;
  row[2] = s2n_tiles<PREC, BM, BN, WM, WN, VEC>;
  row[3] = leaf_tiles<PREC, BM, BN, WM, WN, false, VEC>;
  row[4] = leaf_tiles<PREC, BM, BN, WM, WN, true, VEC>;
  row[5] = s2n_leaf_tiles<PREC, BM, BN, WM, WN, VEC>;
}

// table[cfg * kNumFamily + family], persistent[cfg * 2 + (0 batched, 1 pass)]
template <int PREC, bool VEC>
void fill_table(KernelFn* table, BatchedFn* persistent) {
  fill_family<PREC, 128, 128, 2, 2, VEC>(table + 0 * kNumFamily, persistent + 0);
  fill_family<PREC, 128, 64, 2, 2, VEC>(table + 1 * kNumFamily, persistent + 2);
  fill_family<PREC, 64, 128, 2, 2, VEC>(table + 2 * kNumFamily, persistent + 4);
  fill_family<PREC, 64, 64, 2, 2, VEC>(table + 3 * kNumFamily, persistent + 6);
  fill_family<PREC, 128, 32, 4, 1, VEC>(table + 4 * kNumFamily, persistent + 8);
  fill_family<PREC, 32, 128, 1, 4, VEC>(table + 5 * kNumFamily, persistent + 10);
  fill_family<PREC, 256, 128, 4, 1, VEC>(table + 6 * kNumFamily, persistent + 12);
  fill_family<PREC, 128, 256, 2, 2, VEC>(table + 7 * kNumFamily, persistent + 14);
  // 8 waves (two per SIMD) over the large tiles, each wave 64 x 64
  fill_family<PREC, 256, 128, 4, 2, VEC>(table + 8 * kNumFamily, persistent + 16);
  fill_family<PREC, 128, 256, 2, 4, VEC>(table + 9 * kNumFamily, persistent + 18);
  // 8 waves stacked along the rows, each wave 32 x 128
  fill_family<PREC, 256, 128, 8, 1, VEC>(table + 10 * kNumFamily, persistent + 20);
}

// geo[kind * kNumCfg + cfg], the same tile shapes as fill_table
template <bool VEC, int GEO>
void fill_geo_kind(KernelFn* t) {
  t[0] = l2l_geo_tiles<128, 128, 2, 2, VEC, GEO>;
  t[1] = l2l_geo_tiles<128, 64, 2, 2, VEC, GEO>;
  t[2] = l2l_geo_tiles<64, 128, 2, 2, VEC, GEO>;
  t[3] = l2l_geo_tiles<64, 64, 2, 2, VEC, GEO>;
  t[4] = l2l_geo_tiles<128, 32, 4, 1, VEC, GEO>;
  t[5] = l2l_geo_tiles<32, 128, 1, 4, VEC, GEO>;
  t[6] = l2l_geo_tiles<256, 128, 4, 1, VEC, GEO>;
  t[7] = l2l_geo_tiles<128, 256, 2, 2, VEC, GEO>;
  t[8] = l2l_geo_tiles<256, 128, 4, 2, VEC, GEO>;
  t[9] = l2l_geo_tiles<128, 256, 2, 4, VEC, GEO>;
  t[10] = l2l_geo_tiles<256, 128, 8, 1, VEC, GEO>;
}
template <bool VEC>
void fill_geo(KernelFn* t) {
  static_assert(kNumCfg == 11, "geometric tile table");
  fill_geo_kind<VEC, 1>(t);
  fill_geo_kind<VEC, 2>(t + kNumCfg);
  fill_geo_kind<VEC, 3>(t + 2 * kNumCfg);
}

// One translation unit per (precision, row alignment).
void kernels_f32_vec(KernelFn* table, BatchedFn* batched);
void kernels_f32_any(KernelFn* table, BatchedFn* batched);
void kernels_bf16_vec(KernelFn* table, BatchedFn* batched);
void kernels_bf16_any(KernelFn* table, BatchedFn* batched);
void kernels_x3_vec(KernelFn* table, BatchedFn* batched);
void kernels_x3_any(KernelFn* table, BatchedFn* batched);
void kernels_geo_vec(KernelFn* table);
void kernels_geo_any(KernelFn* table);

}  // namespace dev
}  // namespace gofmm
