// Internal declarations shared by the host compression, the packer, the file
// format and the device evaluator.  Not part of the public ABI.
#pragma once

#include <atomic>
#include <climits>
#include <cstdint>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/gofmm.h"

namespace gofmm {

using i64 = int64_t;
using i32 = int32_t;

// ------------------------------------------------------------------ errors
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};
[[noreturn]] inline void fail(int code, const std::string& msg) { throw Error(code, msg); }
void set_last_error(const std::string& msg);

// ------------------------------------------------------------------ RNG
// SplitMix64 (Steele, Lea, Flood 2014): a counter-based 64-bit generator.
struct Rng {
  uint64_t s;
  explicit Rng(uint64_t seed) : s(seed) {}
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  // uniform integer in [0, n)
  uint64_t below(uint64_t n) { return n ? next() % n : 0; }
};
inline uint64_t mix(uint64_t a, uint64_t b) { Rng r(a ^ (b * 0xD1B54A32D192ED03ull)); r.next(); return r.next(); }

// ------------------------------------------------------------------ heap tree
inline i64 n_nodes(int depth) { return (i64(1) << (depth + 1)) - 1; }
inline i64 first_leaf(int depth) { return (i64(1) << depth) - 1; }
inline int level_of(i64 h) { int l = 0; while (((h + 1) >> (l + 1)) != 0) ++l; return l; }

// ------------------------------------------------------------------ sampler
struct Sampler {
  gofmm_sampler fn = nullptr;
  void* user = nullptr;
  // The callback's own layout: out[i + j * ld] = K(I[i], J[j]), an nI x nJ
  // column-major block with leading dimension ld >= nI (default nI).
  void operator()(i64 nI, const i64* I, i64 nJ, const i64* J, double* out, i64 ld = -1) const {
    if (nI == 0 || nJ == 0) return;
    int rc = fn(user, nI, I, nJ, J, out, ld < 0 ? nI : ld);
    if (rc != 0) fail(GOFMM_ECALLBACK, "sampler returned " + std::to_string(rc));
  }
};

// ------------------------------------------------------------------ device plan
enum Prec { PREC_F32 = 0, PREC_BF16 = 1, PREC_BF16X3 = 2 };

// One gather-GEMM: out[m x r] (=|+=) A[m x k] * B[k x r], where row t of B is
// row rows[idx_off + t] of the right-hand-side space and row i of out is row
// rows[idx_off + lda + i] of the output space (row codes below).
struct TaskDesc {
  i64 a_off;    // element offset of A in its buffer, in matrix-core fragment
                // order (rows padded to 32, k to lda), see the packing
  i64 idx_off;  // offset into the row-code array
  i32 m, k, lda;
  i32 kws;      // leading B rows that are workspace rows (the rest are rows of W)
};

// Row codes: c >= 0 is row c of the caller's W (reads) or U (writes);
// c < 0 (and not ROW_ZERO) is workspace row -c-1; ROW_ZERO reads as zeros.
constexpr i32 ROW_ZERO = INT32_MIN;

enum Phase { PH_N2S = 0, PH_S2S = 1, PH_S2N = 2, PH_L2L = 3 };

struct LaunchDesc {
  int prec;          // Prec of A for every task in the range
  int accumulate;    // 1: out += A B ; 0: out = A B
  i32 t_begin, t_end;
  int kind;          // 0 n2s-leaf, 1 n2s-level, 2 s2s, 3 leaf-out, 4 s2n-leaf, 5 l2l, 6 s2n-level,
                     // 7 l2l with the near blocks computed on the device from the points
  int level;
  std::string name;
  double flops = 0;   // per right-hand side: sum of 2 m k over the tasks
  i64 bytes = 0;      // operator bytes the launch reads
};

struct HostPlan {
  std::vector<TaskDesc> tasks;
  std::vector<LaunchDesc> launches;
  std::vector<i32> rows;
  std::vector<float> a_f32;
  std::vector<uint16_t> a_b16;
  std::vector<uint16_t> a_x3;        // split BF16: hi plane, then lo plane at x3_plane
  i64 x3_plane = 0;
  // kind-7 launches: per task, lda column entries of kGeoStride floats (the
  // column's point, zero-padded to 8 coordinates, then its index as int bits),
  // at the task's a_off; padding columns have index -1
  std::vector<float> geo_cols;
  i64 ws_rows = 0;        // 2 * sum of ranks: skeleton weights then potentials
  double flops_phase[4] = {0, 0, 0, 0};     // per right-hand side
  i64 bytes_phase[4] = {0, 0, 0, 0};        // operator bytes read per evaluate
};

struct DeviceState;  // defined by the evaluator
void device_state_free(DeviceState* d);

// Staging slots for batched launches on one stream (see eval.hip).
struct BatchRing {
  static constexpr int NS = 4;
  struct Slot {
    char* dev = nullptr;
    char* host = nullptr;     // pinned
    size_t cap = 0;
    size_t err_off = 0;
    void* ev = nullptr;       // hipEvent_t
  };
  Slot slot[NS];
  int next = 0;
  int last = -1;
  ~BatchRing();
};

// Near blocks computed on the device (geometric mode): a radial kernel over
// points of at most kGeoDim coordinates.
constexpr int kGeoDim = 8;
constexpr int kGeoStride = 12;   // floats per point entry: 8 coordinates, index bits, 3 zeros
struct GeoKernel {
  int kind = -1;                 // -1: near blocks are stored; else 0 Gaussian, 1 IMQ, 2 Laplacian-like
  int dim = 0;
  float h2inv = 0.f, shift = 0.f;
  std::vector<float> pts;        // n x kGeoStride, original order
};
// Kernel, points and parameters of a gofmm_kernel_create state (false if the
// pointer does not hold one).
bool kernel_state_geo(const void* state, GeoKernel& out);

// ------------------------------------------------------------------ compression
struct Compression {
  // parameters
  i64 n = 0;
  int depth = 0;
  i64 leaf_size = 0, max_rank = 0;
  double tol = 0;
  int kappa = 0;
  double budget = 0;
  int distance = GOFMM_GRAM_L2;
  int storage = GOFMM_FP32, near_storage = GOFMM_FP32;
  uint64_t seed = 0;
  // tree
  std::vector<i64> perm, node_start, node_size, split_p, split_q;
  std::vector<std::vector<i64>> centroid;
  // neighbours (n x kappa, original numbering); may be empty after import
  std::vector<i64> knn;
  int knn_k = 0;
  // lists
  std::vector<std::vector<i64>> near;  // per leaf number, heap ids of leaves
  std::vector<std::vector<i64>> far;   // per heap id
  // skeletons
  std::vector<std::vector<i64>> skel, samp;
  std::vector<std::vector<double>> proj;  // s x ncols row-major
  // near blocks on the device (geometric mode), set by gofmm_use_device_kernel
  GeoKernel geo;
  // device operator
  HostPlan plan;
  DeviceState* dev = nullptr;
  uint64_t uid = next_uid();   // identity for caches keyed by compression
  static uint64_t next_uid() {
    static std::atomic<uint64_t> counter{0};
    return ++counter;
  }

  i64 nn() const { return n_nodes(depth); }
  i64 fl() const { return first_leaf(depth); }
  i64 n_leaves() const { return i64(1) << depth; }
  bool is_leaf(i64 h) const { return h >= fl(); }
  i64 rank(i64 h) const { return (i64)skel[h].size(); }
  i64 ncols(i64 h) const { return is_leaf(h) ? node_size[h] : rank(2 * h + 1) + rank(2 * h + 2); }
  ~Compression() { if (dev) device_state_free(dev); }
};

// host pipeline pieces
int choose_depth(i64 n, i64 m);
void build_compression(Compression& c, const Sampler& K, const gofmm_params& p);
void build_plan(Compression& c, const Sampler& K, int threads);
void validate_structure(const Compression& c);
void write_file(const Compression& c, const char* path);
void read_file(Compression& c, const char* path);

// FP64 ID of a column-major nrow x ncol block A (leading dimension nrow,
// overwritten by the factorization): returns rank s and fills piv (ncol
// entries, first s are the skeleton columns) and P (s x ncol, row-major).
int interp_decomp(double* A, int nrow, int ncol, double tol, int smax,
                  std::vector<int>& piv, std::vector<double>& P);

// Neighbour-list merges on the device (knn.hip).  A task is the sampled
// block K(R, C), column-major with leading dimension nr, at blocks[kofs];
// its rows are idx[rofs .. rofs + nr), its columns idx[cofs .. cofs + nc).
struct KnnTask { i64 kofs, rofs, nr, cofs, nc; };
struct KnnDevice;
KnnDevice* knn_device_create(i64 n, int kappa, int kind, const double* diag);
void knn_device_merge(KnnDevice* k, const std::vector<KnnTask>& tasks, const std::vector<int>& idx,
                      const std::vector<double>& blocks);
void knn_device_read(KnnDevice* k, i64* knn);       // n x kappa, -1 for an empty entry
void knn_device_free(KnnDevice* k);

// Interpolative decompositions of a batch of sampled blocks on the device
// (idqr.hip), with the steps and rounding of interp_decomp: each job's block
// is row-major (nrow x ncol) at blocks[a_off]; fills rank, piv (ncol entries,
// the first rank are the skeleton columns) and P (rank x ncol, row-major).
struct IdJob {
  i64 a_off = 0, nrow = 0, ncol = 0;
  int rank = 0;
  std::vector<int> piv;
  std::vector<double> P;
};
void id_device_batch(std::vector<IdJob>& jobs, const std::vector<double>& blocks, double tol, int smax);

// BF16 round-to-nearest-even of a double (through its nearest float).
uint16_t to_bf16(double x);
double from_bf16(uint16_t h);

}  // namespace gofmm

// The opaque handle of the C ABI.
struct gofmm_compression {
  gofmm::Compression c;
};
