// Neighbour-list merge on the GPU: the ANN task of the compression (Sec. 2.2,
// "index neighbor list", and the ANN row of Table 2).
//
// A task is a block K(R, C) of the matrix, sampled on the host (the sampler is
// the method's only access to K): for a randomized-tree leaf R = C = the
// leaf's indices; for the brute-force search R is a block of rows and C every
// index.  For each row i of R the task forms the Gram distances to the
// columns (eq. 3: d_ij = sqrt(max(K_ii + K_jj - 2 K_ij, 0)); eq. 4: the angle
// 1 - K_ij^2 / (K_ii K_jj), clamped to [0, 1]) in FP64, exactly as the host
// forms them, and keeps in i's list the kappa smallest of the list's entries
// and the candidates, ordered by (distance, index), each index once.  Lists
// stay on the device between tasks.
//
// One 64-wide wave per (task, row).  Lane l holds entry l of the list (kappa
// <= 64) and one candidate column of the current chunk of 64.  A chunk that
// holds no candidate below the list's last entry is skipped; otherwise the
// new list is selected entry by entry: each round takes the smallest
// (distance, index) key over the 128 held by the wave (a butterfly reduction
// across lanes), and every lane drops the entries equal to it, so an index
// seen again (same pair, same sampled entry, same key) is kept once.  Every
// decision is a comparison of the same FP64 values the host compares, so the
// lists equal the host's bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <memory>
#include <string>
#include <vector>

#include "internal.hpp"

namespace gofmm {

namespace {

struct KnnTaskDev {
  long long kofs;      // block at kblk + kofs, column-major with leading dimension nr
  int rofs, nr;        // rows: idx[rofs .. rofs + nr)
  int cofs, nc;        // columns: idx[cofs .. cofs + nc)
};

__device__ __forceinline__ bool key_less(double a, int ja, double b, int jb) {
  return a < b || (a == b && ja < jb);
}

__device__ __forceinline__ double gram_dist(double kij, double di, double dj, int kind) {
  if (kind == GOFMM_GRAM_L2) {
    const double x = di + dj - 2.0 * kij;     // 2 k is exact: no rounding depends on contraction
    return __builtin_sqrt(x > 0.0 ? x : 0.0);
  }
  const double d = 1.0 - (kij * kij) / (di * dj);
  return d < 0.0 ? 0.0 : (d > 1.0 ? 1.0 : d);
}

__global__ __launch_bounds__(256) void knn_merge_kernel(const KnnTaskDev* __restrict__ tasks,
                                                        const int2* __restrict__ items, int n_items,
                                                        const int* __restrict__ idx,
                                                        const double* __restrict__ kblk,
                                                        const double* __restrict__ diag, int kind, int kappa,
                                                        int* __restrict__ lj, double* __restrict__ ld) {
  const int w = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (w >= n_items) return;                          // whole waves leave together
  const int lane = threadIdx.x & 63;
  const int2 it = items[w];
  const KnnTaskDev t = tasks[it.x];
  const int a = it.y;
  const int i = idx[t.rofs + a];
  const double di = diag[i];
  const long long lbase = (long long)i * kappa;
  double kd = INFINITY;
  int kj = INT_MAX;                                 // empty entries sort last
  if (lane < kappa) {
    const int j0 = lj[lbase + lane];
    if (j0 >= 0) {
      kd = ld[lbase + lane];
      kj = j0;
    }
  }
  const double* col = kblk + t.kofs + a;
  for (int c0 = 0; c0 < t.nc; c0 += 64) {
    const int tc = c0 + lane;
    double cd = INFINITY;
    int cj = INT_MAX;
    if (tc < t.nc) {
      cj = idx[t.cofs + tc];
      cd = gram_dist(col[(long long)tc * t.nr], di, diag[cj], kind);
    }
    // the list's last entry (lane kappa - 1) bounds what can enter
    const double td = __shfl(kd, kappa - 1, 64);
    const int tj = __shfl(kj, kappa - 1, 64);
    if (!__any(key_less(cd, cj, td, tj))) continue;
    double nd = INFINITY;
    int nj = INT_MAX;
    for (int s = 0; s < kappa; ++s) {
      double md;
      int mj;
      if (key_less(cd, cj, kd, kj)) { md = cd; mj = cj; } else { md = kd; mj = kj; }
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const double od = __shfl_xor(md, o, 64);
        const int oj = __shfl_xor(mj, o, 64);
        if (key_less(od, oj, md, mj)) { md = od; mj = oj; }
      }
      if (lane == s) { nd = md; nj = mj; }
      if (kd == md && kj == mj) { kd = INFINITY; kj = INT_MAX; }
      if (cd == md && cj == mj) { cd = INFINITY; cj = INT_MAX; }
    }
    kd = nd;
    kj = nj;
  }
  if (lane < kappa) {
    lj[lbase + lane] = kj == INT_MAX ? -1 : kj;
    ld[lbase + lane] = kj == INT_MAX ? INFINITY : kd;
  }
}

#define KNN_HIP(expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      fail(e_ == hipErrorOutOfMemory ? GOFMM_ENOMEM : GOFMM_EHIP,                     \
           std::string(#expr) + ": " + hipGetErrorString(e_));                        \
  } while (0)

template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t cap = 0;
  ~DevBuf() { (void)hipFree(p); }
  void fit(size_t n) {
    if (n <= cap) return;
    (void)hipFree(p);
    p = nullptr;
    cap = 0;
    KNN_HIP(hipMalloc((void**)&p, std::max<size_t>(1, n) * sizeof(T)));
    cap = n;
  }
};

}  // namespace

struct KnnDevice {
  i64 n = 0;
  int kappa = 0, kind = 0;
  DevBuf<double> diag, ld, kblk;
  DevBuf<int> lj, idx;
  DevBuf<KnnTaskDev> tasks;
  DevBuf<int2> items;
};

KnnDevice* knn_device_create(i64 n, int kappa, int kind, const double* diag) {
  if (kappa < 1 || kappa > 64) fail(GOFMM_EINVAL, "the device neighbour search keeps at most 64 neighbours");
  if (n >= INT_MAX) fail(GOFMM_ELIMIT, "the device neighbour search needs n < 2^31");
  std::unique_ptr<KnnDevice> k(new KnnDevice);
  k->n = n;
  k->kappa = kappa;
  k->kind = kind;
  k->diag.fit((size_t)n);
  KNN_HIP(hipMemcpy(k->diag.p, diag, (size_t)n * sizeof(double), hipMemcpyHostToDevice));
  k->lj.fit((size_t)n * kappa);
  k->ld.fit((size_t)n * kappa);
  KNN_HIP(hipMemset(k->lj.p, 0xff, (size_t)n * kappa * sizeof(int)));    // every entry -1: empty
  return k.release();
}

void knn_device_free(KnnDevice* k) { delete k; }

void knn_device_merge(KnnDevice* k, const std::vector<KnnTask>& tasks, const std::vector<int>& idx,
                      const std::vector<double>& blocks) {
  if (tasks.empty()) return;
  std::vector<KnnTaskDev> td(tasks.size());
  std::vector<int2> items;
  for (size_t q = 0; q < tasks.size(); ++q) {
    const KnnTask& t = tasks[q];
    if (t.rofs < 0 || t.cofs < 0 || t.nr < 0 || t.nc < 0 || t.rofs + t.nr > (i64)idx.size() ||
        t.cofs + t.nc > (i64)idx.size() || t.kofs < 0 || t.kofs + t.nr * t.nc > (i64)blocks.size())
      fail(GOFMM_EINVAL, "neighbour task outside its buffers");
    td[q] = KnnTaskDev{(long long)t.kofs, (int)t.rofs, (int)t.nr, (int)t.cofs, (int)t.nc};
    for (i64 a = 0; a < t.nr; ++a) items.push_back(make_int2((int)q, (int)a));
  }
  for (int x : idx)
    if (x < 0 || x >= k->n) fail(GOFMM_EINVAL, "neighbour task index out of range");
  k->tasks.fit(td.size());
  k->items.fit(items.size());
  k->idx.fit(idx.size());
  k->kblk.fit(blocks.size());
  KNN_HIP(hipMemcpy(k->tasks.p, td.data(), td.size() * sizeof(KnnTaskDev), hipMemcpyHostToDevice));
  KNN_HIP(hipMemcpy(k->items.p, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice));
  KNN_HIP(hipMemcpy(k->idx.p, idx.data(), idx.size() * sizeof(int), hipMemcpyHostToDevice));
  KNN_HIP(hipMemcpy(k->kblk.p, blocks.data(), blocks.size() * sizeof(double), hipMemcpyHostToDevice));
  const int n_items = (int)items.size();
  hipLaunchKernelGGL(knn_merge_kernel, dim3((n_items + 3) / 4), dim3(256), 0, nullptr, k->tasks.p, k->items.p,
                     n_items, k->idx.p, k->kblk.p, k->diag.p, k->kind, k->kappa, k->lj.p, k->ld.p);
  KNN_HIP(hipGetLastError());
  KNN_HIP(hipDeviceSynchronize());
}

void knn_device_read(KnnDevice* k, i64* knn) {
  std::vector<int> v((size_t)k->n * k->kappa);
  KNN_HIP(hipMemcpy(v.data(), k->lj.p, v.size() * sizeof(int), hipMemcpyDeviceToHost));
  for (size_t t = 0; t < v.size(); ++t) knn[t] = v[t];
}

}  // namespace gofmm
