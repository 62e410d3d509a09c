// Interpolative decompositions of all nodes of a tree level on the GPU: the
// skeletonization of Sec. 2.2 ("Low-rank approximation", eqs. 7-8), batched.
//
// Each node's sampled block A = K(I', cols) (nrow x ncol, FP64) is factored by
// Householder QR with column pivoting (the column of largest residual norm is
// taken next), stopped at the adaptive rank s: the smallest k >= 1 with
// |R_kk| < tol |R_00|, at most min(s_max, ncol, nrow).  Then T = R11^{-1} R12
// by back substitution gives P = [I, T] Pi^T.
//
// The steps, their order and every floating-point operation are those of the
// host factorization (qrcp.cpp): each column's sums run in one thread, in
// ascending row order, with every product rounded before it is added (no
// fused multiply-add: the host's target has none), and the pivot is the first
// column of largest norm.  So the device gives the host's skeletons and P bit
// for bit.  Blocks are stored row-major, so the threads of a wave, one column
// each, read one row at a time with coalesced loads.
//
// One QR step of every node of the level is two launches: `id_pivot` (one
// block per node: pivot, column swap, rank test, reflector) and `id_update`
// (one thread per trailing column: apply the reflector, downdate the norm).
// Nodes that reached their rank skip the later steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <climits>
#include <cmath>
#include <string>
#include <vector>

#include "internal.hpp"

namespace gofmm {

namespace {

struct IdNode {
  long long a_off;   // block at A + a_off, row-major (row stride ncol)
  int nrow, ncol, kmax;
  int c_off;         // norms, pivots at + c_off (ncol entries)
  int v_off;         // reflector at + v_off (nrow entries)
};

struct IdState {     // per node, device
  double r00, beta;
  int done, rank;
};

constexpr int kIdThreads = 256;

// products rounded before the sum, as on the host
#pragma clang fp contract(off)

__global__ __launch_bounds__(kIdThreads) void id_norms(const IdNode* __restrict__ nodes, int n_nodes,
                                                       const double* __restrict__ A, double* __restrict__ nrm,
                                                       double* __restrict__ ref, int* __restrict__ piv,
                                                       IdState* __restrict__ st) {
  const int b = blockIdx.y;
  const IdNode nd = nodes[b];
  const int j = blockIdx.x * kIdThreads + threadIdx.x;
  if (j == 0) st[b] = IdState{0.0, 0.0, 0, nd.kmax};
  if (j >= nd.ncol) return;
  const double* a = A + nd.a_off + j;
  double t = 0.0;
  for (int i = 0; i < nd.nrow; ++i) {
    const double x = a[(long long)i * nd.ncol];
    t += x * x;
  }
  nrm[nd.c_off + j] = t;
  ref[nd.c_off + j] = t;
  piv[nd.c_off + j] = j;
}

// Step k of every node: pivot (first column of largest norm), swap, rank
// test, Householder reflector H = I - beta v v^T with H x = alpha e_k.
__global__ __launch_bounds__(kIdThreads) void id_pivot(const IdNode* __restrict__ nodes, int k, double* __restrict__ A,
                                                       double* __restrict__ nrm, double* __restrict__ ref,
                                                       int* __restrict__ piv, double* __restrict__ V,
                                                       IdState* __restrict__ st, double tol) {
  const int b = blockIdx.x;
  const IdNode nd = nodes[b];
  if (st[b].done) return;
  if (k >= nd.kmax) {                       // no break: rank kmax
    if (threadIdx.x == 0) st[b].done = 1;
    return;
  }
  double* a = A + nd.a_off;
  double* nr = nrm + nd.c_off;
  double* rf = ref + nd.c_off;
  int* pv = piv + nd.c_off;
  double* v = V + nd.v_off;
  const int ld = nd.ncol;
  __shared__ double sv[kIdThreads];
  __shared__ int si[kIdThreads];
  __shared__ double s_alpha;
  __shared__ int s_stop;
  // argmax over j >= k of nr[j], the smallest j among equal norms
  double best = -1.0;
  int bj = INT_MAX;
  for (int j = k + threadIdx.x; j < nd.ncol; j += kIdThreads) {
    const double x = nr[j];
    if (bj == INT_MAX || x > best) { best = x; bj = j; }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bj;
  __syncthreads();
  for (int o = kIdThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const double x = sv[threadIdx.x + o];
      const int xj = si[threadIdx.x + o];
      if (xj != INT_MAX && (si[threadIdx.x] == INT_MAX || x > sv[threadIdx.x] ||
                            (x == sv[threadIdx.x] && xj < si[threadIdx.x]))) {
        sv[threadIdx.x] = x;
        si[threadIdx.x] = xj;
      }
    }
    __syncthreads();
  }
  const int p = si[0];
  __syncthreads();
  if (p != k) {
    for (int i = threadIdx.x; i < nd.nrow; i += kIdThreads) {
      const double t = a[(long long)i * ld + k];
      a[(long long)i * ld + k] = a[(long long)i * ld + p];
      a[(long long)i * ld + p] = t;
    }
    if (threadIdx.x == 0) {
      const double t0 = nr[k]; nr[k] = nr[p]; nr[p] = t0;
      const double t1 = rf[k]; rf[k] = rf[p]; rf[p] = t1;
      const int t2 = pv[k]; pv[k] = pv[p]; pv[p] = t2;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double xn = 0.0;
    for (int i = k; i < nd.nrow; ++i) {
      const double x = a[(long long)i * ld + k];
      xn += x * x;
    }
    xn = __builtin_sqrt(xn);
    int stop = 0;
    if (k == 0) {
      st[b].r00 = xn;
      if (xn == 0.0) {                      // a zero block keeps one column, no coefficients
        st[b].rank = 1;
        st[b].done = 1;
        stop = 1;
      }
    } else if (xn < tol * st[b].r00) {
      st[b].rank = k;
      st[b].done = 1;
      stop = 1;
    }
    s_stop = stop;
    s_alpha = a[(long long)k * ld + k] >= 0.0 ? -xn : xn;
  }
  __syncthreads();
  if (s_stop) return;
  const double alpha = s_alpha;
  for (int i = k + threadIdx.x; i < nd.nrow; i += kIdThreads) v[i] = a[(long long)i * ld + k];
  __syncthreads();
  if (threadIdx.x == 0) {
    v[k] -= alpha;
    double vv = 0.0;
    for (int i = k; i < nd.nrow; ++i) vv += v[i] * v[i];
    st[b].beta = vv > 0.0 ? 2.0 / vv : 0.0;
    a[(long long)k * ld + k] = alpha;
  }
  for (int i = k + 1 + threadIdx.x; i < nd.nrow; i += kIdThreads) a[(long long)i * ld + k] = 0.0;
}

// Step k, trailing columns j > k: apply the reflector and downdate the
// residual norm (recomputed when more than half of its digits cancelled).
__global__ __launch_bounds__(kIdThreads) void id_update(const IdNode* __restrict__ nodes, int k,
                                                        double* __restrict__ A, double* __restrict__ nrm,
                                                        double* __restrict__ ref, const double* __restrict__ V,
                                                        const IdState* __restrict__ st, double tol3z) {
  const int b = blockIdx.y;
  const IdNode nd = nodes[b];
  if (st[b].done || k >= nd.kmax) return;
  const int j = k + 1 + blockIdx.x * kIdThreads + threadIdx.x;
  const double* v = V + nd.v_off;
  // the reflector, staged through LDS for the block's columns
  extern __shared__ double sv[];
  for (int i = k + threadIdx.x; i < nd.nrow; i += kIdThreads) sv[i - k] = v[i];
  __syncthreads();
  if (j >= nd.ncol) return;
  double* a = A + nd.a_off + j;
  const long long ld = nd.ncol;
  double d = 0.0;
  for (int i = k; i < nd.nrow; ++i) d += sv[i - k] * a[i * ld];
  d *= st[b].beta;
  for (int i = k; i < nd.nrow; ++i) a[i * ld] -= d * sv[i - k];
  const double rkj = a[(long long)k * ld];
  double nj = nrm[nd.c_off + j] - rkj * rkj;
  if (nj <= tol3z * ref[nd.c_off + j] || nj < 0.0) {
    nj = 0.0;
    for (int i = k + 1; i < nd.nrow; ++i) {
      const double x = a[i * ld];
      nj += x * x;
    }
    ref[nd.c_off + j] = nj;
  }
  nrm[nd.c_off + j] = nj;
}

// T = R11^{-1} R12, in place in rows 0 .. s-1 of columns j >= s.
__global__ __launch_bounds__(kIdThreads) void id_solve(const IdNode* __restrict__ nodes, double* __restrict__ A,
                                                       const IdState* __restrict__ st) {
  const int b = blockIdx.y;
  const IdNode nd = nodes[b];
  const int s = st[b].rank;
  const int j = s + blockIdx.x * kIdThreads + threadIdx.x;
  if (j >= nd.ncol) return;
  double* a = A + nd.a_off;
  const long long ld = nd.ncol;
  for (int i = s - 1; i >= 0; --i) {
    double acc = a[i * ld + j];
    for (int q = i + 1; q < s; ++q) acc -= a[i * ld + q] * a[q * ld + j];
    a[i * ld + j] = acc / a[i * ld + i];
  }
}

#define ID_HIP(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      fail(e_ == hipErrorOutOfMemory ? GOFMM_ENOMEM : GOFMM_EHIP,                     \
           std::string(#expr) + ": " + hipGetErrorString(e_));                        \
  } while (0)

template <class T>
struct IdBuf {
  T* p = nullptr;
  ~IdBuf() { (void)hipFree(p); }
  void alloc(size_t n) { ID_HIP(hipMalloc((void**)&p, std::max<size_t>(1, n) * sizeof(T))); }
};

}  // namespace

// Factor the blocks of `jobs` (row-major, in `blocks` at each job's a_off) on
// the current device; fills each job's rank, pivots and P (s x ncol,
// row-major, P[:, piv[:s]] = I).  Synchronous.
void id_device_batch(std::vector<IdJob>& jobs, const std::vector<double>& blocks, double tol, int smax) {
  if (jobs.empty()) return;
  const int nb = (int)jobs.size();
  std::vector<IdNode> nodes(nb);
  long long cols = 0, rowsum = 0;
  int max_ncol = 0, max_nrow = 0, max_k = 0;
  for (int q = 0; q < nb; ++q) {
    const IdJob& jb = jobs[q];
    if (jb.nrow < 1 || jb.ncol < 1 || jb.a_off < 0 || jb.a_off + jb.nrow * jb.ncol > (i64)blocks.size())
      fail(GOFMM_EINVAL, "interpolative-decomposition block outside its buffer");
    if (jb.nrow > 8192 || jb.ncol >= INT_MAX / 2)
      fail(GOFMM_ELIMIT, "device interpolative decomposition takes at most 8192 sampled rows");
    const int kmax = std::max(1, std::min(std::min(smax, (int)jb.ncol), (int)jb.nrow));
    nodes[q] = IdNode{(long long)jb.a_off, (int)jb.nrow, (int)jb.ncol, kmax, (int)cols, (int)rowsum};
    cols += jb.ncol;
    rowsum += jb.nrow;
    max_ncol = std::max(max_ncol, (int)jb.ncol);
    max_nrow = std::max(max_nrow, (int)jb.nrow);
    max_k = std::max(max_k, kmax);
  }
  if (cols >= INT_MAX || rowsum >= INT_MAX) fail(GOFMM_ELIMIT, "too many columns in one level");
  IdBuf<double> A, nrm, ref, V;
  IdBuf<int> piv;
  IdBuf<IdNode> dn;
  IdBuf<IdState> st;
  A.alloc(blocks.size());
  nrm.alloc((size_t)cols);
  ref.alloc((size_t)cols);
  piv.alloc((size_t)cols);
  V.alloc((size_t)rowsum);
  dn.alloc((size_t)nb);
  st.alloc((size_t)nb);
  ID_HIP(hipMemcpy(A.p, blocks.data(), blocks.size() * sizeof(double), hipMemcpyHostToDevice));
  ID_HIP(hipMemcpy(dn.p, nodes.data(), nodes.size() * sizeof(IdNode), hipMemcpyHostToDevice));
  if (nb > 65535) fail(GOFMM_ELIMIT, "too many nodes in one level");
  const int cblocks = (max_ncol + kIdThreads - 1) / kIdThreads;
  hipLaunchKernelGGL(id_norms, dim3(cblocks, nb), dim3(kIdThreads), 0, nullptr, dn.p, nb, A.p, nrm.p, ref.p, piv.p,
                     st.p);
  ID_HIP(hipGetLastError());
  const double tol3z = std::sqrt(DBL_EPSILON);
  for (int k = 0; k < max_k; ++k) {
    hipLaunchKernelGGL(id_pivot, dim3(nb), dim3(kIdThreads), 0, nullptr, dn.p, k, A.p, nrm.p, ref.p, piv.p, V.p,
                       st.p, tol);
    ID_HIP(hipGetLastError());
    const int tb = (max_ncol - k - 1 + kIdThreads - 1) / kIdThreads;
    if (tb > 0) {
      hipLaunchKernelGGL(id_update, dim3(tb, nb), dim3(kIdThreads), (size_t)(max_nrow - k) * sizeof(double),
                         nullptr, dn.p, k, A.p, nrm.p, ref.p, V.p, st.p, tol3z);
      ID_HIP(hipGetLastError());
    }
  }
  // nodes whose loop ran to kmax were marked by a step past it (or by the last one)
  hipLaunchKernelGGL(id_pivot, dim3(nb), dim3(kIdThreads), 0, nullptr, dn.p, max_k, A.p, nrm.p, ref.p, piv.p, V.p,
                     st.p, tol);
  ID_HIP(hipGetLastError());
  hipLaunchKernelGGL(id_solve, dim3(cblocks, nb), dim3(kIdThreads), 0, nullptr, dn.p, A.p, st.p);
  ID_HIP(hipGetLastError());
  ID_HIP(hipDeviceSynchronize());
  std::vector<IdState> hs(nb);
  std::vector<int> hp((size_t)cols);
  ID_HIP(hipMemcpy(hs.data(), st.p, nb * sizeof(IdState), hipMemcpyDeviceToHost));
  ID_HIP(hipMemcpy(hp.data(), piv.p, (size_t)cols * sizeof(int), hipMemcpyDeviceToHost));
  std::vector<double> rows;
  for (int q = 0; q < nb; ++q) {
    IdJob& jb = jobs[q];
    const int ncol = (int)jb.ncol, s = hs[q].rank;
    jb.rank = s;
    jb.piv.assign(hp.begin() + nodes[q].c_off, hp.begin() + nodes[q].c_off + ncol);
    jb.P.assign((size_t)s * ncol, 0.0);
    for (int i = 0; i < s; ++i) jb.P[(size_t)i * ncol + jb.piv[i]] = 1.0;
    if (hs[q].r00 == 0.0) continue;          // zero block: one column, no coefficients
    rows.resize((size_t)s * ncol);
    ID_HIP(hipMemcpy(rows.data(), A.p + nodes[q].a_off, rows.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int i = 0; i < s; ++i)
      for (int j = s; j < ncol; ++j) jb.P[(size_t)i * ncol + jb.piv[j]] = rows[(size_t)i * ncol + j];
  }
}

}  // namespace gofmm
