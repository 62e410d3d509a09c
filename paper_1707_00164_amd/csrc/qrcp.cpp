// Interpolative decomposition by Householder QR with column pivoting, FP64.
//
// The skeletonization of a node (Sec. 2.2, "Low-rank approximation", eqs. 7-8)
// factors the sampled block A = K(I', cols) as A Pi = Q [R11 R12; 0 R22]
// (Businger-Golub column pivoting: the column of largest residual norm is
// taken next), keeps the first s pivots as skeletons and sets
// P = [I, R11^{-1} R12] Pi^T, so that A ~= A(:, skeleton) P.
//
// Rank: s is the smallest k >= 1 with |R_kk| < tol * |R_00|, at most
// min(smax, ncol, nrow); the factorization stops there, so only s
// Householder steps are paid for.  Residual column norms are downdated after
// each step and recomputed when more than half of their digits cancelled
// (the safeguard LAPACK's xGEQP3 uses).
#include <algorithm>
#include <cmath>
#include <limits>

#include "internal.hpp"

namespace gofmm {

int interp_decomp(double* A, int nrow, int ncol, double tol, int smax,
                  std::vector<int>& piv, std::vector<double>& P) {
  const size_t ld = (size_t)nrow;
  double* C = A;                                       // factored in place, column-major
  piv.resize(ncol);
  for (int j = 0; j < ncol; ++j) piv[j] = j;
  std::vector<double> nrm(ncol), ref(ncol);
  for (int j = 0; j < ncol; ++j) {
    const double* c = &C[(size_t)j * ld];
    double t = 0.0;
    for (int i = 0; i < nrow; ++i) t += c[i] * c[i];
    nrm[j] = ref[j] = t;
  }
  const int kmax = std::max(1, std::min(std::min(smax, ncol), nrow));
  const double tol3z = std::sqrt(std::numeric_limits<double>::epsilon());
  double r00 = 0.0;
  int s = kmax;
  std::vector<double> v(nrow);
  for (int k = 0; k < kmax; ++k) {
    int p = k;
    for (int j = k + 1; j < ncol; ++j)
      if (nrm[j] > nrm[p]) p = j;
    if (p != k) {
      std::swap_ranges(&C[(size_t)k * ld], &C[(size_t)k * ld] + nrow, &C[(size_t)p * ld]);
      std::swap(nrm[k], nrm[p]);
      std::swap(ref[k], ref[p]);
      std::swap(piv[k], piv[p]);
    }
    double* ck = &C[(size_t)k * ld];
    double xn = 0.0;
    for (int i = k; i < nrow; ++i) xn += ck[i] * ck[i];
    xn = std::sqrt(xn);
    if (k == 0) {
      r00 = xn;
      if (r00 == 0.0) {           // the whole block is zero: keep one column, no coefficients
        P.assign((size_t)ncol, 0.0);
        P[piv[0]] = 1.0;
        return 1;
      }
    } else if (xn < tol * r00) {
      s = k;
      break;
    }
    // Householder reflector H = I - beta v v^T with H x = alpha e_k
    const double alpha = ck[k] >= 0.0 ? -xn : xn;
    for (int i = k; i < nrow; ++i) v[i] = ck[i];
    v[k] -= alpha;
    double vv = 0.0;
    for (int i = k; i < nrow; ++i) vv += v[i] * v[i];
    const double beta = vv > 0.0 ? 2.0 / vv : 0.0;
    ck[k] = alpha;
    for (int i = k + 1; i < nrow; ++i) ck[i] = 0.0;
    for (int j = k + 1; j < ncol; ++j) {
      double* cj = &C[(size_t)j * ld];
      double d = 0.0;
      for (int i = k; i < nrow; ++i) d += v[i] * cj[i];
      d *= beta;
      for (int i = k; i < nrow; ++i) cj[i] -= d * v[i];
      // downdate the residual norm of column j
      const double rkj = cj[k];
      double nj = nrm[j] - rkj * rkj;
      if (nj <= tol3z * ref[j] || nj < 0.0) {
        nj = 0.0;
        for (int i = k + 1; i < nrow; ++i) nj += cj[i] * cj[i];
        ref[j] = nj;
      }
      nrm[j] = nj;
    }
  }
  // T = R11^{-1} R12 by back substitution; R(i, j) = C[j * ld + i] for i <= j
  P.assign((size_t)s * ncol, 0.0);
  for (int i = 0; i < s; ++i) P[(size_t)i * ncol + piv[i]] = 1.0;
  std::vector<double> t(s);
  for (int j = s; j < ncol; ++j) {
    const double* cj = &C[(size_t)j * ld];
    for (int i = s - 1; i >= 0; --i) {
      double acc = cj[i];
      for (int q = i + 1; q < s; ++q) acc -= C[(size_t)q * ld + i] * t[q];
      t[i] = acc / C[(size_t)i * ld + i];
    }
    for (int i = 0; i < s; ++i) P[(size_t)i * ncol + piv[j]] = t[i];
  }
  return s;
}

uint16_t to_bf16(double x) {
  float f = (float)x;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  if ((u & 0xffffu) == 0x8000u && (double)f != x) {
    // a tie after rounding to float that was not a tie for x: round toward x
    const bool away = std::fabs(x) > std::fabs((double)f);
    return (uint16_t)((u >> 16) + (away ? 1u : 0u));
  }
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

double from_bf16(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return (double)f;
}

}  // namespace gofmm
