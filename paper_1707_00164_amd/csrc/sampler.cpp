// Ready-made entry sampler for radial kernels over a hidden point cloud.
//
// The method sees only K(I, J) (Sec. 1, problem statement); this sampler is an
// input convenience, not part of the method: it owns a copy of the points and
// returns FP64 kernel entries.  |x_i - x_j|^2 is summed coordinate by
// coordinate as (x_i - x_j)^2, so K(i, j) == K(j, i) bitwise.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "internal.hpp"

namespace {

constexpr unsigned kStateMagic = 0x6b65726eu;

struct KernelState {
  unsigned magic = kStateMagic;
  int kind;
  gofmm::i64 n;
  int dim;
  double h2inv;   // 1 / h^2
  double shift;
  std::vector<double> x;
};

inline double entry(const KernelState& s, gofmm::i64 i, gofmm::i64 j) {
  const double* a = &s.x[(size_t)i * s.dim];
  const double* b = &s.x[(size_t)j * s.dim];
  double d2 = 0.0;
  for (int c = 0; c < s.dim; ++c) {
    double t = a[c] - b[c];
    d2 += t * t;
  }
  double v;
  switch (s.kind) {
    case 0: v = std::exp(-0.5 * d2 * s.h2inv); break;
    case 1: v = 1.0 / std::sqrt(1.0 + d2 * s.h2inv); break;
    default: v = 1.0 / (std::sqrt(d2) + 0.05); break;
  }
  return i == j ? v + s.shift : v;
}

}  // namespace

namespace gofmm {

bool kernel_state_geo(const void* state, GeoKernel& out) {
  const KernelState* s = static_cast<const KernelState*>(state);
  if (!s || s->magic != kStateMagic || s->dim > kGeoDim) return false;
  out.kind = s->kind;
  out.dim = s->dim;
  out.h2inv = (float)s->h2inv;
  out.shift = (float)s->shift;
  out.pts.assign((size_t)s->n * kGeoStride, 0.0f);
  for (i64 i = 0; i < s->n; ++i) {
    float* e = &out.pts[(size_t)i * kGeoStride];
    for (int c = 0; c < s->dim; ++c) e[c] = (float)s->x[(size_t)i * s->dim + c];
    const int32_t idx = (int32_t)i;
    std::memcpy(&e[kGeoDim], &idx, sizeof(idx));
  }
  return true;
}

}  // namespace gofmm

extern "C" int gofmm_kernel_create(int32_t kind, int64_t n, int32_t dim, const double* points,
                                   double h, double shift, void** state) {
  if (!state || !points || n <= 0 || dim <= 0 || kind < 0 || kind > 2 ||
      (kind != 2 && !(h > 0.0)) || !std::isfinite(shift)) {
    gofmm::set_last_error("gofmm_kernel_create: invalid argument");
    return GOFMM_EINVAL;
  }
  KernelState* s = new (std::nothrow) KernelState;
  if (!s) { gofmm::set_last_error("gofmm_kernel_create: out of memory"); return GOFMM_ENOMEM; }
  try {
    s->kind = kind;
    s->n = n;
    s->dim = dim;
    s->h2inv = kind == 2 ? 0.0 : 1.0 / (h * h);
    s->shift = shift;
    s->x.assign(points, points + (size_t)n * dim);
  } catch (...) {
    delete s;
    gofmm::set_last_error("gofmm_kernel_create: out of memory");
    return GOFMM_ENOMEM;
  }
  *state = s;
  return GOFMM_OK;
}

extern "C" int gofmm_kernel_sample(void* state, int64_t nI, const int64_t* I, int64_t nJ,
                                   const int64_t* J, double* out, int64_t ld) {
  const KernelState* s = static_cast<const KernelState*>(state);
  if (!s || (nI && !I) || (nJ && !J) || !out || ld < nI) return 1;
  for (int64_t a = 0; a < nI; ++a)
    if (I[a] < 0 || I[a] >= s->n) return 2;
  for (int64_t b = 0; b < nJ; ++b) {
    if (J[b] < 0 || J[b] >= s->n) return 2;
    double* col = out + b * ld;                // column-major: out[a + b * ld]
    for (int64_t a = 0; a < nI; ++a) col[a] = entry(*s, I[a], J[b]);
  }
  return 0;
}

extern "C" void gofmm_kernel_free(void* state) {
  KernelState* s = static_cast<KernelState*>(state);
  if (s) s->magic = 0;
  delete s;
}
