// C ABI entry points: argument checks, error translation, ownership.
#include <omp.h>

#include <cmath>
#include <new>

#include "internal.hpp"

namespace gofmm {

static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }

void device_prepare(Compression& c, i64 r_max);
void device_evaluate(Compression& c, i64 r, const float* W, i64 ldw, float* U, i64 ldu, void* stream);
void device_evaluate_noalloc(Compression& c, i64 r, const float* W, i64 ldw, float* U, i64 ldu, void* stream);
void device_autotune(Compression& c, i64 r, const float* W, i64 ldw, float* U, i64 ldu, void* stream, int reps);
void device_evaluate_batched(int k, Compression* const* c, const i64* r, const float* const* W,
                             const i64* ldw, float* const* U, const i64* ldu, void* stream);
i64 device_footprint(const Compression& c, i64 r_max);
void device_profile(Compression& c, int on);
void device_autotune_batched(int k, Compression* const* c, const i64* r, const float* const* W,
                             const i64* ldw, float* const* U, const i64* ldu, void* stream, int reps);
int device_batched_status();
int device_pass_status(Compression& c);
void device_set_spin_limit(long long v);
void device_profile_read(Compression& c, int n, float* total_ms, int* calls);

}  // namespace gofmm


using namespace gofmm;

template <class F>
static int guarded(F body) {
  try {
    body();
    g_last_error.clear();
    return GOFMM_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("out of host memory");
    return GOFMM_ENOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return GOFMM_EINVAL;
  }
}

static void check_params(const gofmm_params* p) {
  if (!p) fail(GOFMM_EINVAL, "params is NULL");
  if (p->leaf_size < 1) fail(GOFMM_EINVAL, "leaf_size must be >= 1");
  if (p->max_rank < 1) fail(GOFMM_EINVAL, "max_rank must be >= 1");
  if (!(p->tol >= 0.0) || !std::isfinite(p->tol)) fail(GOFMM_EINVAL, "tol must be >= 0");
  if (p->kappa < 1) fail(GOFMM_EINVAL, "kappa must be >= 1");
  if (!(p->budget >= 0.0 && p->budget <= 1.0)) fail(GOFMM_EINVAL, "budget must be in [0, 1]");
  if (p->distance != GOFMM_GRAM_L2 && p->distance != GOFMM_ANGLE) fail(GOFMM_EINVAL, "unknown distance");
  for (int s : {p->storage, p->near_storage})
    if (s != GOFMM_FP32 && s != GOFMM_BF16 && s != GOFMM_BF16X3) fail(GOFMM_EINVAL, "unknown storage precision");
  if (p->threads < 0) fail(GOFMM_EINVAL, "threads must be >= 0");
  if (!(p->ann_target_recall >= 0.0 && p->ann_target_recall <= 1.0)) fail(GOFMM_EINVAL, "ann_target_recall in [0,1]");
  if (p->device_knn != 0 && p->device_knn != 1) fail(GOFMM_EINVAL, "device_knn must be 0 or 1");
  if (p->device_knn && p->kappa > 64) fail(GOFMM_EINVAL, "device_knn keeps at most 64 neighbours");
  if (p->device_id != 0 && p->device_id != 1) fail(GOFMM_EINVAL, "device_id must be 0 or 1");
}

extern "C" void gofmm_default_params(gofmm_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->leaf_size = 256;
  p->max_rank = 256;
  p->tol = 1e-5;
  p->kappa = 32;
  p->budget = 0.03;
  p->distance = GOFMM_GRAM_L2;
  p->storage = GOFMM_FP32;
  p->near_storage = GOFMM_FP32;
  p->seed = 1707;
  p->threads = 0;
  p->ann_max_iters = 10;
  p->ann_target_recall = 0.8;
  p->exact_knn = 0;
  p->device_knn = 0;
  p->device_id = 0;
}

extern "C" int gofmm_compress(int64_t n, gofmm_sampler sampler, void* user, const gofmm_params* params,
                              gofmm_compression** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (!out) fail(GOFMM_EINVAL, "out is NULL");
    if (n < 1) fail(GOFMM_EINVAL, "n must be >= 1");
    if (!sampler) fail(GOFMM_EINVAL, "sampler is NULL");
    check_params(params);
    std::unique_ptr<gofmm_compression> h(new gofmm_compression);
    Sampler K{sampler, user};
    h->c.n = n;
    build_compression(h->c, K, *params);
    build_plan(h->c, K, params->threads > 0 ? params->threads : omp_get_max_threads());
    *out = h.release();
  });
}

extern "C" int gofmm_import(const char* path, gofmm_sampler sampler, void* user, const gofmm_params* params,
                            gofmm_compression** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (!out || !path || !sampler) fail(GOFMM_EINVAL, "NULL argument");
    check_params(params);
    std::unique_ptr<gofmm_compression> h(new gofmm_compression);
    read_file(h->c, path);
    validate_structure(h->c);
    h->c.storage = params->storage;
    h->c.near_storage = params->near_storage;
    h->c.seed = params->seed;
    Sampler K{sampler, user};
    build_plan(h->c, K, params->threads > 0 ? params->threads : omp_get_max_threads());
    *out = h.release();
  });
}

extern "C" int gofmm_use_device_kernel(gofmm_compression* c, void* kernel_state, int32_t threads) {
  return guarded([&] {
    if (!c || !kernel_state) fail(GOFMM_EINVAL, "NULL argument");
    GeoKernel g;
    if (!kernel_state_geo(kernel_state, g))
      fail(GOFMM_EINVAL, "not a gofmm_kernel_create state, or points with more than 8 coordinates");
    if ((i64)(g.pts.size() / kGeoStride) != c->c.n) fail(GOFMM_EINVAL, "the kernel's point count differs from n");
    // Build the new plan next to the old one; a failure restores the old plan
    // and point set, and the device copy of the old plan stays valid.
    HostPlan old_plan = std::move(c->c.plan);
    GeoKernel old_geo = std::move(c->c.geo);
    c->c.geo = std::move(g);
    Sampler K{gofmm_kernel_sample, kernel_state};
    try {
      build_plan(c->c, K, threads > 0 ? threads : omp_get_max_threads());
    } catch (...) {
      c->c.plan = std::move(old_plan);
      c->c.geo = std::move(old_geo);
      throw;
    }
    if (c->c.dev) {                   // the plan changed: drop the old device copy
      device_state_free(c->c.dev);
      c->c.dev = nullptr;
    }
  });
}

extern "C" int gofmm_export(const gofmm_compression* c, const char* path) {
  return guarded([&] {
    if (!c || !path) fail(GOFMM_EINVAL, "NULL argument");
    write_file(c->c, path);
  });
}

extern "C" int gofmm_prepare(gofmm_compression* c, int64_t r_max) {
  return guarded([&] {
    if (!c) fail(GOFMM_EINVAL, "NULL compression");
    if (r_max < 1) fail(GOFMM_EINVAL, "r_max must be >= 1");
    device_prepare(c->c, r_max);
  });
}

static void check_eval(const gofmm_compression* c, int64_t r, const float* W, int64_t ldw, const float* U,
                       int64_t ldu) {
  if (!c) fail(GOFMM_EINVAL, "NULL compression");
  if (r < 0) fail(GOFMM_EINVAL, "r must be >= 0");
  if (r == 0) return;
  if (!W || !U) fail(GOFMM_EINVAL, "NULL W or U");
  if (ldw < r || ldu < r) fail(GOFMM_EINVAL, "leading dimension smaller than r");
  if (ldw > (int64_t)UINT32_MAX) fail(GOFMM_ELIMIT, "leading dimension of W above 2^32 - 1");
  const char* w0 = (const char*)W;
  const char* w1 = w0 + ((c->c.n - 1) * ldw + r) * 4;
  const char* u0 = (const char*)U;
  const char* u1 = u0 + ((c->c.n - 1) * ldu + r) * 4;
  if (w0 < u1 && u0 < w1) fail(GOFMM_EINVAL, "W and U overlap");
}

extern "C" int gofmm_evaluate(gofmm_compression* c, int64_t r, const float* W, int64_t ldw, float* U,
                              int64_t ldu, void* hip_stream) {
  return guarded([&] {
    check_eval(c, r, W, ldw, U, ldu);
    if (r == 0) return;
    device_evaluate(c->c, r, W, ldw, U, ldu, hip_stream);
  });
}

extern "C" int gofmm_evaluate_noalloc(gofmm_compression* c, int64_t r, const float* W, int64_t ldw, float* U,
                                      int64_t ldu, void* hip_stream) {
  return guarded([&] {
    check_eval(c, r, W, ldw, U, ldu);
    if (r == 0) return;
    device_evaluate_noalloc(c->c, r, W, ldw, U, ldu, hip_stream);
  });
}

extern "C" int gofmm_autotune(gofmm_compression* c, int64_t r, const float* W, int64_t ldw, float* U,
                              int64_t ldu, void* hip_stream) {
  return guarded([&] {
    check_eval(c, r, W, ldw, U, ldu);
    if (r == 0) return;
    device_autotune(c->c, r, W, ldw, U, ldu, hip_stream, 3);
  });
}

static std::vector<Compression*> batch_args(int32_t k, gofmm_compression* const* c, const int64_t* r,
                                            const float* const* W, const int64_t* ldw, float* const* U,
                                            const int64_t* ldu) {
  if (!c || !r || !W || !ldw || !U || !ldu) fail(GOFMM_EINVAL, "NULL argument");
  std::vector<Compression*> cs(k);
  for (int i = 0; i < k; ++i) {
    check_eval(c[i], r[i], W[i], ldw[i], U[i], ldu[i]);
    if (r[i] < 1) fail(GOFMM_EINVAL, "every instance of a batch needs r >= 1");
    for (int j = 0; j < i; ++j) {
      if (c[j] == c[i]) fail(GOFMM_EINVAL, "a compression appears twice in one batch");
      const char* a0 = (const char*)U[i];
      const char* a1 = a0 + ((c[i]->c.n - 1) * ldu[i] + r[i]) * 4;
      const char* b0 = (const char*)U[j];
      const char* b1 = b0 + ((c[j]->c.n - 1) * ldu[j] + r[j]) * 4;
      if (a0 < b1 && b0 < a1) fail(GOFMM_EINVAL, "outputs of two instances overlap");
    }
    cs[i] = &c[i]->c;
  }
  return cs;
}

extern "C" int gofmm_evaluate_batched(int32_t k, gofmm_compression* const* c, const int64_t* r,
                                      const float* const* W, const int64_t* ldw, float* const* U,
                                      const int64_t* ldu, void* hip_stream) {
  return guarded([&] {
    if (k < 0) fail(GOFMM_EINVAL, "k must be >= 0");
    if (k == 0) return;
    auto cs = batch_args(k, c, r, W, ldw, U, ldu);
    device_evaluate_batched(k, cs.data(), r, W, ldw, U, ldu, hip_stream);
  });
}

extern "C" int gofmm_autotune_batched(int32_t k, gofmm_compression* const* c, const int64_t* r,
                                      const float* const* W, const int64_t* ldw, float* const* U,
                                      const int64_t* ldu, void* hip_stream) {
  return guarded([&] {
    if (k < 0) fail(GOFMM_EINVAL, "k must be >= 0");
    if (k == 0) return;
    auto cs = batch_args(k, c, r, W, ldw, U, ldu);
    device_autotune_batched(k, cs.data(), r, W, ldw, U, ldu, hip_stream, 3);
  });
}

extern "C" int gofmm_batched_status(int32_t* error) {
  return guarded([&] {
    if (!error) fail(GOFMM_EINVAL, "NULL argument");
    *error = device_batched_status();
  });
}

extern "C" int gofmm_evaluate_status(gofmm_compression* c, int32_t* error) {
  return guarded([&] {
    if (!c || !error) fail(GOFMM_EINVAL, "NULL argument");
    *error = device_pass_status(c->c);
  });
}

extern "C" int gofmm_batched_spin_limit(int64_t polls) {
  return guarded([&] { device_set_spin_limit(polls); });
}

extern "C" int gofmm_launch_count(const gofmm_compression* c, int32_t* count) {
  return guarded([&] {
    if (!c || !count) fail(GOFMM_EINVAL, "NULL argument");
    *count = (int32_t)c->c.plan.launches.size();
  });
}

extern "C" int gofmm_launch_info(const gofmm_compression* c, int32_t i, char* name, int32_t name_len,
                                 double* flops_per_rhs, int64_t* operator_bytes) {
  return guarded([&] {
    if (!c) fail(GOFMM_EINVAL, "NULL compression");
    if (i < 0 || i >= (int32_t)c->c.plan.launches.size()) fail(GOFMM_EINVAL, "launch index out of range");
    const LaunchDesc& l = c->c.plan.launches[i];
    if (name && name_len > 0) {
      std::strncpy(name, l.name.c_str(), (size_t)name_len - 1);
      name[name_len - 1] = 0;
    }
    if (flops_per_rhs) *flops_per_rhs = l.flops;
    if (operator_bytes) *operator_bytes = l.bytes;
  });
}

extern "C" int gofmm_profile(gofmm_compression* c, int32_t enable) {
  return guarded([&] {
    if (!c) fail(GOFMM_EINVAL, "NULL compression");
    if (enable < 0 || (enable >= 2 && (size_t)(enable - 2) >= c->c.plan.launches.size()))
      fail(GOFMM_EINVAL, "profile mode out of range");
    device_profile(c->c, enable);
  });
}

extern "C" int gofmm_profile_read(gofmm_compression* c, int32_t n, float* total_ms, int32_t* calls) {
  return guarded([&] {
    if (!c || (n > 0 && (!total_ms || !calls))) fail(GOFMM_EINVAL, "NULL argument");
    device_profile_read(c->c, n, total_ms, calls);
  });
}

extern "C" int gofmm_footprint(const gofmm_compression* c, int64_t r_max, int64_t* bytes) {
  return guarded([&] {
    if (!c || !bytes) fail(GOFMM_EINVAL, "NULL argument");
    if (r_max < 1) fail(GOFMM_EINVAL, "r_max must be >= 1");
    *bytes = device_footprint(c->c, r_max);
  });
}

extern "C" int gofmm_stats(const gofmm_compression* c, gofmm_stats_t* out) {
  return guarded([&] {
    if (!c || !out) fail(GOFMM_EINVAL, "NULL argument");
    const Compression& x = c->c;
    std::memset(out, 0, sizeof(*out));
    out->n = x.n;
    out->depth = x.depth;
    out->n_leaves = x.n_leaves();
    out->n_nodes = x.nn();
    for (i64 h = 1; h < x.nn(); ++h) {
      out->rank_sum += x.rank(h);
      out->rank_max = std::max<int64_t>(out->rank_max, x.rank(h));
      out->far_pairs += (int64_t)x.far[h].size();
    }
    for (auto& l : x.near) out->near_pairs += (int64_t)l.size();
    out->flops_per_rhs = 0;
    for (int p = 0; p < 4; ++p) {
      out->flops_phase[p] = x.plan.flops_phase[p];
      out->flops_per_rhs += x.plan.flops_phase[p];
      out->operator_bytes_phase[p] = x.plan.bytes_phase[p];
    }
    out->operator_bytes = (int64_t)(x.plan.a_f32.size() * 4 + x.plan.a_b16.size() * 2 +
                                    x.plan.a_x3.size() * 2 + x.plan.geo_cols.size() * 4 +
                                    x.geo.pts.size() * 4);
    out->workspace_rows = x.plan.ws_rows;
  });
}

extern "C" void gofmm_free(gofmm_compression* c) { delete c; }

extern "C" const char* gofmm_last_error(void) { return g_last_error.c_str(); }
