// Serving loop: resident compressions, HBM admission, continuous batching.
//
// A host thread owns the device work.  Compressions ("models") are admitted
// in arrival order when their footprint (operator, workspace and two staging
// blocks of n x r_max) fits the HBM budget; until then their requests wait.
// Requests (model, W, U, r) arrive at any time.  Whenever a stream is free,
// the loop takes every admitted model that has pending requests and no work
// on the GPU (up to a batch limit, one storage precision per batch), packs each
// model's pending requests side by side as columns of one right-hand-side
// block (up to r_max columns; a lone request with suitable alignment is used
// in place), and evaluates all of them in one persistent batched launch.
// Up to `streams` batches are in flight at once, on different streams, with
// disjoint model sets (a model's workspace belongs to one launch at a time).
// Completion is detected with events; latency is measured from submission to
// detection.  The columns of a K~W do not interact and every output element
// is reduced in a fixed order, so a request's result does not depend on what
// it was batched with.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.hpp"

namespace gofmm {

void device_prepare(Compression& c, i64 r_max);
i64 device_footprint(const Compression& c, i64 r_max);
int device_batch_precision(Compression& c);
int device_batch_cfg(int k, Compression* const* c, const i64* r);
void batch_prepare(int k, Compression* const* c, const i64* r);
void ring_launch(BatchRing& ring, int k, Compression* const* c, const i64* r, const float* const* W,
                 const i64* ldw, float* const* U, const i64* ldu, hipStream_t st, int cfg);
int ring_status(BatchRing& ring);

#define SHIP_OK(expr)                                                               \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      fail(e_ == hipErrorOutOfMemory ? GOFMM_ENOMEM : GOFMM_EHIP,                   \
           std::string(#expr) + ": " + hipGetErrorString(e_));                      \
  } while (0)

static double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
  i64 id;
  int model;
  i64 r;
  const float* W;
  i64 ldw;
  float* U;
  i64 ldu;
  double t_submit = 0, t_done = 0;
  int state = 0;      // 0 pending, 1 in flight, 2 done, 3 failed
  std::string error;
};

struct Model {
  int id;
  Compression* c;
  i64 r_max;
  i64 footprint;
  bool admitted = false;
  bool admitting = false;   // its upload runs (outside the server lock)
  bool busy = false;
  bool removing = false;
  int prec = 0;
  float* Wc = nullptr;    // staging n x r_max (packed requests)
  float* Uc = nullptr;
  std::deque<Request*> pending;
};

struct Flight {
  int stream;
  std::vector<int> models;
  std::vector<std::vector<Request*>> reqs;
  void* ev = nullptr;
};

struct Server {
  int device = 0;
  i64 budget = 0, used = 0;
  int max_batch = 16;
  std::vector<hipStream_t> streams;
  std::vector<std::unique_ptr<BatchRing>> rings;
  std::vector<char> stream_busy;
  std::mutex mu;
  std::condition_variable cv, done_cv, admit_cv;
  bool stop = false, stop_admit = false;
  std::thread th, admitter;
  int admit_job = 0;        // model whose upload the admission thread runs
  int next_model = 1;
  i64 next_req = 1;
  std::map<int, std::unique_ptr<Model>> models;
  std::deque<int> admit_q;
  std::map<i64, std::unique_ptr<Request>> reqs;
  std::vector<Flight> flights;
  std::vector<double> lat;
  std::vector<double> lat_admitting;   // requests finished while an admission ran
  i64 completed = 0, failed = 0, batches = 0, columns = 0, packed = 0;
  i64 max_inflight = 0, admissions = 0;
  double host_ms = 0, admit_ms = 0;
  double t0 = now_ms(), busy_ms = 0;
  std::string fatal;

  void loop();
  void admit();
  void admit_loop();
  void retire();
  bool launch_one();
  void release_model(Model& m);
};

void Server::release_model(Model& m) {
  (void)hipFree(m.Wc);
  (void)hipFree(m.Uc);
  m.Wc = m.Uc = nullptr;
  if (m.c->dev) {
    device_state_free(m.c->dev);
    m.c->dev = nullptr;
  }
  if (m.admitted) used -= m.footprint;
  m.admitted = false;
}

// Admit queued models, in order, while they fit the budget.  The loop thread
// only reserves the footprint and hands the model to the admission thread;
// the upload (operator, tables, workspace, staging) runs there with the
// server lock released, so batches keep being retired and launched and
// requests keep arriving meanwhile.  The model is marked busy until its
// upload ends, so a removal waits for it.  One admission at a time.
void Server::admit() {
  if (admit_job || admit_q.empty()) return;
  Model& m = *models[admit_q.front()];
  if (used + m.footprint > budget) return;
  admit_q.pop_front();
  used += m.footprint;
  m.admitting = m.busy = true;
  admit_job = m.id;
  admit_cv.notify_all();
}

void Server::admit_loop() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  while (true) {
    admit_cv.wait(lk, [&] { return admit_job != 0 || stop_admit; });
    if (!admit_job) break;
    Model& m = *models[admit_job];
    const double ta = now_ms();
    std::string err;
    bool ok = true;
    lk.unlock();
    try {
      if (m.c->dev) {                 // drop any earlier device state: the server sizes it
        device_state_free(m.c->dev);
        m.c->dev = nullptr;
      }
      device_prepare(*m.c, m.r_max);
      SHIP_OK(hipMalloc((void**)&m.Wc, (size_t)m.c->n * m.r_max * sizeof(float)));
      SHIP_OK(hipMalloc((void**)&m.Uc, (size_t)m.c->n * m.r_max * sizeof(float)));
    } catch (const std::exception& e) {
      err = e.what();
      ok = false;
    }
    lk.lock();
    admit_ms += now_ms() - ta;
    m.admitting = m.busy = false;
    if (ok) {
      m.admitted = true;
      ++admissions;
    } else {
      // cannot be made resident: fail its requests
      used -= m.footprint;
      for (Request* q : m.pending) {
        q->state = 3;
        q->error = err;
        q->t_done = now_ms();
        ++failed;
      }
      m.pending.clear();
      release_model(m);
    }
    admit_job = 0;
    cv.notify_all();
    done_cv.notify_all();
  }
}

// Finish every flight whose event has completed.
void Server::retire() {
  for (size_t f = 0; f < flights.size();) {
    Flight& fl = flights[f];
    hipError_t q = hipEventQuery((hipEvent_t)fl.ev);
    if (q == hipErrorNotReady) { ++f; continue; }
    const int err = ring_status(*rings[fl.stream]);
    const double t = now_ms();
    for (size_t i = 0; i < fl.models.size(); ++i) {
      auto it = models.find(fl.models[i]);
      if (it != models.end()) it->second->busy = false;
      for (Request* r : fl.reqs[i]) {
        r->t_done = t;
        if (q != hipSuccess || err) {
          r->state = 3;
          r->error = q != hipSuccess ? hipGetErrorString(q) : "a dependency wait hit its poll bound";
          ++failed;
        } else {
          r->state = 2;
          lat.push_back(r->t_done - r->t_submit);
          if (admit_job) lat_admitting.push_back(r->t_done - r->t_submit);
          ++completed;
        }
      }
    }
    (void)hipEventDestroy((hipEvent_t)fl.ev);
    stream_busy[fl.stream] = 0;
    flights.erase(flights.begin() + f);
  }
  done_cv.notify_all();
}

// Form and launch one batch on a free stream; false if nothing to do.
bool Server::launch_one() {
  int si = -1;
  for (size_t s = 0; s < streams.size(); ++s)
    if (!stream_busy[s]) { si = (int)s; break; }
  if (si < 0) return false;
  std::vector<Model*> pick;
  int prec = -1;
  for (auto& kv : models) {
    Model& m = *kv.second;
    if (!m.admitted || m.busy || m.removing || m.pending.empty()) continue;
    if (prec >= 0 && m.prec != prec) continue;
    prec = m.prec;
    pick.push_back(&m);
    if ((int)pick.size() >= max_batch) break;
  }
  if (pick.empty()) return false;
  const double th = now_ms();
  hipStream_t st = streams[si];
  const int k = (int)pick.size();
  std::vector<Compression*> cs(k);
  std::vector<i64> r(k), ldw(k), ldu(k);
  std::vector<const float*> W(k);
  std::vector<float*> U(k);
  Flight fl;
  fl.stream = si;
  for (int i = 0; i < k; ++i) {
    Model& m = *pick[i];
    std::vector<Request*> take;
    i64 cols = 0;
    while (!m.pending.empty() && cols + m.pending.front()->r <= m.r_max) {
      take.push_back(m.pending.front());
      cols += m.pending.front()->r;
      m.pending.pop_front();
    }
    cs[i] = m.c;
    Request* q0 = take[0];
    const bool direct = take.size() == 1 && (uintptr_t)q0->W % 16 == 0 && (uintptr_t)q0->U % 16 == 0 &&
                        q0->ldw % 4 == 0 && q0->ldu % 4 == 0;
    if (direct) {
      r[i] = q0->r;
      W[i] = q0->W;
      ldw[i] = q0->ldw;
      U[i] = q0->U;
      ldu[i] = q0->ldu;
    } else {
      i64 off = 0;
      for (Request* q : take) {
        SHIP_OK(hipMemcpy2DAsync(m.Wc + off, m.r_max * sizeof(float), q->W, q->ldw * sizeof(float),
                                 q->r * sizeof(float), m.c->n, hipMemcpyDeviceToDevice, st));
        off += q->r;
      }
      r[i] = cols;
      W[i] = m.Wc;
      ldw[i] = m.r_max;
      U[i] = m.Uc;
      ldu[i] = m.r_max;
      ++packed;
    }
    for (Request* q : take) q->state = 1;
    m.busy = true;
    fl.models.push_back(m.id);
    fl.reqs.push_back(take);
    columns += cols;
  }
  batch_prepare(k, cs.data(), r.data());
  const int cfg = device_batch_cfg(k, cs.data(), r.data());
  ring_launch(*rings[si], k, cs.data(), r.data(), W.data(), ldw.data(), U.data(), ldu.data(), st, cfg);
  for (int i = 0; i < k; ++i) {
    if (W[i] != pick[i]->Wc) continue;
    i64 off = 0;
    for (Request* q : fl.reqs[i]) {
      SHIP_OK(hipMemcpy2DAsync(q->U, q->ldu * sizeof(float), pick[i]->Uc + off, pick[i]->r_max * sizeof(float),
                               q->r * sizeof(float), pick[i]->c->n, hipMemcpyDeviceToDevice, st));
      off += q->r;
    }
  }
  hipEvent_t ev;
  SHIP_OK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  SHIP_OK(hipEventRecord(ev, st));
  fl.ev = ev;
  stream_busy[si] = 1;
  flights.push_back(std::move(fl));
  max_inflight = std::max<i64>(max_inflight, (i64)flights.size());
  ++batches;
  host_ms += now_ms() - th;
  return true;
}

void Server::loop() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  while (true) {
    try {
      admit();
      retire();
      bool launched = false;
      while (launch_one()) launched = true;
      if (stop && flights.empty() && !admit_job) {
        bool pending = false;
        for (auto& kv : models) pending |= kv.second->admitted && !kv.second->pending.empty();
        if (!pending) break;
      }
      if (!launched) {
        if (flights.empty()) cv.wait_for(lk, std::chrono::milliseconds(2));
        else {
          lk.unlock();
          std::this_thread::sleep_for(std::chrono::microseconds(20));
          lk.lock();
        }
      }
    } catch (const std::exception& e) {
      // a device error: fail everything pending so no caller waits forever
      fatal = e.what();
      for (auto& kv : reqs)
        if (kv.second->state < 2) {
          kv.second->state = 3;
          kv.second->error = fatal;
          kv.second->t_done = now_ms();
          ++failed;
        }
      for (auto& kv : models) kv.second->pending.clear();
      flights.clear();
      done_cv.notify_all();
      if (stop) break;
      cv.wait_for(lk, std::chrono::milliseconds(2));
    }
  }
}

}  // namespace gofmm

using namespace gofmm;

struct gofmm_server {
  Server s;
};

template <class F>
static int sguard(F body) {
  try {
    body();
    return GOFMM_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return GOFMM_EINVAL;
  }
}

extern "C" int gofmm_server_create(int64_t hbm_budget, int32_t streams, int32_t max_batch, gofmm_server** out) {
  if (out) *out = nullptr;
  return sguard([&] {
    if (!out) fail(GOFMM_EINVAL, "out is NULL");
    if (hbm_budget <= 0 || streams < 1 || streams > 16 || max_batch < 1) fail(GOFMM_EINVAL, "bad server parameters");
    std::unique_ptr<gofmm_server> h(new gofmm_server);
    Server& s = h->s;
    SHIP_OK(hipGetDevice(&s.device));
    s.budget = hbm_budget;
    s.max_batch = max_batch;
    for (int i = 0; i < streams; ++i) {
      hipStream_t st;
      SHIP_OK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      s.streams.push_back(st);
      s.rings.emplace_back(new BatchRing);
      s.stream_busy.push_back(0);
    }
    s.th = std::thread([&s] { s.loop(); });
    s.admitter = std::thread([&s] { s.admit_loop(); });
    *out = h.release();
  });
}

extern "C" int gofmm_server_add(gofmm_server* h, gofmm_compression* c, int64_t r_max, int32_t* model) {
  return sguard([&] {
    if (!h || !c || !model) fail(GOFMM_EINVAL, "NULL argument");
    if (r_max < 1) fail(GOFMM_EINVAL, "r_max must be >= 1");
    if (c->c.geo.kind >= 0) fail(GOFMM_EINVAL, "compressions with device-computed near blocks are not served");
    Server& s = h->s;
    std::lock_guard<std::mutex> g(s.mu);
    for (auto& kv : s.models)
      if (kv.second->c == &c->c) fail(GOFMM_EINVAL, "compression already served");
    std::unique_ptr<Model> m(new Model);
    m->id = s.next_model++;
    m->c = &c->c;
    m->r_max = r_max;
    m->prec = device_batch_precision(c->c);
    m->footprint = device_footprint(c->c, r_max) + 2 * c->c.n * r_max * (i64)sizeof(float);
    if (m->footprint > s.budget) fail(GOFMM_ENOMEM, "compression footprint exceeds the server's HBM budget");
    *model = m->id;
    s.admit_q.push_back(m->id);
    s.models[m->id] = std::move(m);
    s.cv.notify_all();
  });
}

extern "C" int gofmm_server_remove(gofmm_server* h, int32_t model) {
  return sguard([&] {
    if (!h) fail(GOFMM_EINVAL, "NULL server");
    Server& s = h->s;
    std::unique_lock<std::mutex> lk(s.mu);
    auto it = s.models.find(model);
    if (it == s.models.end()) fail(GOFMM_EINVAL, "unknown model");
    Model& m = *it->second;
    m.removing = true;
    s.done_cv.wait(lk, [&] { return !m.busy || !s.fatal.empty(); });
    for (Request* q : m.pending) {
      q->state = 3;
      q->error = "model removed";
      q->t_done = now_ms();
      ++s.failed;
    }
    m.pending.clear();
    s.admit_q.erase(std::remove(s.admit_q.begin(), s.admit_q.end(), model), s.admit_q.end());
    s.release_model(m);
    s.models.erase(it);
    s.cv.notify_all();
    s.done_cv.notify_all();
  });
}

extern "C" int gofmm_server_submit(gofmm_server* h, int32_t model, int64_t r, const float* W, int64_t ldw,
                                   float* U, int64_t ldu, int64_t* request) {
  return sguard([&] {
    if (!h || !W || !U || !request) fail(GOFMM_EINVAL, "NULL argument");
    Server& s = h->s;
    const double t_submit = now_ms();     // before waiting for the lock
    std::lock_guard<std::mutex> g(s.mu);
    auto it = s.models.find(model);
    if (it == s.models.end() || it->second->removing) fail(GOFMM_EINVAL, "unknown model");
    Model& m = *it->second;
    if (r < 1 || r > m.r_max) fail(GOFMM_EINVAL, "r must be in [1, r_max]");
    if (ldw < r || ldu < r) fail(GOFMM_EINVAL, "leading dimension smaller than r");
    if (ldw > (int64_t)UINT32_MAX) fail(GOFMM_ELIMIT, "leading dimension of W above 2^32 - 1");
    std::unique_ptr<Request> q(new Request);
    q->id = s.next_req++;
    q->model = model;
    q->r = r;
    q->W = W;
    q->ldw = ldw;
    q->U = U;
    q->ldu = ldu;
    q->t_submit = t_submit;
    m.pending.push_back(q.get());
    *request = q->id;
    s.reqs[q->id] = std::move(q);
    s.cv.notify_all();
  });
}

static int finish_request(Server& s, std::map<i64, std::unique_ptr<Request>>::iterator it, double* latency_ms) {
  Request& q = *it->second;
  if (latency_ms) *latency_ms = q.t_done - q.t_submit;
  const int ok = q.state == 2;
  const std::string err = q.error;
  s.reqs.erase(it);
  if (!ok) fail(GOFMM_EHIP, "request failed: " + err);
  return 0;
}

extern "C" int gofmm_server_wait(gofmm_server* h, int64_t request, int64_t timeout_ms, double* latency_ms) {
  return sguard([&] {
    if (!h) fail(GOFMM_EINVAL, "NULL server");
    Server& s = h->s;
    std::unique_lock<std::mutex> lk(s.mu);
    auto it = s.reqs.find(request);
    if (it == s.reqs.end()) fail(GOFMM_EINVAL, "unknown request");
    auto ready = [&] { return it->second->state >= 2; };
    if (timeout_ms > 0) {
      if (!s.done_cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready))
        fail(GOFMM_ETIMEDOUT, "request not finished within the timeout");
    } else {
      s.done_cv.wait(lk, ready);
    }
    finish_request(s, it, latency_ms);
  });
}

extern "C" int gofmm_server_test(gofmm_server* h, int64_t request, int32_t* done, double* latency_ms) {
  return sguard([&] {
    if (!h || !done) fail(GOFMM_EINVAL, "NULL argument");
    Server& s = h->s;
    std::lock_guard<std::mutex> g(s.mu);
    auto it = s.reqs.find(request);
    if (it == s.reqs.end()) fail(GOFMM_EINVAL, "unknown request");
    *done = it->second->state >= 2;
    if (*done) finish_request(s, it, latency_ms);
  });
}

extern "C" int gofmm_server_stats(gofmm_server* h, gofmm_server_stats_t* out) {
  return sguard([&] {
    if (!h || !out) fail(GOFMM_EINVAL, "NULL argument");
    Server& s = h->s;
    std::lock_guard<std::mutex> g(s.mu);
    std::memset(out, 0, sizeof(*out));
    out->completed = s.completed;
    out->failed = s.failed;
    out->batches = s.batches;
    out->columns = s.columns;
    out->packed = s.packed;
    for (auto& kv : s.models) {
      out->models += kv.second->admitted;
      out->admit_queue += !kv.second->admitted;
      out->pending += (int64_t)kv.second->pending.size();
    }
    out->inflight = (int64_t)s.flights.size();
    out->hbm_used = s.used;
    out->hbm_budget = s.budget;
    if (!s.lat.empty()) {
      std::vector<double> v(s.lat);
      std::sort(v.begin(), v.end());
      auto pct = [&](double p) { return v[std::min(v.size() - 1, (size_t)(p * (double)(v.size() - 1) + 0.5))]; };
      out->p50_ms = pct(0.50);
      out->p99_ms = pct(0.99);
      out->max_ms = v.back();
      double sum = 0;
      for (double x : v) sum += x;
      out->mean_ms = sum / (double)v.size();
    }
    out->elapsed_ms = now_ms() - s.t0;
    out->max_inflight = s.max_inflight;
    out->admissions = s.admissions;
    out->host_ms_mean = s.batches ? s.host_ms / (double)s.batches : 0.0;
    out->admit_ms_mean = s.admissions ? s.admit_ms / (double)s.admissions : 0.0;
    if (!s.lat_admitting.empty()) {
      std::vector<double> v(s.lat_admitting);
      std::sort(v.begin(), v.end());
      out->p99_ms_admitting = v[std::min(v.size() - 1, (size_t)(0.99 * (double)(v.size() - 1) + 0.5))];
    }
  });
}

extern "C" int gofmm_server_reset_stats(gofmm_server* h) {
  return sguard([&] {
    if (!h) fail(GOFMM_EINVAL, "NULL server");
    Server& s = h->s;
    std::lock_guard<std::mutex> g(s.mu);
    s.lat.clear();
    s.lat_admitting.clear();
    s.completed = s.failed = s.batches = s.columns = s.packed = 0;
    s.max_inflight = s.admissions = 0;
    s.host_ms = s.admit_ms = 0;
    s.t0 = now_ms();
  });
}

extern "C" void gofmm_server_destroy(gofmm_server* h) {
  if (!h) return;
  Server& s = h->s;
  {
    std::lock_guard<std::mutex> g(s.mu);
    s.stop = true;
    s.cv.notify_all();
  }
  if (s.th.joinable()) s.th.join();
  {
    std::lock_guard<std::mutex> g(s.mu);
    s.stop_admit = true;
    s.admit_cv.notify_all();
  }
  if (s.admitter.joinable()) s.admitter.join();
  (void)hipSetDevice(s.device);
  for (auto& kv : s.models) s.release_model(*kv.second);
  s.rings.clear();
  for (hipStream_t st : s.streams) (void)hipStreamDestroy(st);
  delete h;
}
