// Host-side compression (Alg. "Compress" of Sec. 2.2), FP64 throughout.
//
//   1. diagonal K_ii, checked positive and finite (the matrix must be SPD);
//   2. kappa nearest neighbours by the iterative randomized-tree search of
//      Sec. 2.2 ("Index nearest neighbor list"): each iteration splits the
//      index set with random poles p, q down to leaves of size m, searches
//      each leaf exhaustively, and merges; stop at the target recall measured
//      on seeded probe indices against their brute-force neighbours, or after
//      ann_max_iters trees.  (Optionally exact brute force.)
//   3. the ball tree by metricSplit (Alg. 1) with Gram distances (eqs. 3, 4);
//   4. Near lists by LeafNear with the ballot and budget (Alg. 2, eq.
//      budget), made symmetric; Far lists by FindFar (Alg. 3) and MergeFar
//      (Alg. 4), then refined so that the far pairs are closed under
//      transposition, which makes K~ exactly symmetric;
//   5. nested interpolative decompositions in postorder (Alg. 5).
// The cached blocks (Kba, SKba) are sampled by the packer.
#include <omp.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>
#include <numeric>
#include <unordered_set>

#include "internal.hpp"

namespace gofmm {

namespace {

// Run body(i) for i in [0, n) on up to `threads` threads; rethrow the first error.
template <class F>
void parallel_for(i64 n, int threads, F body) {
  std::mutex mu;
  bool failed = false;
  int code = 0;
  std::string msg;
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads)
  for (i64 i = 0; i < n; ++i) {
    bool skip;
    {
      std::lock_guard<std::mutex> g(mu);
      skip = failed;
    }
    if (skip) continue;
    try {
      body(i);
    } catch (const Error& e) {
      std::lock_guard<std::mutex> g(mu);
      if (!failed) { failed = true; code = e.code; msg = e.what(); }
    } catch (const std::bad_alloc&) {
      std::lock_guard<std::mutex> g(mu);
      if (!failed) { failed = true; code = GOFMM_ENOMEM; msg = "out of host memory"; }
    } catch (const std::exception& e) {
      std::lock_guard<std::mutex> g(mu);
      if (!failed) { failed = true; code = GOFMM_EINVAL; msg = e.what(); }
    }
  }
  if (failed) fail(code, msg);
}

// Sample K(I, J) (column-major nI x nJ, leading dimension nI), splitting rows
// over threads when large.
void sample(const Sampler& K, const i64* I, i64 nI, const i64* J, i64 nJ, double* out, int threads) {
  const i64 chunk = std::max<i64>(1, (1 << 16) / std::max<i64>(1, nJ));
  const i64 nchunks = (nI + chunk - 1) / chunk;
  if (nchunks <= 1 || omp_in_parallel() || threads <= 1) {
    K(nI, I, nJ, J, out, nI);
    return;
  }
  parallel_for(nchunks, threads, [&](i64 c) {
    const i64 a = c * chunk, b = std::min(nI, a + chunk);
    K(b - a, I + a, nJ, J, out + a, nI);
  });
}

struct Dist {
  const Sampler& K;
  const std::vector<double>& diag;
  int kind;
  int threads;
  double from(double kij, i64 i, i64 j) const {
    if (kind == GOFMM_GRAM_L2) return std::sqrt(std::max(0.0, diag[i] + diag[j] - 2.0 * kij));
    double d = 1.0 - kij * kij / (diag[i] * diag[j]);
    return std::min(1.0, std::max(0.0, d));
  }
  // d(I[t], p) for all t
  void to_point(const i64* I, i64 n, i64 p, double* out) const {
    sample(K, I, n, &p, 1, out, threads);
    for (i64 t = 0; t < n; ++t) out[t] = from(out[t], I[t], p);
  }
};

// Split `idx` (ascending) into the ceil(n/2) smallest and the rest of v (ties by index).
void median_split(const std::vector<i64>& idx, const std::vector<double>& v,
                  std::vector<i64>& left, std::vector<i64>& right) {
  const i64 n = (i64)idx.size();
  std::vector<i64> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](i64 a, i64 b) {
    if (v[a] != v[b]) return v[a] < v[b];
    return idx[a] < idx[b];
  });
  const i64 nl = (n + 1) / 2;
  left.clear();
  right.clear();
  for (i64 t = 0; t < n; ++t) (t < nl ? left : right).push_back(idx[ord[t]]);
  std::sort(left.begin(), left.end());
  std::sort(right.begin(), right.end());
}

// Alg. 1 (metricSplit) with a centroid of n_c = min(n, 32) sampled Gram vectors.
void metric_split(const Dist& d, const std::vector<i64>& idx, Rng& rng, std::vector<i64>& left,
                  std::vector<i64>& right, i64& p, i64& q, std::vector<i64>& cent) {
  const i64 n = (i64)idx.size();
  const i64 nc = std::min<i64>(n, 32);
  std::vector<i64> pool(idx);
  for (i64 t = 0; t < nc; ++t) std::swap(pool[t], pool[t + (i64)rng.below(n - t)]);
  cent.assign(pool.begin(), pool.begin() + nc);
  std::sort(cent.begin(), cent.end());
  std::vector<double> kic((size_t)n * nc);
  sample(d.K, idx.data(), n, cent.data(), nc, kic.data(), d.threads);
  std::vector<double> dc(n);
  if (d.kind == GOFMM_GRAM_L2) {
    for (i64 t = 0; t < n; ++t) {
      double s = 0.0;
      for (i64 j = 0; j < nc; ++j) s += kic[t + j * n];
      dc[t] = d.diag[idx[t]] - 2.0 * s / nc;        // |phi_i - c|^2 minus |c|^2
    }
  } else {
    std::vector<double> kcc((size_t)nc * nc);
    sample(d.K, cent.data(), nc, cent.data(), nc, kcc.data(), 1);
    double cc = 0.0;
    for (double x : kcc) cc += x;
    cc /= (double)(nc * nc);
    for (i64 t = 0; t < n; ++t) {
      double s = 0.0;
      for (i64 j = 0; j < nc; ++j) s += kic[t + j * n];
      s /= nc;
      dc[t] = 1.0 - s * s / (d.diag[idx[t]] * cc);
    }
  }
  i64 a = 0;
  for (i64 t = 1; t < n; ++t) if (dc[t] > dc[a]) a = t;
  p = idx[a];
  std::vector<double> dp(n), dq(n);
  d.to_point(idx.data(), n, p, dp.data());
  a = 0;
  for (i64 t = 1; t < n; ++t) if (dp[t] > dp[a]) a = t;
  q = idx[a];
  d.to_point(idx.data(), n, q, dq.data());
  std::vector<double> v(n);
  for (i64 t = 0; t < n; ++t) v[t] = dp[t] - dq[t];
  median_split(idx, v, left, right);
}

// Random-projection split for the neighbour search: random distinct poles.
void random_split(const Dist& d, const std::vector<i64>& idx, Rng& rng, std::vector<i64>& left,
                  std::vector<i64>& right) {
  const i64 n = (i64)idx.size();
  const i64 a = (i64)rng.below(n);
  i64 b = (i64)rng.below(n - 1);
  if (b >= a) ++b;
  std::vector<double> dp(n), dq(n), v(n);
  d.to_point(idx.data(), n, idx[a], dp.data());
  d.to_point(idx.data(), n, idx[b], dq.data());
  for (i64 t = 0; t < n; ++t) v[t] = dp[t] - dq[t];
  median_split(idx, v, left, right);
}

// Leaves (index sets) of a balanced tree of `depth` levels built by `split`.
template <class SplitFn>
std::vector<std::vector<i64>> build_levels(i64 n, int depth, int threads, SplitFn split,
                                           std::vector<std::vector<i64>>* all_nodes) {
  std::vector<std::vector<i64>> cur(1);
  cur[0].resize(n);
  std::iota(cur[0].begin(), cur[0].end(), 0);
  if (all_nodes) all_nodes->push_back(cur[0]);
  i64 base = 0;
  for (int lev = 0; lev < depth; ++lev) {
    std::vector<std::vector<i64>> nxt(cur.size() * 2);
    const int th = cur.size() >= (size_t)threads ? threads : 1;
    parallel_for((i64)cur.size(), th, [&](i64 t) {
      split(base + t, cur[t], nxt[2 * t], nxt[2 * t + 1]);
    });
    base += (i64)cur.size();
    cur.swap(nxt);
    if (all_nodes)
      for (auto& x : cur) all_nodes->push_back(x);
  }
  return cur;
}

struct Cand {
  double d;
  i64 j;
  bool operator<(const Cand& o) const { return d != o.d ? d < o.d : j < o.j; }
};

// Merge candidates into the sorted kappa-list of index i (unique indices).
void merge_list(i64* ki, double* kd, int kappa, std::vector<Cand>& cand) {
  if ((i64)cand.size() > kappa) {
    std::nth_element(cand.begin(), cand.begin() + kappa, cand.end());
    cand.resize(kappa);
  }
  std::sort(cand.begin(), cand.end());
  std::vector<Cand> out;
  out.reserve(2 * kappa);
  int a = 0;
  size_t b = 0;
  while ((int)out.size() < kappa && (a < kappa || b < cand.size())) {
    Cand x;
    if (a < kappa && ki[a] >= 0 && (b >= cand.size() || Cand{kd[a], ki[a]} < cand[b])) {
      x = {kd[a], ki[a]};
      ++a;
    } else if (b < cand.size()) {
      x = cand[b++];
    } else {
      break;
    }
    bool dup = false;
    for (auto& y : out) if (y.j == x.j) { dup = true; break; }
    if (!dup) out.push_back(x);
    if (a < kappa && ki[a] < 0) a = kappa;     // rest of the old list is empty
  }
  for (int t = 0; t < kappa; ++t) {
    if (t < (int)out.size()) { ki[t] = out[t].j; kd[t] = out[t].d; }
    else { ki[t] = -1; kd[t] = INFINITY; }
  }
}

void exact_neighbours(const Dist& d, i64 n, const i64* rows, i64 nrows, int kappa, i64* out,
                      int threads) {
  std::vector<i64> all(n);
  std::iota(all.begin(), all.end(), 0);
  parallel_for(nrows, threads, [&](i64 t) {
    const i64 i = rows[t];
    std::vector<double> k(n);
    d.K(1, &i, n, all.data(), k.data());
    std::vector<Cand> c(n);
    for (i64 j = 0; j < n; ++j) c[j] = {d.from(k[j], i, j), j};
    std::partial_sort(c.begin(), c.begin() + kappa, c.end());
    for (int a = 0; a < kappa; ++a) out[t * kappa + a] = c[a].j;
  });
}

// The sampled blocks K(rows, cols) of `sets`, merged into the device lists
// in batches of at most kKnnBatch entries (each batch sampled on the host by
// the compression's threads, one block per thread).
struct KnnSet { const i64* rows; i64 nr; const i64* cols; i64 nc; };
constexpr size_t kKnnBatch = (size_t)32 << 20;

void knn_merge_sets(KnnDevice* kd, const Dist& d, const std::vector<KnnSet>& sets) {
  size_t q = 0;
  while (q < sets.size()) {
    std::vector<KnnTask> tasks;
    std::vector<int> idx;
    size_t tot = 0;
    const size_t q0 = q;
    while (q < sets.size() && (q == q0 || tot + (size_t)(sets[q].nr * sets[q].nc) <= kKnnBatch)) {
      const KnnSet& s = sets[q];
      KnnTask t{(i64)tot, (i64)idx.size(), s.nr, 0, s.nc};
      for (i64 a = 0; a < s.nr; ++a) idx.push_back((int)s.rows[a]);
      if (s.cols == s.rows && s.nc == s.nr) {
        t.cofs = t.rofs;
      } else {
        t.cofs = (i64)idx.size();
        for (i64 a = 0; a < s.nc; ++a) idx.push_back((int)s.cols[a]);
      }
      tasks.push_back(t);
      tot += (size_t)(s.nr * s.nc);
      ++q;
    }
    std::vector<double> blocks(tot);
    parallel_for((i64)tasks.size(), d.threads, [&](i64 t) {
      const KnnSet& s = sets[q0 + t];
      d.K(s.nr, s.rows, s.nc, s.cols, &blocks[tasks[t].kofs]);
    });
    knn_device_merge(kd, tasks, idx, blocks);
  }
}

// Recall of the lists on the probes against their exact neighbours.
double knn_recall(const Compression& c, const std::vector<i64>& probes, const std::vector<i64>& truth, int kappa) {
  i64 hit = 0;
  const i64 np = (i64)probes.size();
  for (i64 t = 0; t < np; ++t) {
    const i64* a = &c.knn[(size_t)probes[t] * kappa];
    for (int u = 0; u < kappa; ++u)
      for (int v = 0; v < kappa; ++v)
        if (a[v] == truth[t * kappa + u]) { ++hit; break; }
  }
  return (double)hit / (double)(np * kappa);
}

void neighbours(Compression& c, const Dist& d, const gofmm_params& p) {
  const i64 n = c.n;
  const int kappa = (int)std::min<i64>(p.kappa, n);
  c.knn_k = kappa;
  c.knn.assign((size_t)n * kappa, -1);
  std::vector<i64> all(n);
  std::iota(all.begin(), all.end(), 0);
  // device merges: the same trees, blocks and (distance, index) rule as the
  // host path below, so the same lists
  std::unique_ptr<KnnDevice, void (*)(KnnDevice*)> dev(nullptr, knn_device_free);
  if (p.device_knn) dev.reset(knn_device_create(n, kappa, d.kind, d.diag.data()));
  if (p.exact_knn && dev) {
    const i64 R = std::max<i64>(1, std::min<i64>(64, (i64)(kKnnBatch / 4) / n));
    std::vector<KnnSet> sets;
    for (i64 r0 = 0; r0 < n; r0 += R) sets.push_back({&all[r0], std::min(R, n - r0), all.data(), n});
    knn_merge_sets(dev.get(), d, sets);
    knn_device_read(dev.get(), c.knn.data());
    return;
  }
  if (p.exact_knn) {
    exact_neighbours(d, n, all.data(), n, kappa, c.knn.data(), d.threads);
    return;
  }
  std::vector<double> kd((size_t)n * kappa, INFINITY);
  // probes and their exact neighbours for the recall estimate
  Rng pr(mix(c.seed, 0xA11));
  const i64 np = std::min<i64>(n, 128);
  std::vector<i64> probes(all);
  for (i64 t = 0; t < np; ++t) std::swap(probes[t], probes[t + (i64)pr.below(n - t)]);
  probes.resize(np);
  std::vector<i64> truth((size_t)np * kappa);
  exact_neighbours(d, n, probes.data(), np, kappa, truth.data(), d.threads);
  const i64 leaf = std::max<i64>(c.leaf_size, 2 * (i64)kappa);
  const int depth = choose_depth(n, leaf);
  const int iters = std::max(1, p.ann_max_iters);
  for (int it = 0; it < iters; ++it) {
    auto leaves = build_levels(n, depth, d.threads,
        [&](i64 h, const std::vector<i64>& idx, std::vector<i64>& l, std::vector<i64>& r) {
          Rng rng(mix(mix(c.seed, 0xB0B + it), h));
          random_split(d, idx, rng, l, r);
        }, nullptr);
    if (dev) {
      std::vector<KnnSet> sets;
      for (const auto& idx : leaves) sets.push_back({idx.data(), (i64)idx.size(), idx.data(), (i64)idx.size()});
      knn_merge_sets(dev.get(), d, sets);
      knn_device_read(dev.get(), c.knn.data());
      if (knn_recall(c, probes, truth, kappa) >= p.ann_target_recall) break;
      continue;
    }
    parallel_for((i64)leaves.size(), d.threads, [&](i64 b) {
      const auto& idx = leaves[b];
      const i64 m = (i64)idx.size();
      std::vector<double> blk((size_t)m * m);
      d.K(m, idx.data(), m, idx.data(), blk.data());
      std::vector<Cand> cand(m);
      for (i64 a = 0; a < m; ++a) {
        const i64 i = idx[a];
        cand.resize(m);
        for (i64 t = 0; t < m; ++t) cand[t] = {d.from(blk[a + t * m], i, idx[t]), idx[t]};
        merge_list(&c.knn[(size_t)i * kappa], &kd[(size_t)i * kappa], kappa, cand);
      }
    });
    if (knn_recall(c, probes, truth, kappa) >= p.ann_target_recall) break;
  }
}

}  // namespace

int choose_depth(i64 n, i64 m) {
  int d = 0;
  while ((n + (i64(1) << d) - 1) >> d > m) ++d;
  return d;
}

void build_compression(Compression& c, const Sampler& K, const gofmm_params& p) {
  const int threads = p.threads > 0 ? p.threads : omp_get_max_threads();
  const i64 n = c.n;
  c.leaf_size = p.leaf_size;
  c.max_rank = p.max_rank;
  c.tol = p.tol;
  c.kappa = p.kappa;
  c.budget = p.budget;
  c.distance = p.distance;
  c.storage = p.storage;
  c.near_storage = p.near_storage;
  c.seed = p.seed;
  c.depth = choose_depth(n, c.leaf_size);

  // 1. diagonal
  std::vector<double> diag(n);
  parallel_for((n + 4095) / 4096, threads, [&](i64 b) {
    for (i64 i = b * 4096; i < std::min(n, (b + 1) * 4096); ++i) K(1, &i, 1, &i, &diag[i]);
  });
  for (i64 i = 0; i < n; ++i)
    if (!(diag[i] > 0.0) || !std::isfinite(diag[i]))
      fail(GOFMM_ENOTSPD, "K(" + std::to_string(i) + "," + std::to_string(i) + ") is not positive and finite");
  Dist dist{K, diag, c.distance, threads};

  // 2. neighbours
  neighbours(c, dist, p);

  // 3. ball tree (PRE), level by level
  const int D = c.depth;
  const i64 nn = c.nn(), fl = c.fl(), L = c.n_leaves();
  c.split_p.assign(nn, -1);
  c.split_q.assign(nn, -1);
  c.centroid.assign(nn, {});
  std::vector<std::vector<i64>> nodes;
  auto leaves = build_levels(n, D, threads,
      [&](i64 h, const std::vector<i64>& idx, std::vector<i64>& l, std::vector<i64>& r) {
        Rng rng(mix(c.seed, 0xC0FFEE + h));
        metric_split(dist, idx, rng, l, r, c.split_p[h], c.split_q[h], c.centroid[h]);
      }, &nodes);
  c.perm.clear();
  c.perm.reserve(n);
  c.node_start.assign(nn, 0);
  c.node_size.assign(nn, 0);
  for (i64 b = 0; b < L; ++b) {
    c.node_start[fl + b] = (i64)c.perm.size();
    c.node_size[fl + b] = (i64)leaves[b].size();
    c.perm.insert(c.perm.end(), leaves[b].begin(), leaves[b].end());
  }
  for (i64 h = fl - 1; h >= 0; --h) {
    c.node_start[h] = c.node_start[2 * h + 1];
    c.node_size[h] = c.node_size[2 * h + 1] + c.node_size[2 * h + 2];
  }
  std::vector<i64> leaf_of(n);
  for (i64 b = 0; b < L; ++b)
    for (i64 i : leaves[b]) leaf_of[i] = b;

  // 4a. Near: ballot + budget, then symmetric by union
  const i64 cap = (i64)std::floor(c.budget * (double)n / (double)c.leaf_size + 1e-12);
  std::vector<std::vector<i64>> near(L);
  parallel_for(L, threads, [&](i64 b) {
    std::vector<i64> votes(L, 0);
    std::vector<i64> seen;
    for (i64 i : leaves[b])
      for (int t = 0; t < c.knn_k; ++t) {
        const i64 j = c.knn[(size_t)i * c.knn_k + t];
        if (j < 0) continue;
        const i64 a = leaf_of[j];
        if (votes[a]++ == 0) seen.push_back(a);
      }
    std::vector<i64> cands;
    for (i64 a : seen) if (a != b) cands.push_back(a);
    std::sort(cands.begin(), cands.end(), [&](i64 x, i64 y) {
      return votes[x] != votes[y] ? votes[x] > votes[y] : x < y;
    });
    if ((i64)cands.size() > cap) cands.resize(cap);
    cands.push_back(b);
    near[b] = cands;
  });
  {
    std::vector<std::vector<char>> mark(L, std::vector<char>(L, 0));
    for (i64 b = 0; b < L; ++b) for (i64 a : near[b]) { mark[b][a] = 1; mark[a][b] = 1; }
    c.near.assign(L, {});
    for (i64 b = 0; b < L; ++b)
      for (i64 a = 0; a < L; ++a) if (mark[b][a]) c.near[b].push_back(fl + a);
  }

  // 4b. FindFar per leaf, MergeFar in postorder
  std::vector<std::vector<i64>> far(nn);
  parallel_for(L, threads, [&](i64 b) {
    std::vector<char> marked(nn, 0);
    for (i64 a : c.near[b]) {
      i64 x = a;
      while (true) { marked[x] = 1; if (x == 0) break; x = (x - 1) / 2; }
    }
    std::vector<i64> stack{0};
    std::vector<i64> out;
    while (!stack.empty()) {
      const i64 h = stack.back();
      stack.pop_back();
      if (h >= fl) { if (!marked[h]) out.push_back(h); continue; }
      if (marked[h]) { stack.push_back(2 * h + 2); stack.push_back(2 * h + 1); }
      else out.push_back(h);
    }
    std::sort(out.begin(), out.end());
    far[fl + b] = out;
  });
  for (i64 h = fl - 1; h >= 0; --h) {
    auto& l = far[2 * h + 1];
    auto& r = far[2 * h + 2];
    std::vector<i64> common;
    std::set_intersection(l.begin(), l.end(), r.begin(), r.end(), std::back_inserter(common));
    std::vector<i64> nl, nr;
    std::set_difference(l.begin(), l.end(), common.begin(), common.end(), std::back_inserter(nl));
    std::set_difference(r.begin(), r.end(), common.begin(), common.end(), std::back_inserter(nr));
    l.swap(nl);
    r.swap(nr);
    far[h] = common;
  }
  if (!far[0].empty()) fail(GOFMM_EINVAL, "internal: root received far nodes");

  // 4c. symmetric refinement: cover[b][a] = far pair (B, A) holding leaf pair (b, a)
  {
    std::vector<std::vector<std::pair<i64, i64>>> cover(L, std::vector<std::pair<i64, i64>>(L, {-1, -1}));
    for (i64 h = 1; h < nn; ++h) {
      const int lh = level_of(h);
      const i64 b0 = (h - ((i64(1) << lh) - 1)) << (D - lh), nb = i64(1) << (D - lh);
      for (i64 A : far[h]) {
        const int la = level_of(A);
        const i64 a0 = (A - ((i64(1) << la) - 1)) << (D - la), na = i64(1) << (D - la);
        for (i64 b = b0; b < b0 + nb; ++b)
          for (i64 a = a0; a < a0 + na; ++a) cover[b][a] = {h, A};
      }
    }
    std::vector<std::vector<i64>> ref(nn);
    for (i64 b = 0; b < L; ++b)
      for (i64 a = 0; a < L; ++a) {
        auto [B, A] = cover[b][a];
        if (B < 0) continue;                                // a near pair
        auto [A2, B2] = cover[a][b];
        if (A2 < 0) fail(GOFMM_EINVAL, "internal: far pairs not closed under transposition");
        const i64 Bn = level_of(B) >= level_of(B2) ? B : B2;
        const i64 An = level_of(A) >= level_of(A2) ? A : A2;
        ref[Bn].push_back(An);
      }
    for (auto& v : ref) {
      std::sort(v.begin(), v.end());
      v.erase(std::unique(v.begin(), v.end()), v.end());
    }
    c.far.swap(ref);
  }

  // 5. skeletons: postorder, one level at a time, nodes of a level in parallel
  c.skel.assign(nn, {});
  c.samp.assign(nn, {});
  c.proj.assign(nn, {});
  std::vector<i64> pos_of(n);
  for (i64 k = 0; k < n; ++k) pos_of[c.perm[k]] = k;
  // columns of node h (its indices at a leaf, the children's skeletons above)
  // and its sampled rows I': neighbours outside the node by votes, then
  // uniform draws from the complement (reading R10)
  auto node_cols = [&](i64 h) {
    const i64 st = c.node_start[h], sz = c.node_size[h];
    std::vector<i64> cols;
    if (h >= fl) cols.assign(c.perm.begin() + st, c.perm.begin() + st + sz);
    else {
      cols = c.skel[2 * h + 1];
      cols.insert(cols.end(), c.skel[2 * h + 2].begin(), c.skel[2 * h + 2].end());
    }
    return cols;
  };
  auto node_rows = [&](i64 h, i64 ncols) {
      const i64 st = c.node_start[h], sz = c.node_size[h];
      const i64 ns = std::min(n - sz, 2 * ncols);
      // neighbours outside the node, by votes (ties by index), at most half of the rows
      std::vector<i64> flat;
      flat.reserve((size_t)sz * c.knn_k);
      for (i64 k = st; k < st + sz; ++k)
        for (int u = 0; u < c.knn_k; ++u) {
          const i64 j = c.knn[(size_t)c.perm[k] * c.knn_k + u];
          if (j >= 0 && (pos_of[j] < st || pos_of[j] >= st + sz)) flat.push_back(j);
        }
      std::sort(flat.begin(), flat.end());
      std::vector<std::pair<i64, i64>> vc;   // (-votes, id)
      for (size_t a = 0; a < flat.size();) {
        size_t b = a;
        while (b < flat.size() && flat[b] == flat[a]) ++b;
        vc.push_back({-(i64)(b - a), flat[a]});
        a = b;
      }
      std::sort(vc.begin(), vc.end());
      std::vector<i64> rows;
      for (size_t a = 0; a < vc.size() && (i64)rows.size() < ns / 2; ++a) rows.push_back(vc[a].second);
      // uniform fill from the complement without replacement
      const i64 need = ns - (i64)rows.size();
      if (need > 0) {
        Rng rng(mix(c.seed, 0x5EED00 + h));
        std::unordered_set<i64> used(rows.begin(), rows.end());
        std::vector<i64> extra;
        const i64 avail = n - sz - (i64)rows.size();
        if (need * 4 < avail) {
          while ((i64)extra.size() < need) {
            i64 pidx = (i64)rng.below(n - sz);        // position in the complement
            if (pidx >= st) pidx += sz;
            const i64 j = c.perm[pidx];
            if (used.insert(j).second) extra.push_back(j);
          }
        } else {
          std::vector<i64> pool;
          for (i64 k = 0; k < n; ++k)
            if ((k < st || k >= st + sz) && !used.count(c.perm[k])) pool.push_back(c.perm[k]);
          std::sort(pool.begin(), pool.end());
          for (i64 a = 0; a < need; ++a) std::swap(pool[a], pool[a + (i64)rng.below(pool.size() - a)]);
          extra.assign(pool.begin(), pool.begin() + need);
        }
        std::sort(extra.begin(), extra.end());
        rows.insert(rows.end(), extra.begin(), extra.end());
      }
      return rows;
  };
  for (int lev = D; lev >= 1; --lev) {
    const i64 h0 = (i64(1) << lev) - 1, cnt = i64(1) << lev;
    if (p.device_id) {
      // every node of the level in one batch on the device: sample the
      // blocks row-major (K is symmetric, so the sampler's column-major
      // K(cols, I') is K(I', cols) row-major), then factor them together
      std::vector<std::vector<i64>> cl(cnt), rw(cnt);
      parallel_for(cnt, threads, [&](i64 t) {
        cl[t] = node_cols(h0 + t);
        rw[t] = node_rows(h0 + t, (i64)cl[t].size());
      });
      std::vector<IdJob> jobs(cnt);
      i64 tot = 0;
      for (i64 t = 0; t < cnt; ++t) {
        jobs[t].a_off = tot;
        jobs[t].nrow = (i64)rw[t].size();
        jobs[t].ncol = (i64)cl[t].size();
        tot += jobs[t].nrow * jobs[t].ncol;
      }
      std::vector<double> blocks((size_t)tot);
      parallel_for(cnt, threads, [&](i64 t) {
        double* A = &blocks[jobs[t].a_off];
        K(jobs[t].ncol, cl[t].data(), jobs[t].nrow, rw[t].data(), A, jobs[t].ncol);
        for (i64 q = 0; q < jobs[t].nrow * jobs[t].ncol; ++q)
          if (!std::isfinite(A[q])) fail(GOFMM_ENOTSPD, "sampler returned a non-finite entry");
      });
      id_device_batch(jobs, blocks, c.tol, (int)c.max_rank);
      for (i64 t = 0; t < cnt; ++t) {
        const i64 h = h0 + t;
        std::vector<i64> sk(jobs[t].rank);
        for (int a = 0; a < jobs[t].rank; ++a) sk[a] = cl[t][jobs[t].piv[a]];
        c.skel[h] = std::move(sk);
        c.samp[h] = std::move(rw[t]);
        c.proj[h] = std::move(jobs[t].P);
      }
      continue;
    }
    parallel_for(cnt, threads, [&](i64 t) {
      const i64 h = h0 + t;
      std::vector<i64> cols = node_cols(h);
      const i64 ncols = (i64)cols.size();
      std::vector<i64> rows = node_rows(h, ncols);
      std::vector<double> A((size_t)rows.size() * ncols);     // column-major
      K((i64)rows.size(), rows.data(), ncols, cols.data(), A.data(), (i64)rows.size());
      for (double x : A)
        if (!std::isfinite(x)) fail(GOFMM_ENOTSPD, "sampler returned a non-finite entry");
      std::vector<int> piv;
      std::vector<double> P;
      const int s = interp_decomp(A.data(), (int)rows.size(), (int)ncols, c.tol, (int)c.max_rank, piv, P);
      std::vector<i64> sk(s);
      for (int a = 0; a < s; ++a) sk[a] = cols[piv[a]];
      c.skel[h] = std::move(sk);
      c.samp[h] = std::move(rows);
      c.proj[h] = std::move(P);
    });
  }
}

void validate_structure(const Compression& c) {
  const i64 n = c.n, nn = c.nn(), fl = c.fl(), L = c.n_leaves();
  auto bad = [](const std::string& m) { fail(GOFMM_EIO, "invalid compression: " + m); };
  if ((i64)c.perm.size() != n) bad("perm size");
  std::vector<char> seen(n, 0);
  for (i64 x : c.perm) { if (x < 0 || x >= n || seen[x]) bad("perm is not a permutation"); seen[x] = 1; }
  if ((i64)c.node_start.size() != nn || (i64)c.node_size.size() != nn) bad("node ranges");
  if (c.node_start[0] != 0 || c.node_size[0] != n) bad("root range");
  for (i64 h = 0; h < fl; ++h) {
    if (c.node_start[2 * h + 1] != c.node_start[h] ||
        c.node_start[2 * h + 2] != c.node_start[h] + c.node_size[2 * h + 1] ||
        c.node_size[h] != c.node_size[2 * h + 1] + c.node_size[2 * h + 2]) bad("children ranges");
  }
  for (i64 b = 0; b < L; ++b) if (c.node_size[fl + b] < 1) bad("empty leaf");
  if ((i64)c.near.size() != L || (i64)c.far.size() != nn || (i64)c.skel.size() != nn ||
      (i64)c.proj.size() != nn) bad("list counts");
  for (i64 b = 0; b < L; ++b)
    for (i64 a : c.near[b]) if (a < fl || a >= nn) bad("near entry is not a leaf");
  for (i64 h = 0; h < nn; ++h)
    for (i64 a : c.far[h]) if (a < 1 || a >= nn || h == 0) bad("far entry");
  if (!c.skel[0].empty() && nn > 1) bad("root skeleton");
  for (i64 h = 1; h < nn; ++h) {
    const i64 s = c.rank(h);
    if (s < 1) bad("empty skeleton at node " + std::to_string(h));
    if ((i64)c.proj[h].size() != s * c.ncols(h)) bad("P size at node " + std::to_string(h));
    for (i64 x : c.skel[h]) if (x < 0 || x >= n) bad("skeleton index");
    for (double x : c.proj[h]) if (!std::isfinite(x)) bad("non-finite P");
  }
}

}  // namespace gofmm
