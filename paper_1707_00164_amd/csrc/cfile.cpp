// Compression file format (structure only; kernel blocks are re-sampled by
// whoever loads it).  Little-endian: 8-byte magic "GOFMMC1\0", int64 array
// count, then per array a 24-byte zero-padded name, int32 dtype code
// (1 int32, 2 int64, 3 float64), int32 ndim, two int64 dims and the raw data.
// Ragged lists are stored as "<name>_ptr" (count + 1 offsets) and
// "<name>_val".  Arrays: params [n, m, s, tau, kappa, budget, distance,
// depth], perm, node_start, node_size, split_p, split_q, centroid, near, far,
// skel, samp (ragged), knn (n x kappa, optional), proj (ragged, row-major P).
#include <cstdio>
#include <map>

#include "internal.hpp"

namespace gofmm {

namespace {

struct Arr {
  int dt = 0, nd = 1;
  i64 d0 = 0, d1 = 1;
  std::vector<char> data;
};

struct Writer {
  FILE* f;
  std::vector<std::pair<std::string, Arr>> arrays;
  template <class T>
  void add(const std::string& name, const T* p, i64 d0, i64 d1, int nd) {
    Arr a;
    a.dt = sizeof(T) == 4 ? 1 : (std::is_floating_point<T>::value ? 3 : 2);
    a.nd = nd;
    a.d0 = d0;
    a.d1 = d1;
    a.data.resize(sizeof(T) * d0 * d1);
    if (d0 * d1) std::memcpy(a.data.data(), p, a.data.size());
    arrays.push_back({name, std::move(a)});
  }
  void vec(const std::string& name, const std::vector<i64>& v) { add(name, v.data(), (i64)v.size(), 1, 1); }
  template <class T>
  void ragged(const std::string& name, const std::vector<std::vector<T>>& lists) {
    std::vector<i64> ptr(lists.size() + 1, 0);
    std::vector<T> val;
    for (size_t i = 0; i < lists.size(); ++i) {
      ptr[i + 1] = ptr[i] + (i64)lists[i].size();
      val.insert(val.end(), lists[i].begin(), lists[i].end());
    }
    vec(name + "_ptr", ptr);
    add(name + "_val", val.data(), (i64)val.size(), 1, 1);
  }
};

}  // namespace

void write_file(const Compression& c, const char* path) {
  Writer w;
  const double params[8] = {(double)c.n, (double)c.leaf_size, (double)c.max_rank, c.tol,
                            (double)c.kappa, c.budget, (double)c.distance, (double)c.depth};
  w.add("params", params, 8, 1, 1);
  w.vec("perm", c.perm);
  w.vec("node_start", c.node_start);
  w.vec("node_size", c.node_size);
  w.vec("split_p", c.split_p);
  w.vec("split_q", c.split_q);
  w.ragged("centroid", c.centroid);
  w.ragged("near", c.near);
  w.ragged("far", c.far);
  w.ragged("skel", c.skel);
  w.ragged("samp", c.samp);
  if (!c.knn.empty()) w.add("knn", c.knn.data(), c.n, (i64)c.knn_k, 2);
  w.ragged("proj", c.proj);
  FILE* f = std::fopen(path, "wb");
  if (!f) fail(GOFMM_EIO, std::string("cannot open ") + path + " for writing");
  bool ok = std::fwrite("GOFMMC1\0", 1, 8, f) == 8;
  const i64 cnt = (i64)w.arrays.size();
  ok = ok && std::fwrite(&cnt, 8, 1, f) == 1;
  for (auto& [name, a] : w.arrays) {
    char nm[24] = {0};
    std::strncpy(nm, name.c_str(), 23);
    const int32_t hdr[2] = {a.dt, a.nd};
    const i64 dims[2] = {a.d0, a.d1};
    ok = ok && std::fwrite(nm, 1, 24, f) == 24 && std::fwrite(hdr, 4, 2, f) == 2 &&
         std::fwrite(dims, 8, 2, f) == 2 &&
         (a.data.empty() || std::fwrite(a.data.data(), 1, a.data.size(), f) == a.data.size());
  }
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) fail(GOFMM_EIO, std::string("write failed: ") + path);
}

void read_file(Compression& c, const char* path) {
  FILE* f = std::fopen(path, "rb");
  if (!f) fail(GOFMM_EIO, std::string("cannot open ") + path);
  std::map<std::string, Arr> m;
  char magic[8];
  i64 cnt = 0;
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "GOFMMC1\0", 8) == 0 &&
            std::fread(&cnt, 8, 1, f) == 1 && cnt >= 0 && cnt < 1000;
  for (i64 t = 0; ok && t < cnt; ++t) {
    char nm[25] = {0};
    int32_t hdr[2];
    i64 dims[2];
    ok = std::fread(nm, 1, 24, f) == 24 && std::fread(hdr, 4, 2, f) == 2 && std::fread(dims, 8, 2, f) == 2;
    if (!ok || hdr[0] < 1 || hdr[0] > 3 || dims[0] < 0 || dims[1] < 0 || dims[0] > (i64(1) << 40) ||
        dims[1] > (i64(1) << 20)) { ok = false; break; }
    Arr a;
    a.dt = hdr[0];
    a.nd = hdr[1];
    a.d0 = dims[0];
    a.d1 = dims[1];
    const size_t es = a.dt == 1 ? 4 : 8;
    a.data.resize(es * a.d0 * a.d1);
    ok = a.data.empty() || std::fread(a.data.data(), 1, a.data.size(), f) == a.data.size();
    m[nm] = std::move(a);
  }
  std::fclose(f);
  if (!ok) fail(GOFMM_EIO, std::string("malformed compression file ") + path);
  auto get = [&](const std::string& name, int dt) -> const Arr& {
    auto it = m.find(name);
    if (it == m.end() || it->second.dt != dt) fail(GOFMM_EIO, "compression file lacks " + name);
    return it->second;
  };
  auto ivec = [&](const std::string& name) {
    const Arr& a = get(name, 2);
    std::vector<i64> v(a.d0 * a.d1);
    if (!v.empty()) std::memcpy(v.data(), a.data.data(), v.size() * 8);
    return v;
  };
  auto ragged_i = [&](const std::string& name, i64 count) {
    auto ptr = ivec(name + "_ptr");
    auto val = ivec(name + "_val");
    if ((i64)ptr.size() != count + 1) fail(GOFMM_EIO, "bad ragged list " + name);
    std::vector<std::vector<i64>> out(count);
    for (i64 i = 0; i < count; ++i) {
      if (ptr[i] < 0 || ptr[i] > ptr[i + 1] || ptr[i + 1] > (i64)val.size()) fail(GOFMM_EIO, "bad offsets in " + name);
      out[i].assign(val.begin() + ptr[i], val.begin() + ptr[i + 1]);
    }
    return out;
  };
  const Arr& pa = get("params", 3);
  if (pa.d0 * pa.d1 < 8) fail(GOFMM_EIO, "bad params");
  const double* pr = reinterpret_cast<const double*>(pa.data.data());
  c.n = (i64)pr[0];
  c.leaf_size = (i64)pr[1];
  c.max_rank = (i64)pr[2];
  c.tol = pr[3];
  c.kappa = (int)pr[4];
  c.budget = pr[5];
  c.distance = (int)pr[6];
  c.depth = (int)pr[7];
  if (c.n < 1 || c.depth < 0 || c.depth > 30 || (i64(1) << c.depth) > c.n) fail(GOFMM_EIO, "bad n/depth");
  const i64 nn = c.nn(), L = c.n_leaves();
  c.perm = ivec("perm");
  c.node_start = ivec("node_start");
  c.node_size = ivec("node_size");
  c.split_p = ivec("split_p");
  c.split_q = ivec("split_q");
  c.centroid = ragged_i("centroid", nn);
  c.near = ragged_i("near", L);
  c.far = ragged_i("far", nn);
  c.skel = ragged_i("skel", nn);
  c.samp = ragged_i("samp", nn);
  if (m.count("knn")) {
    const Arr& k = get("knn", 2);
    c.knn.resize(k.d0 * k.d1);
    std::memcpy(c.knn.data(), k.data.data(), c.knn.size() * 8);
    c.knn_k = (int)k.d1;
  }
  {
    auto ptr = ivec("proj_ptr");
    const Arr& v = get("proj_val", 3);
    if ((i64)ptr.size() != nn + 1) fail(GOFMM_EIO, "bad proj");
    const double* pv = reinterpret_cast<const double*>(v.data.data());
    c.proj.assign(nn, {});
    for (i64 h = 0; h < nn; ++h) {
      if (ptr[h] < 0 || ptr[h] > ptr[h + 1] || ptr[h + 1] > v.d0 * v.d1) fail(GOFMM_EIO, "bad proj offsets");
      c.proj[h].assign(pv + ptr[h], pv + ptr[h + 1]);
    }
  }
}

}  // namespace gofmm
