// Device operator layout: every step of the evaluation as gather-GEMM tasks.
//
// Each task computes out[m x r] = A[m x k] * B[k x r] (or +=), where A is a
// dense block in the operator buffer of its precision, in matrix-core fragment
// order, and
// the rows of B and of out are addressed through a row-code list (caller's W
// or U rows through the permutation, or rows of the skeleton workspace).  The
// steps of Alg. "Evaluate" (Sec. 2.2, Table 2) become:
//
//   n2s-leaf        w~_b = P_b W[perm(b)]                          (N2S, leaves)
//   n2s-level l     w~_a = P_a [w~_l; w~_r]           for l = D-1 .. 1 (N2S)
//   s2s             u~_b = [K(b~, a~1) | K(b~, a~2) ...] [w~_a1; w~_a2; ...]
//                   for every non-root node in one launch
//   s2n-level l     u~_c += (P_p^T)_c u~_p for the nodes c of level l = 2 .. D,
//                   p the parent of c (each task owns its child's rows)
//   leaf            U[perm(b)] = [P_b^T | K(b, a1) ...] [u~_b; W[perm(a1)]; ...]
//                   (S2N at the leaf fused with L2L; U written once)
//
// When P/coupling and near blocks use different precisions the leaf step is
// split into s2n-leaf (overwrite) and l2l (accumulate).  The permutation of W
// and U is folded into the row codes, so no separate permute pass exists.
#include <omp.h>

#include <algorithm>
#include <cmath>

#include <cstring>

#include "internal.hpp"

namespace gofmm {

namespace {

// k padding of A blocks (one k slab of the kernels: 32 FP32 or 64 BF16
// values); rows are padded to 32.
i64 round_up(i64 x, i64 a) { return (x + a - 1) / a * a; }
i64 kalign(int prec) { return prec == PREC_F32 ? 32 : 64; }
i64 rows_stored(i64 m) { return round_up(m, 32); }

// Fragment order: A is cut into chunks of 32 rows, ordered by row block, then
// k; inside a chunk, lane L = 32 h + i' of a 64-wide wave holds one 16-byte
// vector of row i', exactly its A operand for one step of the kernel.
//  FP32 (chunk = 8 k): k = 32 slab + 16 h + 4 s + q, chunk s of the slab,
//                      element q of the vector (four 32x32x2 steps).
//  BF16 (chunk = 16 k): k = 16 c + 8 h + e, element e (one 32x32x16 step).
inline i64 frag_pos_f32(i64 i, i64 j, i64 lda) {
  const i64 chunk = (i >> 5) * (lda >> 3) + ((j >> 5) << 2) + ((j >> 2) & 3);
  return chunk * 256 + ((((j >> 4) & 1) << 5) + (i & 31)) * 4 + (j & 3);
}
inline i64 frag_pos_b16(i64 i, i64 j, i64 lda) {
  return ((i >> 5) * (lda >> 4) + (j >> 4)) * 512 + ((((j >> 3) & 1) << 5) + (i & 31)) * 8 + (j & 7);
}
int elem_bytes(int prec) { return prec == PREC_BF16 ? 2 : 4; }

// One part of a task's A: either a P-based block or a kernel block.
struct Part {
  int type;        // 0: P_h (s x ncols); 1: P_h^T restricted (see cols); 2: K(rows, cols);
                   // 3: K(rows, cols) computed on the device (nothing stored)
  i64 node;        // for types 0/1
  i64 c0, c1;      // column range of P_h for type 1 (rows of P^T)
  std::vector<i64> krows, kcols;  // for type 2 (original indices)
  i64 width;       // columns of A this part occupies
};

struct Draft {
  int prec;
  bool geo = false;        // A computed on the device from points (kind-7 launch)
  i64 m;
  std::vector<Part> parts;
  std::vector<i32> brow;   // B row codes (k of them)
  std::vector<i32> orow;   // out row codes (m of them)
  int phase_of_part[8];
};

}  // namespace

void build_plan(Compression& c, const Sampler& K, int threads) {
  HostPlan& pl = c.plan;
  pl = HostPlan();
  const int D = c.depth;
  const i64 nn = c.nn(), fl = c.fl(), L = c.n_leaves();
  // workspace rows: skeleton weights of non-root nodes in heap order, then potentials
  std::vector<i64> soff(nn + 1, 0);
  for (i64 h = 1; h < nn; ++h) soff[h + 1] = soff[h] + c.rank(h);
  const i64 S = soff[nn];
  pl.ws_rows = 2 * S;
  if (2 * S + 1 >= (i64)INT32_MAX || c.n >= (i64)INT32_MAX) fail(GOFMM_ELIMIT, "problem too large for 32-bit row codes");
  auto wrow = [&](i64 h, i64 j) { return (i32)(-(soff[h] + j) - 1); };
  auto urow = [&](i64 h, i64 j) { return (i32)(-(S + soff[h] + j) - 1); };
  const int pst = c.storage, pnear = c.near_storage;

  std::vector<Draft> drafts;
  auto begin_launch = [&](int prec, int acc, int kind, int level, const std::string& name) {
    LaunchDesc l;
    l.prec = prec;
    l.accumulate = acc;
    l.t_begin = (i32)drafts.size();
    l.t_end = l.t_begin;
    l.kind = kind;
    l.level = level;
    l.name = name;
    pl.launches.push_back(l);
  };
  auto end_launch = [&]() {
    pl.launches.back().t_end = (i32)drafts.size();
    if (pl.launches.back().t_end == pl.launches.back().t_begin) pl.launches.pop_back();
  };
  auto leaf_rows = [&](i64 h, std::vector<i32>& out) {
    for (i64 t = 0; t < c.node_size[h]; ++t) out.push_back((i32)c.perm[c.node_start[h] + t]);
  };
  auto leaf_idx = [&](i64 h) {
    return std::vector<i64>(c.perm.begin() + c.node_start[h], c.perm.begin() + c.node_start[h] + c.node_size[h]);
  };

  if (D >= 1) {
    // N2S at the leaves
    begin_launch(pst, 0, 0, D, "n2s_leaf");
    for (i64 b = 0; b < L; ++b) {
      const i64 h = fl + b;
      Draft d;
      d.prec = pst;
      d.m = c.rank(h);
      d.parts.push_back({0, h, 0, 0, {}, {}, c.node_size[h]});
      leaf_rows(h, d.brow);
      for (i64 j = 0; j < d.m; ++j) d.orow.push_back(wrow(h, j));
      drafts.push_back(std::move(d));
    }
    end_launch();
    // N2S up the levels
    for (int lev = D - 1; lev >= 1; --lev) {
      begin_launch(pst, 0, 1, lev, "n2s_l" + std::to_string(lev));
      for (i64 h = (i64(1) << lev) - 1; h < (i64(2) << lev) - 1; ++h) {
        Draft d;
        d.prec = pst;
        d.m = c.rank(h);
        d.parts.push_back({0, h, 0, 0, {}, {}, c.ncols(h)});
        for (i64 ch : {2 * h + 1, 2 * h + 2})
          for (i64 j = 0; j < c.rank(ch); ++j) d.brow.push_back(wrow(ch, j));
        for (i64 j = 0; j < d.m; ++j) d.orow.push_back(wrow(h, j));
        drafts.push_back(std::move(d));
      }
      end_launch();
    }
    // S2S for every non-root node in one launch (any order once w~ is ready)
    begin_launch(pst, 0, 2, 0, "s2s");
    for (i64 h = 1; h < nn; ++h) {
      Draft d;
      d.prec = pst;
      d.m = c.rank(h);
      for (i64 a : c.far[h]) {
        d.parts.push_back({2, 0, 0, 0, c.skel[h], c.skel[a], c.rank(a)});
        for (i64 j = 0; j < c.rank(a); ++j) d.brow.push_back(wrow(a, j));
      }
      for (i64 j = 0; j < d.m; ++j) d.orow.push_back(urow(h, j));
      drafts.push_back(std::move(d));
    }
    end_launch();
    // S2N down the levels, pull form: u~_c += (P_p^T)_c u~_p for every child c
    // of an internal node p, children at level l = 2 .. D (no atomics: each
    // task owns the rows of its child)
    for (int lev = 2; lev <= D; ++lev) {
      begin_launch(pst, 1, 6, lev, "s2n_l" + std::to_string(lev));
      for (i64 h = (i64(1) << lev) - 1; h < (i64(2) << lev) - 1; ++h) {
        const i64 p = (h - 1) / 2;
        const i64 sl = c.rank(2 * p + 1);
        const bool left = (h == 2 * p + 1);
        const i64 c0 = left ? 0 : sl, c1 = left ? sl : sl + c.rank(2 * p + 2);
        Draft d;
        d.prec = pst;
        d.m = c.rank(h);
        d.parts.push_back({1, p, c0, c1, {}, {}, c.rank(p)});
        for (i64 j = 0; j < c.rank(p); ++j) d.brow.push_back(urow(p, j));
        for (i64 j = 0; j < d.m; ++j) d.orow.push_back(urow(h, j));
        drafts.push_back(std::move(d));
      }
      end_launch();
    }
  }
  // leaf output: S2N at the leaf and L2L
  auto near_parts = [&](i64 h, Draft& d) {
    for (i64 a : c.near[h - fl]) {
      d.parts.push_back({2, 0, 0, 0, leaf_idx(h), leaf_idx(a), c.node_size[a]});
      leaf_rows(a, d.brow);
    }
  };
  if (c.geo.kind >= 0) {
    // geometric mode: S2N at the leaf from the stored P^T, then L2L with the
    // near blocks computed on the device (FP32) from the points
    if (D >= 1) {
      begin_launch(pst, 0, 4, D, "s2n_leaf");
      for (i64 b = 0; b < L; ++b) {
        const i64 h = fl + b;
        Draft d;
        d.prec = pst;
        d.m = c.node_size[h];
        d.parts.push_back({1, h, 0, c.node_size[h], {}, {}, c.rank(h)});
        for (i64 j = 0; j < c.rank(h); ++j) d.brow.push_back(urow(h, j));
        leaf_rows(h, d.orow);
        drafts.push_back(std::move(d));
      }
      end_launch();
    }
    begin_launch(PREC_F32, D >= 1 ? 1 : 0, 7, D, "l2l");
    for (i64 b = 0; b < L; ++b) {
      const i64 h = fl + b;
      Draft d;
      d.prec = PREC_F32;
      d.geo = true;
      d.m = c.node_size[h];
      for (i64 a : c.near[h - fl]) {
        d.parts.push_back({3, 0, 0, 0, {}, {}, c.node_size[a]});
        leaf_rows(a, d.brow);
      }
      leaf_rows(h, d.orow);
      drafts.push_back(std::move(d));
    }
    end_launch();
  } else if (D >= 1 && pst != pnear) {
    begin_launch(pst, 0, 4, D, "s2n_leaf");
    for (i64 b = 0; b < L; ++b) {
      const i64 h = fl + b;
      Draft d;
      d.prec = pst;
      d.m = c.node_size[h];
      d.parts.push_back({1, h, 0, c.node_size[h], {}, {}, c.rank(h)});
      for (i64 j = 0; j < c.rank(h); ++j) d.brow.push_back(urow(h, j));
      leaf_rows(h, d.orow);
      drafts.push_back(std::move(d));
    }
    end_launch();
    begin_launch(pnear, 1, 5, D, "l2l");
    for (i64 b = 0; b < L; ++b) {
      const i64 h = fl + b;
      Draft d;
      d.prec = pnear;
      d.m = c.node_size[h];
      near_parts(h, d);
      leaf_rows(h, d.orow);
      drafts.push_back(std::move(d));
    }
    end_launch();
  } else {
    const int prec = D >= 1 ? pst : pnear;
    begin_launch(prec, 0, 3, D, "leaf");
    for (i64 b = 0; b < L; ++b) {
      const i64 h = fl + b;
      Draft d;
      d.prec = prec;
      d.m = c.node_size[h];
      if (D >= 1) {
        d.parts.push_back({1, h, 0, c.node_size[h], {}, {}, c.rank(h)});
        for (i64 j = 0; j < c.rank(h); ++j) d.brow.push_back(urow(h, j));
      }
      near_parts(h, d);
      leaf_rows(h, d.orow);
      drafts.push_back(std::move(d));
    }
    end_launch();
  }

  // offsets
  const i64 T = (i64)drafts.size();
  pl.tasks.resize(T);
  i64 off[3] = {0, 0, 0};
  i64 goff = 0;
  i64 roff = 0;
  for (i64 t = 0; t < T; ++t) {
    Draft& d = drafts[t];
    i64 k = 0;
    for (auto& p : d.parts) k += p.width;
    if ((i64)d.brow.size() != k || (i64)d.orow.size() != d.m) fail(GOFMM_EINVAL, "internal: task shape");
    const i64 lda = round_up(k, kalign(d.prec));
    TaskDesc& td = pl.tasks[t];
    td.m = (i32)d.m;
    td.k = (i32)k;
    td.lda = (i32)lda;
    td.kws = 0;
    for (i32 code : d.brow) {
      if (code >= 0) break;
      ++td.kws;
    }
    td.idx_off = roff;
    if (d.geo) {
      td.a_off = goff;
      goff += lda * kGeoStride;
    } else {
      td.a_off = off[d.prec];
      off[d.prec] += rows_stored(d.m) * lda;
    }
    roff += lda + d.m;
  }
  pl.rows.assign(roff, ROW_ZERO);
  for (i64 t = 0; t < T; ++t) {
    const Draft& d = drafts[t];
    const TaskDesc& td = pl.tasks[t];
    std::copy(d.brow.begin(), d.brow.end(), pl.rows.begin() + td.idx_off);
    std::copy(d.orow.begin(), d.orow.end(), pl.rows.begin() + td.idx_off + td.lda);
  }
  pl.a_f32.assign(off[PREC_F32], 0.0f);
  pl.a_b16.assign(off[PREC_BF16], 0);
  pl.x3_plane = off[PREC_BF16X3];
  pl.a_x3.assign(2 * off[PREC_BF16X3], 0);
  pl.geo_cols.assign(goff, 0.0f);
  for (i64 t = 0; t < T; ++t) {
    const Draft& d = drafts[t];
    if (!d.geo) continue;
    const TaskDesc& td = pl.tasks[t];
    for (i64 j = 0; j < td.lda; ++j) {
      float* e = &pl.geo_cols[td.a_off + j * kGeoStride];
      if (j < td.k) {
        const i32 code = d.brow[j];
        if (code < 0 || code >= c.n) fail(GOFMM_EINVAL, "internal: near column code");
        std::copy(c.geo.pts.begin() + (size_t)code * kGeoStride,
                  c.geo.pts.begin() + (size_t)(code + 1) * kGeoStride, e);
      } else {
        const int32_t none = -1;
        std::memcpy(&e[kGeoDim], &none, sizeof(none));
      }
    }
  }

  // flop and byte accounting per right-hand side (Table 2)
  for (size_t li = 0; li < pl.launches.size(); ++li) {
    LaunchDesc& l = pl.launches[li];
    for (i32 t = l.t_begin; t < l.t_end; ++t) {
      const Draft& d = drafts[t];
      if (d.geo) l.bytes += pl.tasks[t].lda * kGeoStride * (i64)sizeof(float);
      for (const Part& p : d.parts) {
        l.flops += 2.0 * (double)d.m * (double)p.width;
        if (!d.geo) l.bytes += d.m * p.width * elem_bytes(d.prec);
        int ph;
        if (p.type == 0) ph = PH_N2S;
        else if (p.type == 1) ph = PH_S2N;
        else ph = (l.kind == 2) ? PH_S2S : PH_L2L;
        pl.flops_phase[ph] += 2.0 * (double)d.m * (double)p.width;
        if (!d.geo) pl.bytes_phase[ph] += d.m * p.width * elem_bytes(d.prec);
      }
    }
  }

  // fill A blocks (sampling the kernel blocks) in parallel over tasks
  std::vector<int> err(T, 0);
  std::vector<std::string> emsg(T);
  const int th = threads > 0 ? threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(th)
  for (i64 t = 0; t < T; ++t) {
    try {
      const Draft& d = drafts[t];
      if (d.geo) continue;                      // computed on the device
      const TaskDesc& td = pl.tasks[t];
      const i64 m = d.m, k = td.k;
      // A column-major (leading dimension m), the sampler's own layout, so
      // kernel blocks are sampled in place
      std::vector<double> A((size_t)m * std::max<i64>(k, 1), 0.0);
      i64 col = 0;
      for (const Part& p : d.parts) {
        if (p.type == 0) {
          const i64 nc = c.ncols(p.node);
          const double* P = c.proj[p.node].data();
          for (i64 j = 0; j < nc; ++j)
            for (i64 i = 0; i < m; ++i) A[i + (col + j) * m] = P[i * nc + j];
        } else if (p.type == 1) {
          // rows c0..c1 of P_node^T = columns c0..c1 of P_node
          const i64 nc = c.ncols(p.node), s = c.rank(p.node);
          const double* P = c.proj[p.node].data();
          for (i64 j = 0; j < s; ++j)
            for (i64 i = 0; i < p.c1 - p.c0; ++i) A[i + (col + j) * m] = P[j * nc + p.c0 + i];
        } else {
          K((i64)p.krows.size(), p.krows.data(), (i64)p.kcols.size(), p.kcols.data(), &A[col * m], m);
        }
        col += p.width;
      }
      for (double x : A)
        if (!std::isfinite(x)) fail(GOFMM_ENOTSPD, "non-finite entry in a cached block");
      const i64 lda = td.lda;
      if (d.prec == PREC_F32) {
        float* dst = &pl.a_f32[td.a_off];
        for (i64 j = 0; j < k; ++j)
          for (i64 i = 0; i < m; ++i) dst[frag_pos_f32(i, j, lda)] = (float)A[i + j * m];
      } else if (d.prec == PREC_BF16) {
        uint16_t* dst = &pl.a_b16[td.a_off];
        for (i64 j = 0; j < k; ++j)
          for (i64 i = 0; i < m; ++i) dst[frag_pos_b16(i, j, lda)] = to_bf16(A[i + j * m]);
      } else {
        uint16_t* hi = &pl.a_x3[td.a_off];
        uint16_t* lo = &pl.a_x3[pl.x3_plane + td.a_off];
        for (i64 j = 0; j < k; ++j)
          for (i64 i = 0; i < m; ++i) {
            const double x = A[i + j * m];
            const uint16_t h = to_bf16(x);
            hi[frag_pos_b16(i, j, lda)] = h;
            lo[frag_pos_b16(i, j, lda)] = to_bf16(x - from_bf16(h));
          }
      }
    } catch (const Error& e) {
      err[t] = e.code;
      emsg[t] = e.what();
    } catch (const std::bad_alloc&) {
      err[t] = GOFMM_ENOMEM;
      emsg[t] = "out of host memory";
    }
  }
  for (i64 t = 0; t < T; ++t)
    if (err[t]) fail(err[t], emsg[t]);
}

}  // namespace gofmm
