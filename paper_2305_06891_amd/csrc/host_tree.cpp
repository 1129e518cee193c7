// Host side: facet geometry, index tree (Algorithm 1) and block tree
// (Algorithm 2) of "Hierarchical Block Low-rank Approximation of Cavity
// Radiation", Sec. 4.1-4.2.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "hm_internal.hpp"

namespace hm {

namespace {

// (x*x + y*y) + z*z, no fused multiply-add (the order is part of the contract
// of the admissibility test so that ties are decided reproducibly).
#pragma clang fp contract(off)
double norm3(double x, double y, double z) { return std::sqrt((x * x + y * y) + z * z); }

struct TreeBuilder {
  const double* c;
  int32_t n_min;
  std::vector<int32_t> idx;  // working index array, permuted in place
  std::vector<ClusterNode>& nodes;
  std::vector<int32_t>& leaves;

  int32_t rec(int32_t begin, int32_t end, int32_t level) {
    ClusterNode nd{};
    nd.begin = begin;
    nd.end = end;
    nd.level = level;
    nd.child[0] = nd.child[1] = -1;
    for (int a = 0; a < 3; ++a) { nd.lo[a] = INFINITY; nd.hi[a] = -INFINITY; }
    for (int32_t k = begin; k < end; ++k) {
      const double* p = c + 3 * (int64_t)idx[k];
      for (int a = 0; a < 3; ++a) {
        nd.lo[a] = std::min(nd.lo[a], p[a]);
        nd.hi[a] = std::max(nd.hi[a], p[a]);
      }
    }
    int32_t me = (int32_t)nodes.size();
    nodes.push_back(nd);
    int32_t cnt = end - begin;
    if (cnt <= n_min) {
      leaves.push_back(me);
      return me;
    }
    // longest axis of the bounding box; first maximum wins (x < y < z)
    int axis = 0;
    double ext = nd.hi[0] - nd.lo[0];
    for (int a = 1; a < 3; ++a) {
      double e = nd.hi[a] - nd.lo[a];
      if (e > ext) { ext = e; axis = a; }
    }
    // order by (coordinate, original index); left child takes floor(cnt/2)
    std::sort(idx.begin() + begin, idx.begin() + end, [&](int32_t x, int32_t y) {
      double cx = c[3 * (int64_t)x + axis], cy = c[3 * (int64_t)y + axis];
      if (cx != cy) return cx < cy;
      return x < y;
    });
    int32_t mid = begin + cnt / 2;
    int32_t l = rec(begin, mid, level + 1);
    int32_t r = rec(mid, end, level + 1);
    nodes[me].child[0] = l;
    nodes[me].child[1] = r;
    return me;
  }
};

double diam(const ClusterNode& a) { return norm3(a.hi[0] - a.lo[0], a.hi[1] - a.lo[1], a.hi[2] - a.lo[2]); }

double dist(const ClusterNode& a, const ClusterNode& b) {
  double g[3];
  for (int k = 0; k < 3; ++k) g[k] = std::max(0.0, std::max(b.lo[k] - a.hi[k], a.lo[k] - b.hi[k]));
  return norm3(g[0], g[1], g[2]);
}

bool admissible(const ClusterNode& s, const ClusterNode& t, double eta) {
  double d = dist(s, t);
  if (!(d > 0.0)) return false;
  return std::min(diam(s), diam(t)) <= eta * d;
}

}  // namespace

bool tree_admissible(const ClusterNode& s, const ClusterNode& t, double eta) { return admissible(s, t, eta); }

void build_tree(hm_tree& t) {
  const int64_t n = t.n;
  t.nodes.clear();
  t.leaves.clear();
  t.dense.clear();
  t.lowrank.clear();
  TreeBuilder tb{t.c.data(), t.params.leaf_size, std::vector<int32_t>(n), t.nodes, t.leaves};
  std::iota(tb.idx.begin(), tb.idx.end(), 0);
  tb.rec(0, (int32_t)n, 0);
  t.perm = std::move(tb.idx);
  // Algorithm 2 with an explicit stack (depth-first; the output is sorted below)
  std::vector<std::pair<int32_t, int32_t>> st;
  st.emplace_back(0, 0);
  const double eta = t.params.eta;
  while (!st.empty()) {
    auto [si, ti] = st.back();
    st.pop_back();
    const ClusterNode& s = t.nodes[si];
    const ClusterNode& u = t.nodes[ti];
    BlockRef b{s.begin, s.end, u.begin, u.end};
    if (admissible(s, u, eta)) {
      t.lowrank.push_back(b);
    } else if (s.child[0] < 0 || u.child[0] < 0) {
      t.dense.push_back(b);
    } else {
      for (int a = 0; a < 2; ++a)
        for (int bb = 0; bb < 2; ++bb) st.emplace_back(s.child[a], u.child[bb]);
    }
  }
  auto key = [](const BlockRef& x, const BlockRef& y) { return x.rb != y.rb ? x.rb < y.rb : x.cb < y.cb; };
  std::sort(t.dense.begin(), t.dense.end(), key);
  std::sort(t.lowrank.begin(), t.lowrank.end(), key);
}

}  // namespace hm

using namespace hm;

extern "C" {

hm_status hm_facets_from_triangles(int64_t nv, const double* v, int64_t nt, const int32_t* tri, int orient,
                                   double* centroid, double* normal, double* area) {
  try {
    HM_REQUIRE(nv >= 3 && nt >= 1 && v && tri && centroid && normal && area, "hm_facets_from_triangles: bad arguments");
    for (int64_t k = 0; k < 3 * nv; ++k) HM_REQUIRE(std::isfinite(v[k]), "hm_facets_from_triangles: non-finite vertex");
    double g[3] = {0, 0, 0};
    for (int64_t k = 0; k < nv; ++k)
      for (int a = 0; a < 3; ++a) g[a] += v[3 * k + a];
    for (int a = 0; a < 3; ++a) g[a] /= (double)nv;
    for (int64_t f = 0; f < nt; ++f) {
      int32_t i0 = tri[3 * f], i1 = tri[3 * f + 1], i2 = tri[3 * f + 2];
      HM_REQUIRE(i0 >= 0 && i0 < nv && i1 >= 0 && i1 < nv && i2 >= 0 && i2 < nv,
                 "hm_facets_from_triangles: vertex index out of range");
      const double* a = v + 3 * (int64_t)i0;
      const double* b = v + 3 * (int64_t)i1;
      const double* c = v + 3 * (int64_t)i2;
      double e1[3], e2[3], cr[3], cen[3];
      for (int k = 0; k < 3; ++k) {
        e1[k] = b[k] - a[k];
        e2[k] = c[k] - a[k];
        cen[k] = (a[k] + b[k] + c[k]) / 3.0;
      }
      cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
      cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
      cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
      double tw = std::sqrt((cr[0] * cr[0] + cr[1] * cr[1]) + cr[2] * cr[2]);
      HM_REQUIRE(tw > 0.0 && std::isfinite(tw), "hm_facets_from_triangles: degenerate triangle");
      double nn[3] = {cr[0] / tw, cr[1] / tw, cr[2] / tw};
      bool flip = orient < 0;
      if (orient == 0) {
        double d = (nn[0] * (cen[0] - g[0]) + nn[1] * (cen[1] - g[1])) + nn[2] * (cen[2] - g[2]);
        flip = d > 0.0;
      }
      for (int k = 0; k < 3; ++k) {
        centroid[3 * f + k] = cen[k];
        normal[3 * f + k] = flip ? -nn[k] : nn[k];
      }
      area[f] = 0.5 * tw;
    }
    return HM_OK;
  } catch (const Error& e) {
    set_tl_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    set_tl_error(e.what());
    return HM_EINVAL;
  }
}

hm_status hm_build_cluster_tree(hm_ctx* ctx, int64_t n, const double* centroid, const double* normal,
                                const double* area, const hm_tree_params* params, hm_tree** out) {
  try {
    HM_REQUIRE(out && centroid && normal && area && params, "hm_build_cluster_tree: NULL argument");
    HM_REQUIRE(n >= 1 && n < (int64_t)1 << 31, "hm_build_cluster_tree: n out of range");
    HM_REQUIRE(params->leaf_size >= 1, "hm_build_cluster_tree: leaf_size must be >= 1");
    HM_REQUIRE(params->eta > 0.0 && std::isfinite(params->eta), "hm_build_cluster_tree: eta must be > 0");
    for (int64_t k = 0; k < 3 * n; ++k)
      HM_REQUIRE(std::isfinite(centroid[k]) && std::isfinite(normal[k]), "hm_build_cluster_tree: non-finite geometry");
    for (int64_t k = 0; k < n; ++k)
      HM_REQUIRE(area[k] > 0.0 && std::isfinite(area[k]), "hm_build_cluster_tree: facet area must be > 0");
    auto t = std::make_unique<hm_tree>();
    t->n = n;
    t->params = *params;
    t->c.assign(centroid, centroid + 3 * n);
    t->nrm.assign(normal, normal + 3 * n);
    t->area.assign(area, area + n);
    build_tree(*t);
    *out = t.release();
    return HM_OK;
  } catch (const Error& e) {
    if (ctx) ctx->last_error = e.what(); else set_tl_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_tl_error("hm_build_cluster_tree: out of host memory");
    return HM_ENOMEM;
  }
}

hm_status hm_tree_stats(const hm_tree* t, int64_t* n_nodes, int64_t* n_dense, int64_t* n_lowrank, int32_t* perm_out) {
  if (!t) { set_tl_error("hm_tree_stats: NULL tree"); return HM_EINVAL; }
  if (n_nodes) *n_nodes = (int64_t)t->nodes.size();
  if (n_dense) *n_dense = (int64_t)t->dense.size();
  if (n_lowrank) *n_lowrank = (int64_t)t->lowrank.size();
  if (perm_out) std::copy(t->perm.begin(), t->perm.end(), perm_out);
  return HM_OK;
}

hm_status hm_tree_blocks(const hm_tree* t, int32_t* dense_out, int32_t* lowrank_out) {
  if (!t) { set_tl_error("hm_tree_blocks: NULL tree"); return HM_EINVAL; }
  auto put = [](const std::vector<BlockRef>& v, int32_t* o) {
    for (size_t k = 0; k < v.size(); ++k) {
      o[4 * k] = v[k].rb; o[4 * k + 1] = v[k].re; o[4 * k + 2] = v[k].cb; o[4 * k + 3] = v[k].ce;
    }
  };
  if (dense_out) put(t->dense, dense_out);
  if (lowrank_out) put(t->lowrank, lowrank_out);
  return HM_OK;
}

void hm_tree_destroy(hm_tree* t) { delete t; }

}  // extern "C"
