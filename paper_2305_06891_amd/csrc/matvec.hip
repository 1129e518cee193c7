// Block-wise H-matrix product on gfx950 (Sec. 5.2): y = F_H x with
//   phase 1:  t_b = V_b^T x_tau          for every low-rank block b
//   phase 2:  y_sigma += D_b x_tau  and  y_sigma += U_b t_b, row tile by row tile.
// Both phases are bandwidth kernels: every stored entry is read once per
// product (non-temporal loads), from panels packed so that each lane loads
// four consecutive entries (8-32 bytes) and each wave load is one contiguous
// run (see the layouts in hm_internal.hpp).  Phase 2 runs one workgroup per
// row tile whose waves share the tile's items (cut to nearly equal column
// counts) and add their sums in LDS in a fixed order; phase-1
// groups whose rows are split over several items write partials that a
// separate kernel adds in item order.  No kernel communicates across
// workgroups, so results do not depend on scheduling.  Several matrices can
// be multiplied in one launch ("slots" of a block-diagonal operator).
#include <algorithm>
#include <type_traits>
#include <cmath>
#include <map>
#include <numeric>

#include "dev_common.hpp"
#include "hm_internal.hpp"

namespace hm {

// ------------------------------------------------------------------ plan
namespace {

constexpr int64_t ITEM_BYTES = 64 << 10;  // target matrix bytes per phase-2 item (FP32)

struct Tile {
  int32_t row0, m;
};

inline int32_t round4(int32_t v) { return (v + 3) & ~3; }

}  // namespace

void plan_host(hm_matrix& M, const std::vector<LrInfo>& lr, const std::vector<BlockRef>& dn, const hm_tree& t,
               PackLists& pk) {
  Plan& P = M.plan;
  P.p1.clear();
  P.p1red.clear();
  P.p2t.clear();
  P.p2.clear();
  P.segs.clear();
  pk.nf.clear();
  pk.ur.clear();
  pk.vr.clear();
  // ---- column clusters of the low-rank blocks, their group panels and t layout
  std::vector<int32_t> ord(lr.size());
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
    const BlockRef &x = lr[a].b, &y = lr[b].b;
    if (x.cb != y.cb) return x.cb < y.cb;
    if (x.ce != y.ce) return x.ce < y.ce;
    return x.rb < y.rb;
  });
  std::vector<int32_t> tidx(lr.size());  // t index of rank column 0 of each block
  int64_t tcur = 0, vcur = 0;
  P.taus.clear();
  for (size_t q = 0; q < ord.size();) {
    size_t e = q;
    const BlockRef& b0 = lr[ord[q]].b;
    int32_t ktau = 0;
    while (e < ord.size() && lr[ord[e]].b.cb == b0.cb && lr[ord[e]].b.ce == b0.ce) ktau += lr[ord[e++]].k;
    const int32_t n = b0.ce - b0.cb, np = round4(n);
    const int64_t tau_base = vcur;
    int32_t lc = 0;
    for (size_t z = q; z < e; ++z) {
      const LrInfo& L = lr[ord[z]];
      tidx[ord[z]] = (int32_t)(tcur + lc);
      pk.vr.push_back(VRepack{L.sv, tau_base, L.stage, n, L.k, lc, ktau, np, L.b.cb, L.b.rb});
      lc += L.k;
    }
    P.taus.push_back(P1Tau{tau_base, tcur, b0.cb, n, np, ktau});
    vcur += (int64_t)np * (ktau + (ktau & 1));
    tcur += ktau;
    q = e;
  }
  HM_REQUIRE(tcur < (int64_t)1 << 30, "build_plan: too many rank columns");
  P.v_elems = vcur;
  // ---- row tiles: leaves cut into <= TILE rows
  std::vector<Tile> tiles;
  for (int32_t li : t.leaves) {
    const auto& nd = t.nodes[li];
    const int32_t sz = nd.end - nd.begin;
    const int32_t nt = (sz + TILE - 1) / TILE;
    for (int32_t q = 0; q < nt; ++q) {
      const int32_t a = nd.begin + (int32_t)((int64_t)sz * q / nt);
      const int32_t b = nd.begin + (int32_t)((int64_t)sz * (q + 1) / nt);
      tiles.push_back(Tile{a, b - a});
    }
  }
  std::vector<int32_t> row0s(tiles.size());
  for (size_t q = 0; q < tiles.size(); ++q) row0s[q] = tiles[q].row0;
  // ---- per-tile column runs: (kind, src, width, block index)
  struct Run {
    int32_t kind, src, w, blk;
  };
  std::vector<std::vector<Run>> truns(tiles.size());
  auto add = [&](const BlockRef& b, int32_t kind, int32_t src, int32_t w, int32_t blk) {
    size_t q = std::lower_bound(row0s.begin(), row0s.end(), b.rb) - row0s.begin();
    for (; q < tiles.size() && tiles[q].row0 < b.re; ++q) truns[q].push_back(Run{kind, src, w, blk});
  };
  for (size_t q = 0; q < dn.size(); ++q) add(dn[q], 0, dn[q].cb, dn[q].ce - dn[q].cb, (int32_t)q);
  for (size_t q = 0; q < lr.size(); ++q) add(lr[q].b, 1, ~tidx[q], lr[q].k, (int32_t)q);
  int64_t dcur = 0, ucur = 0;
  for (size_t q = 0; q < tiles.size(); ++q) {
    auto& v = truns[q];
    std::stable_sort(v.begin(), v.end(), [](const Run& a, const Run& b) {
      if (a.kind != b.kind) return a.kind < b.kind;
      return a.src < b.src;
    });
    const int32_t m = tiles[q].m;
    const int32_t row0 = tiles[q].row0;
    P2Tile tl{row0, m, (int32_t)P.p2.size(), 0};
    // columns of each kind, split into parts of nearly equal width so that
    // the waves of the tile's workgroup get the same number of bytes
    int32_t W[2] = {0, 0};
    for (const Run& r : v) W[r.kind] += r.w;
    const int32_t Wt = W[0] + W[1];
    const int32_t cN = (Wt + P2_WAVES * P2_MAXW - 1) / (P2_WAVES * P2_MAXW);
    const int32_t N = std::max<int32_t>(1, std::min<int32_t>(P2_WAVES * std::max(1, cN), (Wt + 15) / 16));
    int32_t nk[2];
    nk[0] = W[0] > 0 ? std::max<int32_t>(1, (int32_t)std::lround((double)N * W[0] / std::max(1, Wt))) : 0;
    nk[1] = W[1] > 0 ? std::max<int32_t>(1, N - nk[0]) : 0;
    for (int kd = 0; kd < 2; ++kd)
      if (W[kd] > 0) nk[kd] = std::max(nk[kd], (W[kd] + P2_MAXW - 1) / P2_MAXW);
    // walk the runs of each kind, cutting at the part boundaries
    size_t r0 = 0;
    for (int kd = 0; kd < 2; ++kd) {
      std::vector<Run> kv;
      while (r0 < v.size() && v[r0].kind == kd) kv.push_back(v[r0++]);
      if (kv.empty()) continue;
      std::vector<int32_t> cut;
      for (int32_t i = 0; i <= nk[kd]; ++i)
        cut.push_back(i == nk[kd] ? W[kd] : std::min(W[kd], round4((int32_t)((int64_t)W[kd] * i / nk[kd]))));
      size_t ri = 0;
      int32_t roff = 0;  // columns of kv[ri] already used
      for (int32_t i = 0; i < nk[kd]; ++i) {
        int32_t want = cut[i + 1] - cut[i];
        while (want > 0) {
          // one item: up to want columns and P2_MAXSEG runs
          P2Item it{};
          it.kind = kd;
          it.seg0 = (int32_t)P.segs.size();
          int32_t col = 0;
          while (want > 0 && (int32_t)P.segs.size() - it.seg0 < P2_MAXSEG) {
            const Run& R = kv[ri];
            const int32_t take = std::min(want, R.w - roff);
            const int32_t src = kd == 0 ? R.src + roff : ~((~R.src) + roff);
            P.segs.push_back(Seg{col, take, src, 0});
            if (kd == 0) {
              pk.nf.push_back(NfDev{0, row0, m, R.src + roff, take, col, 0});
            } else {
              const LrInfo& L = lr[R.blk];
              const int32_t ld = L.b.re - L.b.rb;
              pk.ur.push_back(URepack{L.su + (row0 - L.b.rb) + (int64_t)roff * ld, 0, L.stage, ld, m, take, col, row0,
                                      L.b.cb, roff});
            }
            col += take;
            want -= take;
            roff += take;
            if (roff == R.w) {
              ++ri;
              roff = 0;
            }
          }
          it.nseg = (int32_t)P.segs.size() - it.seg0;
          it.w = round4(col);
          int64_t& cur = kd == 0 ? dcur : ucur;
          it.base = cur;
          cur += (int64_t)m * it.w;
          // the packing entries just added belong to this item
          if (kd == 0)
            for (size_t z = pk.nf.size() - it.nseg; z < pk.nf.size(); ++z) pk.nf[z].base = it.base;
          else
            for (size_t z = pk.ur.size() - it.nseg; z < pk.ur.size(); ++z) pk.ur[z].base = it.base;
          P.p2.push_back(it);
        }
      }
    }
    tl.nit = (int32_t)P.p2.size() - tl.it0;
    P.p2t.push_back(tl);
  }
  P.dense_elems = dcur;
  P.u_elems = ucur;
  plan_phase1(P, P.p1p);
  M.Ktot = tcur;
}

void plan_phase1(Plan& P, const P1Params& pp) {
  HM_REQUIRE(pp.rows >= 64 && pp.rows % 64 == 0 && pp.task_bytes >= 0, "plan: bad phase-1 split");
  P.p1p = pp;
  P.p1.clear();
  P.p1red.clear();
  P.p1_task.assign(1, 0);
  int32_t parts = 0;
  int64_t acc = 0;
  const int32_t qch = pp.rows / 4;
  for (const P1Tau& T : P.taus) {
    const int32_t ngroups = (T.ktau + P1_GW - 1) / P1_GW;
    const int32_t nq = T.np / 4;
    const int32_t nch = (nq + qch - 1) / qch;
    for (int32_t g = 0; g < ngroups; ++g) {
      const int32_t gw = std::min(P1_GW, T.ktau - g * P1_GW);
      const int32_t trow = (int32_t)(T.trow + g * P1_GW);
      if (nch > 1) P.p1red.push_back(P1Red{trow, gw, parts, nch});
      for (int32_t c = 0; c < nch; ++c) {
        P1Item it{};
        it.base = T.vbase + (int64_t)g * P1_GW * T.np;
        it.gw = gw;
        it.gs = gw + (gw & 1);
        it.q0 = c * qch;
        it.nq = std::min(qch, nq - c * qch);
        it.nrows = T.n;
        it.xrow = T.xrow;
        it.trow = trow;
        it.part = nch > 1 ? parts + c : -1;
        P.p1.push_back(it);
        // consecutive items of at least task_bytes form one wave's task
        acc += (int64_t)it.nq * 4 * gw * 4;
        if (acc >= pp.task_bytes) {
          P.p1_task.push_back((int32_t)P.p1.size());
          acc = 0;
        }
      }
      if (nch > 1) parts += nch;
    }
  }
  if (P.p1_task.back() != (int32_t)P.p1.size()) P.p1_task.push_back((int32_t)P.p1.size());
  P.n_p1_parts = parts;
}

void replan_phase1(hm_matrix& M, const P1Params& pp, hipStream_t s) {
  Plan& P = M.plan;
  plan_phase1(P, pp);
  upload(P.d_p1, P.p1, s);
  upload(P.d_p1_task, P.p1_task, s);
  upload(P.d_p1red, P.p1red, s);
  HM_HIP(hipStreamSynchronize(s));
}

void build_plan(hm_matrix& M, const std::vector<LrInfo>& lr, const std::vector<BlockRef>& dn, const hm_tree& t,
                PackLists& pk, hipStream_t s) {
  plan_host(M, lr, dn, t, pk);
  Plan& P = M.plan;
  upload(P.d_p1, P.p1, s);
  upload(P.d_p1_task, P.p1_task, s);
  upload(P.d_p1red, P.p1red, s);
  upload(P.d_p2t, P.p2t, s);
  upload(P.d_p2, P.p2, s);
  upload(P.d_segs, P.segs, s);
  HM_HIP(hipStreamSynchronize(s));
}

// Streams a buffer through the caches without writing it; the sum is
// stored only if it is NaN, which keeps the loads alive.
__global__ void k_tune_flush(const float4* __restrict__ p, int64_t n4, float* __restrict__ sink) {
  float acc = 0.f;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n4; k += (int64_t)gridDim.x * blockDim.x) {
    const float4 v = p[k];
    acc += v.x + v.y + v.z + v.w;
  }
  if (acc != acc) sink[0] = acc;
}

void autotune_phase1_joint(const std::vector<hm_matrix*>& mats, hipStream_t s, int width) {
  HM_REQUIRE(width >= 1 && width <= 16, "autotune: product width must be in 1..16");
  std::vector<hm_matrix*> ms;
  for (hm_matrix* M : mats)
    if (!M->plan.taus.empty()) ms.push_back(M);
  if (ms.empty()) return;
  // FP64 vectors only when every matrix stores FP64 factors
  const bool all64 = std::all_of(ms.begin(), ms.end(), [](const hm_matrix* M) { return M->lr_dtype == HM_F64; });
  const int vb = all64 ? 8 : 4;
  int64_t n = 0, vbytes = 0;
  for (const hm_matrix* M : ms) {
    n += M->n;
    vbytes += M->v_entries * (int64_t)dtype_size(M->lr_dtype);
  }
  // factors that could stay in the last-level cache are timed after a read
  // of 512 MB, as in the solve where phase 2 runs in between
  const int64_t flush_bytes = vbytes > (16 << 20) ? (int64_t)512 << 20 : 0;
  // products of the width the matrices will mostly see: with many columns
  // the partial sums of split column clusters cost as many times more, so
  // longer items are candidates too
  const int W = pad_width(width);
  DevBuf X((size_t)n * W * vb), Y((size_t)n * W * vb), flush(flush_bytes), sink(16);
  HM_HIP(hipMemsetAsync(X.get(), 0, (size_t)n * W * vb, s));
  if (flush_bytes) HM_HIP(hipMemsetAsync(flush.get(), 0, (size_t)flush_bytes, s));
  const std::vector<const hm_matrix*> cms(ms.begin(), ms.end());
  hipEvent_t ev[3];
  for (auto& e : ev) HM_HIP(hipEventCreate(&e));
  const std::vector<int> rows = width > 1 ? std::vector<int>{128, 256, 512, 1024} : std::vector<int>{64, 128, 256};
  const int task[] = {0, 8 << 10, 16 << 10, 32 << 10, 64 << 10};
  P1Params best = ms[0]->plan.p1p;
  double best_us = 1e30;
  try {
    for (int r : rows)
      for (int tb : task) {
        P1Params pp;
        pp.rows = r;
        pp.task_bytes = tb;
        for (hm_matrix* M : ms) replan_phase1(*M, pp, s);
        auto comp = make_composition(cms, W, vb, s);
        double tot = 0;
        const int reps = 6;
        for (int k = 0; k < reps + 1; ++k) {
          if (flush_bytes)
            hipLaunchKernelGGL(k_tune_flush, dim3(1024), dim3(256), 0, s, flush.get<float4>(), flush_bytes / 16,
                               sink.get<float>());
          launch_matvec(*comp, width, vb, false, X.get(), n, Y.get(), n, Epilogue{}, nullptr, s, ev);
          HM_HIP(hipEventSynchronize(ev[2]));
          float a = 0;
          HM_HIP(hipEventElapsedTime(&a, ev[0], ev[1]));
          if (k > 0) tot += a;  // the first product warms up
        }
        const double us = 1e3 * tot / reps;
        if (us < best_us) {
          best_us = us;
          best = pp;
        }
      }
  } catch (...) {
    for (auto& e : ev) (void)hipEventDestroy(e);
    throw;
  }
  for (hm_matrix* M : ms) {
    replan_phase1(*M, best, s);
    M->plan.p1_us = best_us;
    M->plan.p2_waves = 0;
    M->plan.p2_us = 0.0;
  }
  // phase 2 of one- and two-column products: 2, 4 or 8 waves per
  // workgroup (all give the same bits); the split above does not affect
  // phase 2
  int best_w = 0;
  double best_p2 = 1e30;
  try {
    if (W <= 2) {
      auto comp = make_composition(cms, W, vb, s);
      for (int w : {2, 4, 8}) {
        comp->p2_waves = w;
        double tot = 0;
        const int reps = 6;
        for (int k = 0; k < reps + 1; ++k) {
          launch_matvec(*comp, width, vb, false, X.get(), n, Y.get(), n, Epilogue{}, nullptr, s, ev);
          HM_HIP(hipEventSynchronize(ev[2]));
          float a = 0;
          HM_HIP(hipEventElapsedTime(&a, ev[1], ev[2]));
          if (k > 0) tot += a;
        }
        const double us = 1e3 * tot / reps;
        if (us < best_p2) {
          best_p2 = us;
          best_w = w;
        }
      }
    }
  } catch (...) {
    for (auto& e : ev) (void)hipEventDestroy(e);
    throw;
  }
  for (auto& e : ev) HM_HIP(hipEventDestroy(e));
  if (best_w)
    for (hm_matrix* M : ms) {
      M->plan.p2_waves = best_w;
      M->plan.p2_us = best_p2;
    }
}

void autotune_phase1(hm_matrix& M, hipStream_t s, int width) { autotune_phase1_joint({&M}, s, width); }

int64_t matrix_bytes(const hm_matrix& M, bool hi) {
  const size_t dsz = hi && M.has_hi && M.dense_dtype == HM_BF16 ? 4 : dtype_size(M.dense_dtype);
  const size_t lsz = hi && M.has_hi ? 4 : dtype_size(M.lr_dtype);
  return M.dense_entries * (int64_t)dsz + M.lr_entries * (int64_t)lsz;
}

std::unique_ptr<Composition> make_composition(const std::vector<const hm_matrix*>& mats, int nr, int vec_bytes,
                                              hipStream_t s) {
  HM_REQUIRE(nr == 1 || nr == 2 || nr == 4 || nr == 8 || nr == 16, "matvec: composition width must be 1, 2, 4, 8 or 16");
  auto C = std::make_unique<Composition>();
  C->nr = nr;
  C->vec_bytes = vec_bytes;
  C->mats = mats;
  int64_t tsz = 0, p1 = 0;
  for (const auto* M : mats) {
    C->xoff.push_back(C->N);
    C->N += M->n;
    tsz += M->Ktot;
    p1 += M->plan.n_p1_parts;
  }
  const int64_t eb = 8;  // buffers sized for FP64 so one composition serves both vector types
  C->t.alloc(std::max<int64_t>(1, tsz * nr) * eb);
  C->part1.alloc(std::max<int64_t>(1, p1 * P1_GW * nr) * eb);
  if (nr == 16) C->xr.alloc(std::max<int64_t>(1, C->N) * 16 * eb);
  int64_t to = 0;
  p1 = 0;
  int32_t t1 = 0, r1 = 0, t2 = 0;
  for (size_t q = 0; q < mats.size(); ++q) {
    const hm_matrix& M = *mats[q];
    SlotDev d{};
    d.p1 = M.plan.d_p1.get<P1Item>();
    d.p1_task = M.plan.d_p1_task.get<int32_t>();
    d.p1red = M.plan.d_p1red.get<P1Red>();
    d.p2t = M.plan.d_p2t.get<P2Tile>();
    d.p2 = M.plan.d_p2.get<P2Item>();
    d.segs = M.plan.d_segs.get<Seg>();
    d.dense = M.dense.get();
    d.U = M.U.get();
    d.V = M.V.get();
    d.part1 = C->part1.get<char>() + p1 * P1_GW * nr * eb;
    d.t = C->t.get<char>() + to * nr * eb;
    d.ldt = std::max<int64_t>(1, M.Ktot);
    d.xoff = C->xoff[q];
    d.p1_task_begin = t1;
    d.p1red_begin = r1;
    d.p2_tile_begin = t2;
    d.n = (int32_t)M.n;
    d.slot = (int32_t)q;
    t1 += (int32_t)M.plan.p1_task.size() - 1;
    r1 += (int32_t)M.plan.p1red.size();
    t2 += (int32_t)M.plan.p2t.size();
    to += M.Ktot;
    p1 += M.plan.n_p1_parts;
    C->slots_lo.push_back(d);
    SlotDev h = d;
    if (M.has_hi) {
      h.U = M.U_hi.get();
      h.V = M.V_hi.get();
      if (M.dense_dtype == HM_BF16) h.dense = M.dense_hi.get();
    }
    C->slots_hi.push_back(h);
    C->bytes_lo += matrix_bytes(M, false);
    C->bytes_hi += matrix_bytes(M, true);
  }
  C->p1_tasks = t1;
  C->p1_reds = r1;
  C->p2_tiles = t2;
  C->p2_waves = mats[0]->plan.p2_waves;
  for (const hm_matrix* M : mats)
    if (M->plan.p2_waves != C->p2_waves) C->p2_waves = 0;
  C->slot_of.clear();
  for (int pass = 0; pass < 3; ++pass)
    for (size_t q = 0; q < mats.size(); ++q) {
      const Plan& P = mats[q]->plan;
      const size_t cnt = pass == 0 ? P.p1_task.size() - 1 : (pass == 1 ? P.p1red.size() : P.p2t.size());
      C->slot_of.insert(C->slot_of.end(), cnt, (int32_t)q);
    }
  C->slot_of.push_back(0);  // never empty
  upload(C->d_slot_of, C->slot_of, s);
  upload(C->d_slots_lo, C->slots_lo, s);
  upload(C->d_slots_hi, C->slots_hi, s);
  HM_HIP(hipStreamSynchronize(s));
  return C;
}

// ------------------------------------------------------------------ kernels
template <class VT>
struct EpiDev {
  const VT* rowscale;
  VT a_acc, a_x, a_z;
  const VT* z;
  int64_t ldz;
  VT* acc_out;  // optional second output: the plain product
  int64_t ld_acc;
};

// Four consecutive panel entries in their stored type (one 8-32 byte load);
// they are converted to the vector type only when they are used, so a batch
// of loads in flight costs the stored bytes in registers, not the widened ones.
// The loads are non-temporal: each panel entry is read once per product
// and the panels exceed the last-level cache, so caching them would only
// displace the vectors and partial sums that are reused.
using f32x4 = float __attribute__((ext_vector_type(4)));
using f64x2 = double __attribute__((ext_vector_type(2)));
using u32x2 = uint32_t __attribute__((ext_vector_type(2)));

template <class MT> struct Quad;
template <> struct Quad<float> {
  f32x4 v;
  __device__ void zero() { v = f32x4{0.f, 0.f, 0.f, 0.f}; }
  __device__ void load(const float* p) { v = ld_stream(reinterpret_cast<const f32x4*>(p)); }
  template <class VT> __device__ VT get(int e) const { return (VT)v[e]; }
};
template <> struct Quad<double> {
  f64x2 a, b;
  __device__ void zero() { a = b = f64x2{0.0, 0.0}; }
  __device__ void load(const double* p) {
    a = ld_stream(reinterpret_cast<const f64x2*>(p));
    b = ld_stream(reinterpret_cast<const f64x2*>(p) + 1);
  }
  template <class VT> __device__ VT get(int e) const { return (VT)(e < 2 ? a[e] : b[e - 2]); }
};
template <> struct Quad<bf16_t> {
  u32x2 v;
  __device__ void zero() { v = u32x2{0u, 0u}; }
  __device__ void load(const bf16_t* p) { v = ld_stream(reinterpret_cast<const u32x2*>(p)); }
  template <class VT> __device__ VT get(int e) const {
    const uint32_t w = v[e >> 1];
    return (VT)bf16_to_f32((bf16_t)((e & 1) ? (w >> 16) : (w & 0xffffu)));
  }
};

// Ordering of LDS traffic inside one wave (no workgroup barrier: the waves
// of a workgroup run independent tasks).  A wave's LDS operations execute in
// issue order, so only the compiler must keep them in program order: a
// signal fence does that without waiting on outstanding global loads.
__device__ __forceinline__ void wave_lds_sync() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <class VT, int NR>
__device__ __forceinline__ void epilogue_store(int row, int lane, int m, int nrr, const VT* acc,
                                               const VT* __restrict__ X, int64_t ldx, VT* __restrict__ Y,
                                               int64_t ldy, const EpiDev<VT>& ep) {
  if (lane >= m) return;
  const VT w = ep.rowscale ? gbl(ep.rowscale)[row] : VT(1);
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    if (j >= nrr) break;
    VT o = ep.a_acc * w * acc[j];
    if (ep.a_x != VT(0)) o += ep.a_x * gbl(X)[row + j * ldx];
    if (ep.a_z != VT(0)) o += ep.a_z * gbl(ep.z)[row + j * ep.ldz];
    gbl_w(Y)[row + j * ldy] = o;
    if (ep.acc_out) gbl_w(ep.acc_out)[row + j * ep.ld_acc] = acc[j];
  }
}

// Quads per load batch of the second kernel; two batches are in flight
// (the next one is loaded while the current one is used): 8 quads of FP32
// entries with FP32 sums, 16 of BF16 entries (the same bytes), 4 with FP64
// entries or sums or several right-hand sides, which take more registers.
template <class MT, class VT, int NR>
constexpr int load_depth() {
  return (NR > 1 || sizeof(VT) == 8 || sizeof(MT) == 8) ? 4 : (sizeof(MT) == 2 ? 16 : 8);
}

// One batch: quads [g, g + UN) of a panel row (the tail re-reads quad g1 - 1
// instead of branching; its terms are skipped).
template <class MT, int UN>
__device__ __forceinline__ void quads_load(Quad<MT> (&v)[UN], const MT* __restrict__ a, int64_t step, int g, int g1) {
#pragma unroll
  for (int u = 0; u < UN; ++u) v[u].load(a + (int64_t)(g + u < g1 ? g + u : g1 - 1) * step);
}

// acc[j] += sum over the batch's quads (< g1) of A(row, c) * in[c - 4 g0][j].
template <class MT, class VT, int NR, int UN>
__device__ __forceinline__ void quads_fma(const Quad<MT> (&v)[UN], int g, int g0, int g1, const VT* __restrict__ in,
                                          VT* acc) {
#pragma unroll
  for (int u = 0; u < UN; ++u)
    if (g + u < g1)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const VT w = v[u].template get<VT>(e);
#pragma unroll
        for (int j = 0; j < NR; ++j) acc[j] += w * in[((g - g0 + u) * 4 + e) * NR + j];
      }
}

// Staged columns per chunk: at most P2_MAXW and 4 KB of inputs per wave.
template <class VT, int NR>
constexpr int p2_chunk() {
  return (int)std::min<int64_t>(P2_MAXW, ((4096 / ((int64_t)NR * sizeof(VT))) / 4) * 4);
}

// Inputs of item columns [c0, c0 + cw) staged in two steps, so that panel
// loads can be issued in between and stay in flight (the vector-memory
// counter retires loads in issue order): stage_issue finds the run of each
// of the lane's columns (LDS) and issues its gathers into registers;
// stage_commit writes them to LDS (in[col][rhs]).  Columns past the item's
// width read 0; clamped addresses keep every gather in bounds.
template <class VT, int NR, int CW>
struct Staged {
  static constexpr int K = CW >= 64 ? CW / 64 : 1;
  VT v[K][NR];
};

template <class VT, int NR, int CW>
__device__ __forceinline__ void stage_issue(Staged<VT, NR, CW>& st, const Seg* sg_lds, int nseg, int wtrue, int c0,
                                            int cw, int lane, int nrr, const VT* Xs, int64_t ldx, const VT* Ts,
                                            int64_t ldt) {
#pragma unroll
  for (int k = 0; k < Staged<VT, NR, CW>::K; ++k) {
    const int cc = lane + 64 * k;
    const int c = c0 + cc;
    const bool valid = cc < cw && c < wtrue;
    const int cs = min(c, wtrue - 1);
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (sg_lds[mid].col0 <= cs) lo = mid;
      else hi = mid - 1;
    }
    const Seg sg = sg_lds[lo];
    const int kk = cs - sg.col0;
    const VT* src = sg.src >= 0 ? Xs + sg.src + kk : Ts + (~sg.src) + kk;
    const int64_t ld = sg.src >= 0 ? ldx : ldt;
    VT t[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) t[j] = gbl(src)[(int64_t)min(j, nrr - 1) * ld];
#pragma unroll
    for (int j = 0; j < NR; ++j) st.v[k][j] = (valid && j < nrr) ? t[j] : VT(0);
  }
}

template <class VT, int NR, int CW>
__device__ __forceinline__ void stage_commit(const Staged<VT, NR, CW>& st, VT* in, int lane, int cw) {
  wave_lds_sync();
#pragma unroll
  for (int k = 0; k < Staged<VT, NR, CW>::K; ++k) {
    const int cc = lane + 64 * k;
    if (cc < cw)
#pragma unroll
      for (int j = 0; j < NR; ++j) in[cc * NR + j] = st.v[k][j];
  }
  wave_lds_sync();
}

// acc += one item panel (m rows, w columns) times its inputs, chunk by
// chunk: the chunk's first batch of panel loads goes out before its inputs
// are staged, and each later batch is loaded while the previous one is used.
template <class MT, class VT, int NR>
__device__ __forceinline__ void panel_item(const MT* __restrict__ a, int m, int w, VT* in, const Seg* sg_lds, int nseg,
                                           int wtrue, int lane, int nrr, const VT* Xs, int64_t ldx, const VT* Ts,
                                           int64_t ldt, VT* acc) {
  constexpr int CW = p2_chunk<VT, NR>();
  constexpr int UN = load_depth<MT, VT, NR>();
  const int64_t step = (int64_t)m * 4;
  for (int c0 = 0; c0 < w; c0 += CW) {
    const int cw = min(CW, w - c0);
    const int g0 = c0 >> 2, g1 = (c0 + cw) >> 2;
    Staged<VT, NR, CW> st;
    stage_issue<VT, NR, CW>(st, sg_lds, nseg, wtrue, c0, cw, lane, nrr, Xs, ldx, Ts, ldt);
    Quad<MT> va[UN], vb[UN];
    quads_load<MT, UN>(va, a, step, g0, g1);
    stage_commit<VT, NR, CW>(st, in, lane, cw);
    for (int g = g0; g < g1; g += 2 * UN) {
      if (g + UN < g1) quads_load<MT, UN>(vb, a, step, g + UN, g1);
      quads_fma<MT, VT, NR, UN>(va, g, g0, g1, in, acc);
      if (g + UN >= g1) break;
      if (g + 2 * UN < g1) quads_load<MT, UN>(va, a, step, g + 2 * UN, g1);
      quads_fma<MT, VT, NR, UN>(vb, g + UN, g0, g1, in, acc);
    }
  }
}

// Row tile of phase-2 workgroup i among G.  Workgroups go to the eight
// XCDs in turn (i to XCD i % 8), each XCD with its own L2; neighbouring row
// tiles read many of the same input entries (x columns of shared near-field
// blocks, t rows of shared low-rank blocks), so each XCD takes runs of
// XCD_RUN consecutive tiles, the runs dealt out in turn (balanced like the
// plain order at run granularity).  Tiles past the last full round keep
// their index.  A renumbering only: every tile's result is the same.
constexpr int XCD_COUNT = 8, XCD_RUN = 8;
__device__ __forceinline__ int xcd_tile(int i, int G) {
  constexpr int R = XCD_COUNT * XCD_RUN;
  if (i >= (G / R) * R) return i;
  const int x = i % XCD_COUNT, k = i / XCD_COUNT;
  return ((k / XCD_RUN) * XCD_COUNT + x) * XCD_RUN + k % XCD_RUN;
}

// Phase 2: one workgroup of WG waves per row tile, lane = row of the tile;
// the waves share the tile's items (each takes every WG-th) and add their
// sums in LDS in wave order.  Compositions with many tiles and one or two
// right-hand sides run with four waves per workgroup (a workgroup's slots
// are released only when its last wave ends, and there are tiles enough to
// fill the GPU); the others with eight, one item per wave.
template <class DT, class LT, class VT, int NR, int WG>
__global__ __launch_bounds__(64 * WG) void k_phase2(const SlotDev* __restrict__ slots, const int* __restrict__ slot_of,
                                                          const int* __restrict__ slot_active, int nrr,
                                                          const VT* __restrict__ X, int64_t ldx,
                                                          VT* __restrict__ Y, int64_t ldy, EpiDev<VT> ep) {
  constexpr int CW = p2_chunk<VT, NR>();
  constexpr int RJ = NR < 4 ? NR : 4;
  // item k is summed in slot k % P2_WAVES whatever WG is, and the slots are
  // added in slot order, so every workgroup shape gives the same bits
  constexpr int SL = P2_WAVES / WG;  // slots per wave
  static_assert(P2_WAVES % WG == 0, "phase 2: WG must divide P2_WAVES");
  __shared__ VT lds_in[WG][CW * NR];
  __shared__ Seg lds_seg[WG][P2_MAXSEG];
  __shared__ VT lds_red[P2_WAVES][RJ][TILE];
  const int lane = threadIdx.x & 63;
  const int wv = uniform_int(threadIdx.x >> 6);  // wave index (uniform)
  const int tile = xcd_tile(blockIdx.x, gridDim.x);  // uniform
  const SlotDev S = uniform_load(slots + uniform_load(slot_of + tile));
  if (slot_active && !uniform_int(*gbl(slot_active + S.slot))) return;  // uniform over the workgroup
  const P2Tile T = uniform_load(S.p2t + (tile - S.p2_tile_begin));
  const VT* Xs = X + S.xoff;
  VT* Ys = Y + S.xoff;
  const VT* Ts = (const VT*)S.t;
  VT* in = lds_in[wv];
  Seg* sg_lds = lds_seg[wv];
  // lanes past the tile's rows repeat its last row; their sums are not stored
  const int prow = lane < T.m ? lane : T.m - 1;
  VT accs[SL][NR];
#pragma unroll
  for (int q = 0; q < SL; ++q)
#pragma unroll
    for (int j = 0; j < NR; ++j) accs[q][j] = VT(0);
  for (int k = wv; k < T.nit; k += WG) {
    VT* acc = accs[SL > 1 ? (k / WG) % SL : 0];
    const P2Item item = uniform_load(S.p2 + (T.it0 + k));
    wave_lds_sync();
    for (int q = lane; q < item.nseg; q += 64) sg_lds[q] = gbl(S.segs)[item.seg0 + q];
    wave_lds_sync();
    const Seg lastseg = sg_lds[item.nseg - 1];
    const int wtrue = lastseg.col0 + lastseg.w;
    if (item.kind == 0)
      panel_item<DT, VT, NR>((const DT*)S.dense + item.base + prow * 4, T.m, item.w, in, sg_lds, item.nseg, wtrue, lane,
                             nrr, Xs, ldx, Ts, S.ldt, acc);
    else
      panel_item<LT, VT, NR>((const LT*)S.U + item.base + prow * 4, T.m, item.w, in, sg_lds, item.nseg, wtrue, lane,
                             nrr, Xs, ldx, Ts, S.ldt, acc);
  }
  // combine the slots in order and finish the tile
  VT sum[NR];
#pragma unroll
  for (int j = 0; j < NR; ++j) sum[j] = VT(0);
#pragma unroll
  for (int j0 = 0; j0 < NR; j0 += RJ) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < SL; ++q)
#pragma unroll
      for (int j = 0; j < RJ; ++j) lds_red[wv + WG * q][j][lane] = accs[q][j0 + j];
    __syncthreads();
    if (wv == 0) {
#pragma unroll
      for (int j = 0; j < RJ; ++j) {
        VT t = lds_red[0][j][lane];
        for (int w = 1; w < P2_WAVES; ++w) t += lds_red[w][j][lane];
        sum[j0 + j] = t;
      }
    }
  }
  if (wv == 0) {
    EpiDev<VT> e = ep;
    if (e.rowscale) e.rowscale += S.xoff;
    if (e.z) e.z += S.xoff;
    if (e.acc_out) e.acc_out += S.xoff;
    epilogue_store<VT, NR>(T.row0 + lane, lane, T.m, nrr, sum, Xs, ldx, Ys, ldy, e);
  }
}

// Value of v held by lane l (l wave-uniform), for every lane.
__device__ __forceinline__ float lane_bcast(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_bcast(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Phase 1: t[trow + c] (+ j*ldt) = sum_r V(r, c) x(xrow + r) for the rank
// columns c of a group panel.  The rows of an item go in batches of UN
// quads (64 rows with BF16 entries); the x entries of a batch come with one
// coalesced load (lane = row).  The loads of the next batch are issued before
// the current one is used, so each wave keeps two batches in flight (no load
// of a pipelined batch sits behind a branch); with one right-hand side an
// item's last, partial batch loads its quads in groups of four instead of
// re-reading its last quad; rows past the item meet x = 0.
//
// FP32 and FP64 entries: lane l owns column l, reads one quad (16 or 32
// bytes) per row quad and takes x by lane broadcast.
// BF16 entries (8-byte quads): lane l owns the column pair 2 (l mod 32),
// 2 (l mod 32) + 1 and reads the pair's two quads of a row quad with one
// 16-byte load (panel rows of two columns start on 16-byte boundaries);
// lanes 0-31 take the even row quads of a batch and lanes 32-63 the odd
// ones, so a wave moves 1 KB per load instruction instead of 512 bytes.
// The halves need different x entries, which they read from the wave's LDS
// copy of the batch's x (one read per row quad), and they add their sums
// across halves at the end of the item.
template <class LT>
constexpr int p1_batch_quads() {
  return (int)(128 / sizeof(Quad<LT>));
}

template <class VT, int NR>
__device__ __forceinline__ void p1_load_x(VT (&x)[NR], bool& ok, const VT* xr, int64_t ldx, int nrr, int nrows, int qb,
                                          int qe, int nq_batch, int lane) {
  const int row = qb * 4 + lane;
  ok = lane < 4 * nq_batch && row < 4 * qe && row < nrows;
  const int rr = min(row, nrows - 1);
#pragma unroll
  for (int j = 0; j < NR; ++j) x[j] = gbl(xr)[rr + (int64_t)min(j, nrr - 1) * ldx];
}

// lane = column: UN quads of one column
template <class LT, class VT, int NR, int UN>
struct P1Batch {
  Quad<LT> v[UN];
  VT x[NR];
  bool ok;  // this lane's x row lies inside the item and the cavity

  // TAIL: the last, partial batch of an item: its quads are loaded in
  // groups of four (uniform branches), so at most three quads past the item
  // are read.  Otherwise quads past the item re-read its last quad.
  template <bool TAIL>
  __device__ __forceinline__ void issue(const LT* a, int64_t step, int qb, int qe, const VT* xr, int64_t ldx, int nrr,
                                        int nrows, int lane) {
    p1_load_x<VT, NR>(x, ok, xr, ldx, nrr, nrows, qb, qe, UN, lane);
#pragma unroll
    for (int g = 0; g < UN; g += 4) {
      if (!TAIL || qb + g < qe) {
#pragma unroll
        for (int u = g; u < g + 4; ++u) v[u].load(a + (int64_t)min(qb + u, qe - 1) * step);
      } else {
#pragma unroll
        for (int u = g; u < g + 4; ++u) v[u].zero();
      }
    }
  }

  __device__ __forceinline__ void use(int nrr, VT* acc) const {
    VT xm[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) xm[j] = (ok && j < nrr) ? x[j] : VT(0);
#pragma unroll
    for (int u = 0; u < UN; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const VT w = v[u].template get<VT>(e);
#pragma unroll
        for (int j = 0; j < NR; ++j) acc[j] += w * lane_bcast(xm[j], u * 4 + e);
      }
  }
};

using u32x4 = uint32_t __attribute__((ext_vector_type(4)));

// The four x entries of a row quad from LDS (16-byte aligned).
__device__ __forceinline__ void lds_quad(const float* p, float (&q)[4]) {
  const f32x4 v = *reinterpret_cast<const f32x4*>(p);
#pragma unroll
  for (int e = 0; e < 4; ++e) q[e] = v[e];
}
__device__ __forceinline__ void lds_quad(const double* p, double (&q)[4]) {
  const f64x2 a = reinterpret_cast<const f64x2*>(p)[0], b = reinterpret_cast<const f64x2*>(p)[1];
  q[0] = a[0];
  q[1] = a[1];
  q[2] = b[0];
  q[3] = b[1];
}

// lane = column pair (BF16 entries): UN / 2 row quads of two columns, row
// quad qb + 2u + h (h = lane / 32) in v[u]; quad words 0-1 hold the first
// column, 2-3 the second.
template <class VT, int NR, int UN>
struct P1Pair {
  u32x4 v[UN / 2];
  VT x[NR];
  bool ok;

  template <bool TAIL>
  __device__ __forceinline__ void issue(const bf16_t* a, int64_t step, int h, int qb, int qe, const VT* xr, int64_t ldx,
                                        int nrr, int nrows, int lane) {
    p1_load_x<VT, NR>(x, ok, xr, ldx, nrr, nrows, qb, qe, UN, lane);
#pragma unroll
    for (int g = 0; g < UN / 2; g += 2) {
      if (!TAIL || qb + 2 * g < qe) {
#pragma unroll
        for (int u = g; u < g + 2; ++u)
          v[u] = ld_stream(reinterpret_cast<const u32x4*>(a + (int64_t)min(qb + 2 * u + h, qe - 1) * step));
      } else {
#pragma unroll
        for (int u = g; u < g + 2; ++u) v[u] = u32x4{0u, 0u, 0u, 0u};
      }
    }
  }

  // xl: the wave's LDS copy of the batch's x (64 * NR entries)
  __device__ __forceinline__ void use(int nrr, int lane, int h, VT* xl, VT* acc0, VT* acc1) const {
#pragma unroll
    for (int j = 0; j < NR; ++j) xl[j * 64 + lane] = (ok && j < nrr) ? x[j] : VT(0);
    wave_lds_sync();
#pragma unroll
    for (int u = 0; u < UN / 2; ++u) {
      VT w0[4], w1[4];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        w0[2 * k] = (VT)__uint_as_float(v[u][k] << 16);
        w0[2 * k + 1] = (VT)__uint_as_float(v[u][k] & 0xffff0000u);
        w1[2 * k] = (VT)__uint_as_float(v[u][2 + k] << 16);
        w1[2 * k + 1] = (VT)__uint_as_float(v[u][2 + k] & 0xffff0000u);
      }
#pragma unroll
      for (int j = 0; j < NR; ++j) {
        VT xq[4];
        lds_quad(xl + j * 64 + (2 * u + h) * 4, xq);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          acc0[j] += w0[e] * xq[e];
          acc1[j] += w1[e] * xq[e];
        }
      }
    }
    wave_lds_sync();  // the reads are done before the next batch is written
  }
};

// The batches of one item [q0, q0 + nq): full batches with the next one in
// flight; with one right-hand side a partial last batch loads only its quads
// (with more, its loads are better kept in the pipeline: clamped quads).
template <class B, int UN, int NR, class Issue, class Use>
__device__ __forceinline__ void p1_batches(int q0, int nq, Issue issue, Use use) {
  const int qe = q0 + nq;
  const int qf = NR == 1 ? q0 + (nq / UN) * UN : qe;  // end of the pipelined batches
  int qb = q0;
  if (qb < qf) {
    B A, C;
    issue(A, qb, false);
    for (;;) {
      if (qb + UN >= qf) {
        use(A);
        break;
      }
      issue(C, qb + UN, false);
      use(A);
      qb += UN;
      if (qb + UN >= qf) {
        use(C);
        break;
      }
      issue(A, qb + UN, false);
      use(C);
      qb += UN;
    }
    qb = qf;
  }
  if constexpr (NR == 1) {
    if (qb < qe) {
      B T;
      issue(T, qb, true);
      use(T);
    }
  }
}

template <class LT, class VT, int NR, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_phase1(const SlotDev* __restrict__ slots, const int* __restrict__ slot_of, int ntasks,
                                                     const int* __restrict__ slot_active, int nrr,
                                                     const VT* __restrict__ X, int64_t ldx) {
  constexpr int UN = p1_batch_quads<LT>();
  constexpr bool PAIR = sizeof(LT) == 2;
  __shared__ __align__(16) VT p1x[PAIR ? WPB : 1][PAIR ? 64 * NR : 1];
  const int lane = threadIdx.x & 63;
  const int wv = uniform_int(threadIdx.x >> 6);  // wave index (uniform)
  const int task = blockIdx.x * WPB + wv;
  if (task >= ntasks) return;
  const SlotDev S = uniform_load(slots + uniform_load(slot_of + task));
  if (slot_active && !uniform_int(*gbl(slot_active + S.slot))) return;
  const int lt = task - S.p1_task_begin;
  const int ib = uniform_int(gbl(S.p1_task)[lt]), ie = uniform_int(gbl(S.p1_task)[lt + 1]);
  const VT* Xs = X + S.xoff;
  VT* T = (VT*)S.t;
  for (int it = ib; it < ie; ++it) {
    const P1Item item = uniform_load(S.p1 + it);
    const int64_t step = (int64_t)item.gs * 4;
    const VT* xr = Xs + item.xrow;
    const int qe = item.q0 + item.nq;
    VT res[NR];
    int col;  // the column whose sums this lane stores
    if constexpr (PAIR) {
      const int h = lane >> 5;
      // lanes past the group's columns repeat its last pair (not stored)
      const int pc = min(lane & 31, (item.gs >> 1) - 1);
      const bf16_t* a = (const bf16_t*)S.V + item.base + (int64_t)pc * 8;
      VT* xl = p1x[wv];
      VT acc0[NR], acc1[NR];
#pragma unroll
      for (int j = 0; j < NR; ++j) acc0[j] = acc1[j] = VT(0);
      using B = P1Pair<VT, NR, UN>;
      p1_batches<B, UN, NR>(
          item.q0, item.nq,
          [&](B& b, int qb, bool tail) {
            if (tail)
              b.template issue<true>(a, step, h, qb, qe, xr, ldx, nrr, item.nrows, lane);
            else
              b.template issue<false>(a, step, h, qb, qe, xr, ldx, nrr, item.nrows, lane);
          },
          [&](const B& b) { b.use(nrr, lane, h, xl, acc0, acc1); });
      // each half summed half of the row quads: add the other half's sums
      // (the same two terms in both halves, so both hold the same bits)
#pragma unroll
      for (int j = 0; j < NR; ++j) {
        acc0[j] += __shfl_xor(acc0[j], 32, 64);
        acc1[j] += __shfl_xor(acc1[j], 32, 64);
        res[j] = h ? acc1[j] : acc0[j];
      }
      col = 2 * (lane & 31) + h;
    } else {
      // lanes past the group's columns repeat its last column (not stored)
      const LT* a = (const LT*)S.V + item.base + (int64_t)min(lane, item.gw - 1) * 4;
#pragma unroll
      for (int j = 0; j < NR; ++j) res[j] = VT(0);
      using B = P1Batch<LT, VT, NR, UN>;
      p1_batches<B, UN, NR>(
          item.q0, item.nq,
          [&](B& b, int qb, bool tail) {
            if (tail)
              b.template issue<true>(a, step, qb, qe, xr, ldx, nrr, item.nrows, lane);
            else
              b.template issue<false>(a, step, qb, qe, xr, ldx, nrr, item.nrows, lane);
          },
          [&](const B& b) { b.use(nrr, res); });
      col = lane;
    }
    if (item.part < 0) {
      if (col < item.gw)
#pragma unroll
        for (int j = 0; j < NR; ++j)
          if (j < nrr) gbl_w(T)[item.trow + col + j * S.ldt] = res[j];
    } else {
      VT* P = (VT*)S.part1 + (int64_t)item.part * P1_GW * NR;
#pragma unroll
      for (int j = 0; j < NR; ++j) gbl_w(P)[j * P1_GW + col] = res[j];
    }
  }
}

// t of the row-split groups, lane = rank column.  WPR waves per group
// (1 with one or two right-hand sides, 4 with more, whose groups carry more
// partials): wave w reads the partials p = w, w + WPR, ... IL at a time into
// independent sums (IL * NR loads in flight per lane); the sums are added in
// a fixed order, so the result does not depend on the rest of the batch.
template <class VT, int NR>
constexpr int p1red_waves() {
  return NR >= 4 ? 4 : 1;
}

// ROWS: t is row-major (16 values a row, the matrix-core products), each
// lane storing its row in four 16-byte stores.
template <class VT, int NR, bool ROWS = false>
__global__ __launch_bounds__(256) void k_p1reduce(const SlotDev* __restrict__ slots, const int* __restrict__ slot_of,
                                                  int nreds, const int* __restrict__ slot_active, int nrr) {
  static_assert(!ROWS || NR == 16, "row-major t: 16 columns");
  constexpr int WPR = p1red_waves<VT, NR>();
  constexpr int IL = NR == 1 ? 8 : (NR == 2 ? 4 : (NR == 4 ? 2 : 1));
  __shared__ VT red[WPR > 1 ? WPR : 1][WPR > 1 ? NR : 1][64];
  const int lane = threadIdx.x & 63;
  const int wv = uniform_int(threadIdx.x >> 6);  // wave index (uniform)
  const int r = WPR > 1 ? blockIdx.x : blockIdx.x * 4 + wv;
  const int w = WPR > 1 ? wv : 0;
  if (r >= nreds) return;  // uniform over the workgroup when WPR > 1
  const SlotDev S = uniform_load(slots + uniform_load(slot_of + r));
  if (slot_active && !uniform_int(*gbl(slot_active + S.slot))) return;
  const P1Red R = uniform_load(S.p1red + (r - S.p1red_begin));
  const VT* P0 = (const VT*)S.part1 + (int64_t)R.part0 * P1_GW * NR;
  VT acc[IL][NR];
#pragma unroll
  for (int i = 0; i < IL; ++i)
#pragma unroll
    for (int j = 0; j < NR; ++j) acc[i][j] = VT(0);
  for (int p = w * IL; p < R.nparts; p += WPR * IL) {
#pragma unroll
    for (int i = 0; i < IL; ++i) {
      // past the last partial: re-read it and add nothing
      const int pi = p + i < R.nparts ? p + i : R.nparts - 1;
      const VT* Pp = P0 + (int64_t)pi * NR * P1_GW;
#pragma unroll
      for (int j = 0; j < NR; ++j) {
        const VT v = gbl(Pp)[j * P1_GW + lane];
        acc[i][j] += p + i < R.nparts ? v : VT(0);
      }
    }
  }
  VT sum[NR];
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    sum[j] = acc[0][j];
#pragma unroll
    for (int i = 1; i < IL; ++i) sum[j] += acc[i][j];
  }
  if constexpr (WPR > 1) {
#pragma unroll
    for (int j = 0; j < NR; ++j) red[wv][j][lane] = sum[j];
    __syncthreads();
    if (wv != 0) return;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      VT t = red[0][j][lane];
      for (int q = 1; q < WPR; ++q) t += red[q][j][lane];
      sum[j] = t;
    }
  }
  if (lane < R.gw) {
    VT* T = (VT*)S.t;
    if constexpr (ROWS) {
      // columns past nrr hold zero sums (their inputs are zero)
      VT* o = T + (int64_t)(R.trow + lane) * NR;
      if constexpr (std::is_same<VT, float>::value) {
        const gptr<f32x4> q = (gptr<f32x4>)gbl_w(o);
#pragma unroll
        for (int k = 0; k < NR / 4; ++k) q[k] = f32x4{sum[4 * k], sum[4 * k + 1], sum[4 * k + 2], sum[4 * k + 3]};
      } else {
        const gptr<f64x2> q = (gptr<f64x2>)gbl_w(o);
#pragma unroll
        for (int k = 0; k < NR / 2; ++k) q[k] = f64x2{sum[2 * k], sum[2 * k + 1]};
      }
    } else {
#pragma unroll
      for (int j = 0; j < NR; ++j)
        if (j < nrr) gbl_w(T)[R.trow + lane + j * S.ldt] = sum[j];
    }
  }
}

// ------------------------------------------------------------------ launch
namespace {

// ---- 16 right-hand sides: the products are dense contractions (16 rank
// columns or rows x 16 right-hand sides per 4-deep step) and run on the
// matrix cores, with v_mfma_f32_16x16x4f32 for FP32 vectors and
// v_mfma_f64_16x16x4f64 for FP64 vectors (the stored FP32/BF16 entries are
// widened exactly).  Operand layout of both for lane l (li = l % 16,
// lk = l / 16): A[li][lk], B[lk][li]; element v of the result holds
// D[4 lk + v][li] (FP32) or D[lk + 4 v][li] (FP64, rows interleaved).  The
// depth index of a step may stand for any four panel
// columns (or rows) as long as A and B agree, so each lane loads one
// 16-byte quad of its panel row and element e of the quad feeds step e: in
// step st lane group lk takes quad st + 4 lk of a 16-quad chunk, whose
// element e is chunk column (or row) 16 lk + 4 st + e.  One 16-byte load per
// lane serves four steps, as in the one-right-hand-side kernels.
//
// The vectors are read row-major (16 values a row): the input rows are
// copied to that order first, and t is written in it.  The rows of a chunk
// are staged in LDS with an odd row stride of 17 values: each lane's stores
// of its row, and the operand reads (lane groups 16 rows apart), then fall
// in distinct banks.

using f64x4 = double __attribute__((ext_vector_type(4)));
template <class VT> struct Acc16;
template <> struct Acc16<float> { using type = f32x4; };
template <> struct Acc16<double> { using type = f64x4; };
template <class VT> using acc16_t = typename Acc16<VT>::type;

// Row of the 16 x 16 result held in element v by lane group lk.
template <class VT> __device__ __forceinline__ int acc_row(int lk, int v) {
  return std::is_same<VT, double>::value ? lk + 4 * v : 4 * lk + v;
}

__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int IN16_LD = 17;  // LDS row stride of staged vector rows (values)
constexpr int P2M_WAVES = 4;  // waves per phase-2 workgroup (one row tile)

// Input rows of a 16-column product in row-major order: xr(r, j) = X(r, j)
// for j < nrr and 0 past it, so that a row's values come with 16-byte loads
// instead of a gather over 16 columns.
template <class VT>
__global__ __launch_bounds__(256) void k_rows16(const VT* __restrict__ X, int64_t ldx, int nrr, int64_t n,
                                               VT* __restrict__ xr) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  VT v[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) v[j] = j < nrr ? X[r + j * ldx] : VT(0);
  VT* o = xr + r * 16;
#pragma unroll
  for (int j = 0; j < 16; ++j) o[j] = v[j];
}

// A vector row of 16 values in registers (four or eight 16-byte loads).
template <class VT> struct Row16;
template <> struct Row16<float> {
  f32x4 v[4];
  __device__ void load(const float* p) {
    const gptr<const f32x4> q = (gptr<const f32x4>)gbl(p);
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = q[k];
  }
  __device__ float get(int j) const { return v[j >> 2][j & 3]; }
};
template <> struct Row16<double> {
  f64x2 v[8];
  __device__ void load(const double* p) {
    const gptr<const f64x2> q = (gptr<const f64x2>)gbl(p);
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = q[k];
  }
  __device__ double get(int j) const { return v[j >> 1][j & 1]; }
};

// Row `lane` of the chunk's staging area: the loaded row, or zero.
template <class VT>
__device__ __forceinline__ void stage_row16(const Row16<VT>& r, bool valid, VT* in, int lane) {
#pragma unroll
  for (int j = 0; j < 16; ++j) in[lane * IN16_LD + j] = valid ? r.get(j) : VT(0);
}

// acc[t] += the loaded quads times the staged rows of the chunk (zero past
// the item, so the clamped quads that meet them add nothing), for the NT
// 16-wide tiles that hold columns (phase 1) or rows (phase 2) of the item.
template <class MT, class VT, int NT>
__device__ __forceinline__ void mfma_quads16(const Quad<MT> (&av)[4][4], const VT* __restrict__ in, int li, int lk,
                                             acc16_t<VT>* acc) {
#pragma unroll
  for (int st = 0; st < 4; ++st) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const VT b = in[((st + 4 * lk) * 4 + e) * IN16_LD + li];
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = mfma16(av[st][t].template get<VT>(e), b, acc[t]);
    }
  }
}

// Phase 1, one item with NT column tiles: its 64-row chunks in turn.
template <class LT, class VT, int NT>
__device__ __forceinline__ void p1_item16(const char* vb, uint32_t step, const uint32_t (&coff)[4], const VT* xr,
                                          int q0b, int qe, int rend, VT* xs, int lane, int li, int lk,
                                          acc16_t<VT>* acc) {
  for (int q0 = q0b; q0 < qe; q0 += 16) {
    const int r0 = q0 * 4;
    // the chunk's x rows (clamped into the item; rows past it become zero
    // below), then its panel quads: one round trip covers both
    Row16<VT> xv;
    xv.load(xr + (int64_t)min(r0 + lane, rend - 1) * 16);
    Quad<LT> a[4][4];
    const char* vc = vb + (int64_t)q0 * step;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int q = q0 + st + 4 * lk;
      const uint32_t qo = (uint32_t)((q < qe ? q : qe - 1) - q0) * step;
#pragma unroll
      for (int t = 0; t < NT; ++t) a[st][t].load(reinterpret_cast<const LT*>(vc + (qo + coff[t])));
    }
    wave_lds_sync();
    stage_row16<VT>(xv, r0 + lane < rend, xs, lane);
    wave_lds_sync();
    mfma_quads16<LT, VT, NT>(a, xs, li, lk, acc);
  }
}

// Phase 1, 16 right-hand sides: t(trow + col, j) = sum_r V(r, col) x(xrow + r, j)
// for the <= 64 rank columns of a group panel (four 16-column tiles).  The
// x rows of a 64-row chunk are staged in LDS, zero past the item's rows.
template <class LT, class VT>
__global__ __launch_bounds__(256, sizeof(VT) == 4 ? 4 : 3) void k_phase1_mfma(const SlotDev* __restrict__ slots, const int* __restrict__ slot_of,
                                                        int ntasks, const int* __restrict__ slot_active,
                                                        const VT* __restrict__ Xr) {
  constexpr int NR = 16;
  using AT = acc16_t<VT>;
  __shared__ VT lds_x[4][64 * IN16_LD];
  const int lane = threadIdx.x & 63;
  const int wv = uniform_int(threadIdx.x >> 6);  // wave index (uniform)
  const int li = lane & 15, lk = lane >> 4;
  const int task = blockIdx.x * 4 + wv;
  if (task >= ntasks) return;
  const SlotDev S = uniform_load(slots + uniform_load(slot_of + task));
  if (slot_active && !uniform_int(*gbl(slot_active + S.slot))) return;
  const int lt = task - S.p1_task_begin;
  const int ib = uniform_int(gbl(S.p1_task)[lt]), ie = uniform_int(gbl(S.p1_task)[lt + 1]);
  VT* T = (VT*)S.t;
  VT* xs = lds_x[wv];
  for (int it = ib; it < ie; ++it) {
    const P1Item item = uniform_load(S.p1 + it);
    const int ntile = (item.gw + 15) >> 4;
    // 32-bit byte offsets from the chunk's wave-uniform base (a chunk spans
    // 16 quads of at most 64 columns): one address register per load
    const char* vb = reinterpret_cast<const char*>((const LT*)S.V + item.base);
    const uint32_t step = (uint32_t)item.gs * 4u * (uint32_t)sizeof(LT);
    // lanes past the group's columns repeat its last column (not stored)
    uint32_t coff[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) coff[t] = (uint32_t)min(16 * t + li, item.gw - 1) * 4u * (uint32_t)sizeof(LT);
    const VT* xr = Xr + (S.xoff + item.xrow) * NR;
    const int qe = item.q0 + item.nq;
    const int rend = min(item.nrows, qe * 4);
    AT acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = AT{0, 0, 0, 0};
    // only the column tiles that hold group columns are computed (in the
    // last one, lanes past the width repeat its last column, not stored)
    switch (ntile) {
      case 1: p1_item16<LT, VT, 1>(vb, step, coff, xr, item.q0, qe, rend, xs, lane, li, lk, acc); break;
      case 2: p1_item16<LT, VT, 2>(vb, step, coff, xr, item.q0, qe, rend, xs, lane, li, lk, acc); break;
      case 3: p1_item16<LT, VT, 3>(vb, step, coff, xr, item.q0, qe, rend, xs, lane, li, lk, acc); break;
      default: p1_item16<LT, VT, 4>(vb, step, coff, xr, item.q0, qe, rend, xs, lane, li, lk, acc); break;
    }
    if (item.part < 0) {
      // t row-major; columns past nrr hold zero (their inputs are zero)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int col = 16 * t + acc_row<VT>(lk, v);
          if (t < ntile && col < item.gw) gbl_w(T)[(int64_t)(item.trow + col) * NR + li] = acc[t][v];
        }
    } else {
      VT* P = (VT*)S.part1 + (int64_t)item.part * P1_GW * NR;
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (t < ntile) gbl_w(P)[li * P1_GW + 16 * t + acc_row<VT>(lk, v)] = acc[t][v];
    }
  }
}

// The 16 quads [g, g + 16) of an item panel of m rows, for the four 16-row
// tiles: lane group lk takes quad g + st + 4 lk in step st (lanes past m
// repeat row m - 1; quads past g1 repeat quad g1 - 1).  32-bit element
// offsets from the wave-uniform panel base (an item panel holds far fewer
// than 2^32 entries) keep one address register per load.
template <class MT, int NT>
__device__ __forceinline__ void load_quads16(Quad<MT> (&av)[4][4], const MT* __restrict__ a, int m, int g, int g1,
                                             int li, int lk) {
  const char* base = reinterpret_cast<const char*>(a);
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int q = g + st + 4 * lk;
    const uint32_t go = (uint32_t)(q < g1 ? q : g1 - 1) * (uint32_t)m * 4u;
#pragma unroll
    for (int rt = 0; rt < NT; ++rt) {
      const uint32_t off = (go + (uint32_t)min(16 * rt + li, m - 1) * 4u) * (uint32_t)sizeof(MT);
      av[st][rt].load(reinterpret_cast<const MT*>(base + off));
    }
  }
}

// Phase-2 inputs of chunk column c0 + lane: its row-major input row (x or
// t, found in the item's runs), or nothing past the chunk or the item.
template <class VT>
__device__ __forceinline__ bool stage16_issue(Row16<VT>& r, const Seg* sg_lds, int nseg, int wtrue, int c0, int cw,
                                              int lane, const VT* Xr, const VT* Tr) {
  const int c = c0 + lane;
  const int cs = min(c, wtrue - 1);
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sg_lds[mid].col0 <= cs) lo = mid;
    else hi = mid - 1;
  }
  const Seg sg = sg_lds[lo];
  const int kk = cs - sg.col0;
  r.load(sg.src >= 0 ? Xr + (int64_t)(sg.src + kk) * 16 : Tr + (int64_t)(~sg.src + kk) * 16);
  return lane < cw && c < wtrue;
}

// Phase 2, one item of a row tile with NT 16-row tiles: per chunk of 64
// columns the input loads and then the panel loads go out, the inputs are
// written to LDS while the panel loads are in flight, then 16 NT
// matrix-core steps.
template <class MT, class VT, int NT>
__device__ __forceinline__ void p2_item16(const MT* pa, int m, int w, const Seg* sg_lds, int nseg, int wtrue,
                                          int lane, int li, int lk, const VT* Xrs, const VT* Ts, VT* in,
                                          acc16_t<VT>* acc) {
  constexpr int CW = 64;  // staged columns per chunk
  for (int c0 = 0; c0 < w; c0 += CW) {
    const int cw = min(CW, w - c0);
    Row16<VT> xin;
    const bool valid = stage16_issue<VT>(xin, sg_lds, nseg, wtrue, c0, cw, lane, Xrs, Ts);
    Quad<MT> av[4][4];
    load_quads16<MT, NT>(av, pa, m, c0 >> 2, (c0 + cw) >> 2, li, lk);
    wave_lds_sync();
    stage_row16<VT>(xin, valid, in, lane);
    wave_lds_sync();
    mfma_quads16<MT, VT, NT>(av, in, li, lk, acc);
  }
}

// Phase 2, 16 right-hand sides: as k_phase2, with the row tile split into
// 16-row MFMA tiles (only those that hold rows are computed); WG waves share a tile's items (each takes every
// WG-th) and their sums meet in LDS in wave order.
template <class DT, class LT, class VT, int WG>
__global__ __launch_bounds__(64 * WG, sizeof(VT) == 4 ? 4 : 3) void k_phase2_mfma(const SlotDev* __restrict__ slots, const int* __restrict__ slot_of,
                                                                  const int* __restrict__ slot_active, int nrr,
                                                                  const VT* __restrict__ X, int64_t ldx,
                                                                  const VT* __restrict__ Xr,
                                                                  VT* __restrict__ Y, int64_t ldy, EpiDev<VT> ep) {
  constexpr int NR = 16;
  constexpr int CW = 64;  // staged columns per chunk
  using AT = acc16_t<VT>;
  static_assert(CW * IN16_LD >= NR * TILE, "the wave sums reuse the staging area");
  __shared__ VT lds_in[WG][CW * IN16_LD];  // reused for the wave sums [wave][rhs][row]
  __shared__ Seg lds_seg[WG][P2_MAXSEG];
  const int lane = threadIdx.x & 63;
  const int wv = uniform_int(threadIdx.x >> 6);  // wave index (uniform)
  const int li = lane & 15, lk = lane >> 4;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);  // uniform
  const SlotDev S = uniform_load(slots + uniform_load(slot_of + tile));
  if (slot_active && !uniform_int(*gbl(slot_active + S.slot))) return;  // uniform over the workgroup
  const P2Tile T = uniform_load(S.p2t + (tile - S.p2_tile_begin));
  const VT* Xs = X + S.xoff;
  VT* Ys = Y + S.xoff;
  const VT* Xrs = Xr + S.xoff * NR;
  const VT* Ts = (const VT*)S.t;
  VT* in = lds_in[wv];
  Seg* sg_lds = lds_seg[wv];
  const int ntile = (T.m + 15) >> 4;  // 16-row tiles holding rows (uniform)
  AT acc[4];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) acc[rt] = AT{0, 0, 0, 0};
  for (int k = wv; k < T.nit; k += WG) {
    const P2Item item = uniform_load(S.p2 + (T.it0 + k));
    wave_lds_sync();
    for (int q = lane; q < item.nseg; q += 64) sg_lds[q] = gbl(S.segs)[item.seg0 + q];
    wave_lds_sync();
    const Seg lastseg = sg_lds[item.nseg - 1];
    const int wtrue = lastseg.col0 + lastseg.w;
    if (item.kind == 0) {
      const DT* pa = (const DT*)S.dense + item.base;
      switch (ntile) {
        case 1: p2_item16<DT, VT, 1>(pa, T.m, item.w, sg_lds, item.nseg, wtrue, lane, li, lk, Xrs, Ts, in, acc); break;
        case 2: p2_item16<DT, VT, 2>(pa, T.m, item.w, sg_lds, item.nseg, wtrue, lane, li, lk, Xrs, Ts, in, acc); break;
        case 3: p2_item16<DT, VT, 3>(pa, T.m, item.w, sg_lds, item.nseg, wtrue, lane, li, lk, Xrs, Ts, in, acc); break;
        default: p2_item16<DT, VT, 4>(pa, T.m, item.w, sg_lds, item.nseg, wtrue, lane, li, lk, Xrs, Ts, in, acc); break;
      }
    } else {
      const LT* pa = (const LT*)S.U + item.base;
      switch (ntile) {
        case 1: p2_item16<LT, VT, 1>(pa, T.m, item.w, sg_lds, item.nseg, wtrue, lane, li, lk, Xrs, Ts, in, acc); break;
        case 2: p2_item16<LT, VT, 2>(pa, T.m, item.w, sg_lds, item.nseg, wtrue, lane, li, lk, Xrs, Ts, in, acc); break;
        case 3: p2_item16<LT, VT, 3>(pa, T.m, item.w, sg_lds, item.nseg, wtrue, lane, li, lk, Xrs, Ts, in, acc); break;
        default: p2_item16<LT, VT, 4>(pa, T.m, item.w, sg_lds, item.nseg, wtrue, lane, li, lk, Xrs, Ts, in, acc); break;
      }
    }
  }
  __syncthreads();
  VT* red = &lds_in[0][0];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int v = 0; v < 4; ++v) red[(wv * NR + li) * TILE + 16 * rt + acc_row<VT>(lk, v)] = acc[rt][v];
  __syncthreads();
  if (wv == 0) {
    VT sum[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) sum[j] = red[j * TILE + lane];
    for (int w = 1; w < WG; ++w)
#pragma unroll
      for (int j = 0; j < NR; ++j) sum[j] += red[(w * NR + j) * TILE + lane];
    EpiDev<VT> e = ep;
    if (e.rowscale) e.rowscale += S.xoff;
    if (e.z) e.z += S.xoff;
    if (e.acc_out) e.acc_out += S.xoff;
    epilogue_store<VT, NR>(T.row0 + lane, lane, T.m, nrr, sum, Xs, ldx, Ys, ldy, e);
  }
}

template <class VT, int NR>
constexpr int p1_waves_per_block() {
  return 4;
}

template <class DT, class LT, class VT, int NR>
void launch_typed(const CompView& C, int nrr, bool hi, const void* X, int64_t ldx, void* Y, int64_t ldy,
                  const Epilogue& ep, const int* slot_active, hipStream_t s, hipEvent_t* ev) {
  constexpr int WPB = p1_waves_per_block<VT, NR>();
  const SlotDev* slots = hi ? C.slots_hi : C.slots_lo;
  const int* sof = C.slot_of;
  // 16 right-hand sides of FP32/BF16 entries: matrix cores (FP32 or FP64 sums)
  constexpr bool mfma = NR == 16 && sizeof(DT) <= 4 && sizeof(LT) <= 4;
  if (ev) HM_HIP(hipEventRecord(ev[0], s));
  if constexpr (mfma) {
    HM_REQUIRE(C.xr != nullptr, "matvec: 16-column composition without its row-major input buffer");
    if (C.N > 0)
      hipLaunchKernelGGL(k_rows16<VT>, dim3((unsigned)((C.N + 255) / 256)), dim3(256), 0, s, (const VT*)X, ldx, nrr,
                         C.N, (VT*)C.xr);
  }
  if (C.p1_tasks > 0) {
    if constexpr (mfma)
      hipLaunchKernelGGL((k_phase1_mfma<LT, VT>), dim3((C.p1_tasks + 3) / 4), dim3(256), 0, s, slots, sof,
                         C.p1_tasks, slot_active, (const VT*)C.xr);
    else
      hipLaunchKernelGGL((k_phase1<LT, VT, NR, WPB>), dim3((C.p1_tasks + WPB - 1) / WPB), dim3(64 * WPB), 0, s,
                         slots, sof, C.p1_tasks, slot_active, nrr, (const VT*)X, ldx);
  }
  if (C.p1_reds > 0) {
    constexpr int WPR = p1red_waves<VT, NR>();
    const unsigned nb = WPR > 1 ? (unsigned)C.p1_reds : (unsigned)((C.p1_reds + 3) / 4);
    hipLaunchKernelGGL((k_p1reduce<VT, NR, mfma>), dim3(nb), dim3(256), 0, s, slots, sof + C.p1_tasks, C.p1_reds,
                       slot_active, nrr);
  }
  if (ev) HM_HIP(hipEventRecord(ev[1], s));
  EpiDev<VT> e;
  e.rowscale = (const VT*)ep.rowscale;
  e.a_acc = (VT)ep.a_acc;
  e.a_x = (VT)ep.a_x;
  e.a_z = (VT)ep.a_z;
  e.z = (const VT*)ep.z;
  e.ldz = ep.ldz;
  e.acc_out = (VT*)ep.acc_out;
  e.ld_acc = ep.ld_acc;
  if (C.p2_tiles > 0) {
    if constexpr (mfma)
      hipLaunchKernelGGL((k_phase2_mfma<DT, LT, VT, P2M_WAVES>), dim3(C.p2_tiles), dim3(64 * P2M_WAVES), 0, s, slots,
                         sof + C.p1_tasks + C.p1_reds, slot_active, nrr, (const VT*)X, ldx,
                         (const VT*)C.xr, (VT*)Y, ldy, e);
    else {
      // two or four waves per workgroup (tuned, else four on many tiles),
      // for one or two right-hand sides (wider products would spill the
      // further sets of sums)
      int wg = P2_WAVES;
      if constexpr (NR <= 2) wg = C.p2_waves ? C.p2_waves : (C.p2_tiles >= P2_MANY_TILES ? 4 : P2_WAVES);
      if constexpr (NR <= 2) {
        if (wg == 2)
          hipLaunchKernelGGL((k_phase2<DT, LT, VT, NR, 2>), dim3(C.p2_tiles), dim3(64 * 2), 0, s, slots,
                             sof + C.p1_tasks + C.p1_reds, slot_active, nrr, (const VT*)X, ldx, (VT*)Y, ldy, e);
        else if (wg == 4)
          hipLaunchKernelGGL((k_phase2<DT, LT, VT, NR, 4>), dim3(C.p2_tiles), dim3(64 * 4), 0, s, slots,
                             sof + C.p1_tasks + C.p1_reds, slot_active, nrr, (const VT*)X, ldx, (VT*)Y, ldy, e);
      }
      if (wg == P2_WAVES)
        hipLaunchKernelGGL((k_phase2<DT, LT, VT, NR, P2_WAVES>), dim3(C.p2_tiles), dim3(64 * P2_WAVES), 0, s,
                           slots, sof + C.p1_tasks + C.p1_reds, slot_active, nrr, (const VT*)X, ldx, (VT*)Y, ldy, e);
    }
  }
  if (ev) HM_HIP(hipEventRecord(ev[2], s));
  HM_HIP(hipGetLastError());
}

template <class DT, class LT, class VT>
void launch_nr(const CompView& C, int nrr, bool hi, const void* X, int64_t ldx, void* Y, int64_t ldy,
               const Epilogue& ep, const int* sa, hipStream_t s, hipEvent_t* ev) {
  switch (C.nr) {
    case 1: launch_typed<DT, LT, VT, 1>(C, nrr, hi, X, ldx, Y, ldy, ep, sa, s, ev); break;
    case 2: launch_typed<DT, LT, VT, 2>(C, nrr, hi, X, ldx, Y, ldy, ep, sa, s, ev); break;
    case 4: launch_typed<DT, LT, VT, 4>(C, nrr, hi, X, ldx, Y, ldy, ep, sa, s, ev); break;
    case 8: launch_typed<DT, LT, VT, 8>(C, nrr, hi, X, ldx, Y, ldy, ep, sa, s, ev); break;
    case 16: launch_typed<DT, LT, VT, 16>(C, nrr, hi, X, ldx, Y, ldy, ep, sa, s, ev); break;
    default: fail(HM_EINVAL, "matvec: composition width must be 1, 2, 4, 8 or 16");
  }
}

}  // namespace

void launch_matvec(const Composition& C, int nrr, int vb, bool hi, const void* X, int64_t ldx, void* Y, int64_t ldy,
                   const Epilogue& ep, const int* slot_active, hipStream_t s, hipEvent_t* ev) {
  HM_REQUIRE(!C.mats.empty(), "matvec: empty composition");
  const hm_matrix& M0 = *C.mats[0];
  for (const auto* M : C.mats)
    HM_REQUIRE(M->dense_dtype == M0.dense_dtype && M->lr_dtype == M0.lr_dtype && M->has_hi == M0.has_hi,
               "matvec: matrices of one batch must share storage types");
  CompView V;
  V.slots_lo = C.d_slots_lo.get<SlotDev>();
  V.slots_hi = C.d_slots_hi.get<SlotDev>();
  V.slot_of = C.d_slot_of.get<int32_t>();
  V.xr = C.xr.get();
  V.N = C.N;
  V.p1_tasks = C.p1_tasks;
  V.p1_reds = C.p1_reds;
  V.p2_tiles = C.p2_tiles;
  V.p2_waves = C.p2_waves;
  V.nr = C.nr;
  V.dense_dtype = M0.dense_dtype;
  V.lr_dtype = M0.lr_dtype;
  V.has_hi = M0.has_hi;
  launch_matvec_view(V, nrr, vb, hi, X, ldx, Y, ldy, ep, slot_active, s, ev);
}

void launch_matvec_view(const CompView& C, int nrr, int vb, bool hi, const void* X, int64_t ldx, void* Y,
                        int64_t ldy, const Epilogue& ep, const int* slot_active, hipStream_t s, hipEvent_t* ev) {
  HM_REQUIRE(nrr >= 1 && nrr <= C.nr, "matvec: more right-hand sides than the composition holds");
  const bool use_hi = hi && C.has_hi;
  const hm_dtype lt = use_hi ? HM_F32 : C.lr_dtype;
  const hm_dtype dt = use_hi && C.dense_dtype == HM_BF16 ? HM_F32 : C.dense_dtype;
  if (vb == 8) {
    if (dt == HM_F64 && lt == HM_F64) return launch_nr<double, double, double>(C, nrr, use_hi, X, ldx, Y, ldy, ep, slot_active, s, ev);
    if (dt == HM_F32 && lt == HM_F32) return launch_nr<float, float, double>(C, nrr, use_hi, X, ldx, Y, ldy, ep, slot_active, s, ev);
    if (dt == HM_F32 && lt == HM_BF16) return launch_nr<float, bf16_t, double>(C, nrr, use_hi, X, ldx, Y, ldy, ep, slot_active, s, ev);
    if (dt == HM_F64 && lt == HM_F32) return launch_nr<double, float, double>(C, nrr, use_hi, X, ldx, Y, ldy, ep, slot_active, s, ev);
    if (dt == HM_BF16 && lt == HM_BF16) return launch_nr<bf16_t, bf16_t, double>(C, nrr, use_hi, X, ldx, Y, ldy, ep, slot_active, s, ev);
  } else {
    if (dt == HM_F32 && lt == HM_F32) return launch_nr<float, float, float>(C, nrr, use_hi, X, ldx, Y, ldy, ep, slot_active, s, ev);
    if (dt == HM_F32 && lt == HM_BF16) return launch_nr<float, bf16_t, float>(C, nrr, use_hi, X, ldx, Y, ldy, ep, slot_active, s, ev);
    if (dt == HM_BF16 && lt == HM_BF16) return launch_nr<bf16_t, bf16_t, float>(C, nrr, use_hi, X, ldx, Y, ldy, ep, slot_active, s, ev);
    if (dt == HM_F64 && lt == HM_F64) return launch_nr<double, double, float>(C, nrr, use_hi, X, ldx, Y, ldy, ep, slot_active, s, ev);
  }
  fail(HM_EINVAL, "matvec: unsupported combination of storage and vector types");
}

}  // namespace hm
