// Block-wise H-matrix product on gfx950 (Sec. 5.2): y = F_H x with
//   phase 1:  t_b = V_b^T x_tau          for every low-rank block b
//   phase 2:  y_sigma += D_b x_tau  and  y_sigma += U_b t_b, row tile by row tile.
// Both phases are bandwidth kernels: every stored entry is read once per
// product.  Work is cut into items of similar byte size; an item whose
// output is shared with other items writes a partial sum, and the last item
// to finish (device-scope atomic counter) adds the partials in a fixed
// order, so results do not depend on scheduling.  Several matrices can be
// multiplied in one launch ("slots" of a block-diagonal operator).
#include <algorithm>
#include <cmath>
#include <numeric>

#include "dev_common.hpp"
#include "hm_internal.hpp"

namespace hm {

// ------------------------------------------------------------------ plan
namespace {

constexpr int64_t ITEM_BYTES = 64 << 10;  // target matrix bytes per phase-2 item
constexpr int64_t TASK_BYTES = 24 << 10;  // minimum matrix bytes per wave task

struct Tile {
  int32_t row0, m;
};

}  // namespace

void build_plan(hm_matrix& M, const std::vector<LrInfo>& lr, const std::vector<DnInfo>& dn, const hm_tree& t,
                hipStream_t s) {
  Plan& P = M.plan;
  P.p1.clear();
  P.p2.clear();
  P.segs.clear();
  P.p1_task.clear();
  P.p2_task.clear();
  // tiles: leaves cut into <= TILE rows
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
  // t offsets of the low-rank blocks
  std::vector<int32_t> toff(lr.size());
  int64_t kt = 0;
  for (size_t q = 0; q < lr.size(); ++q) {
    toff[q] = (int32_t)kt;
    kt += lr[q].k;
  }
  HM_REQUIRE(kt < (int64_t)1 << 30, "build_plan: too many rank columns");
  // ---- phase 2 segments per tile
  std::vector<std::vector<Seg>> tseg(tiles.size());
  auto add = [&](const BlockRef& b, int64_t off, int32_t w, int32_t src, int32_t kind) {
    size_t q = std::lower_bound(row0s.begin(), row0s.end(), b.rb) - row0s.begin();
    for (; q < tiles.size() && tiles[q].row0 < b.re; ++q) {
      Seg sg;
      sg.off = off + (tiles[q].row0 - b.rb);
      sg.ld = b.re - b.rb;
      sg.w = w;
      sg.src = src;
      sg.kind = kind;
      tseg[q].push_back(sg);
    }
  };
  for (const auto& d : dn) add(d.b, d.off, d.b.ce - d.b.cb, d.b.cb, 0);
  for (size_t q = 0; q < lr.size(); ++q) add(lr[q].b, lr[q].u_off, lr[q].k, ~toff[q], 1);
  int32_t parts2 = 0, counters2 = 0;
  std::vector<int64_t> item_bytes2;
  for (size_t q = 0; q < tiles.size(); ++q) {
    auto& v = tseg[q];
    std::stable_sort(v.begin(), v.end(), [](const Seg& a, const Seg& b) {
      if (a.kind != b.kind) return a.kind < b.kind;
      return a.src < b.src;
    });
    const int64_t rowbytes = (int64_t)tiles[q].m * 4;
    std::vector<std::pair<int32_t, int32_t>> runs;  // [seg begin, seg end) per item
    int32_t b0 = (int32_t)P.segs.size();
    int64_t acc = 0;
    int32_t cur = b0;
    for (size_t k = 0; k < v.size(); ++k) {
      const int64_t sb = rowbytes * v[k].w;
      if (acc > 0 && acc + sb > ITEM_BYTES) {
        runs.emplace_back(cur, (int32_t)(b0 + k));
        cur = (int32_t)(b0 + k);
        acc = 0;
      }
      acc += sb;
    }
    runs.emplace_back(cur, (int32_t)(b0 + v.size()));
    for (const auto& sg : v) P.segs.push_back(sg);
    const int32_t np = (int32_t)runs.size();
    const int32_t part = np > 1 ? parts2 : -1;
    if (np > 1) {
      parts2 += np;
      ++counters2;
    }
    for (int32_t k = 0; k < np; ++k) {
      P2Item it{tiles[q].row0, tiles[q].m, runs[k].first, runs[k].second - runs[k].first, part, k, np,
                np > 1 ? counters2 - 1 : 0};
      P.p2.push_back(it);
      int64_t by = 0;
      for (int32_t z = runs[k].first; z < runs[k].second; ++z) by += rowbytes * P.segs[z].w;
      item_bytes2.push_back(by);
    }
  }
  // ---- phase 1 items
  int32_t parts1 = 0, counters1 = 0;
  std::vector<int64_t> item_bytes1;
  for (size_t q = 0; q < lr.size(); ++q) {
    const int32_t nb = lr[q].b.ce - lr[q].b.cb;
    const int32_t k = lr[q].k;
    const int32_t nch = (nb + P1_RCH - 1) / P1_RCH;
    for (int32_t l0 = 0; l0 < k; l0 += KG) {
      const int32_t nl = std::min(KG, k - l0);
      const int32_t part = nch > 1 ? parts1 : -1;
      if (nch > 1) {
        parts1 += nch;
        ++counters1;
      }
      for (int32_t c = 0; c < nch; ++c) {
        const int32_t r0 = (int32_t)((int64_t)nb * c / nch);
        const int32_t r1 = (int32_t)((int64_t)nb * (c + 1) / nch);
        P1Item it{};
        it.v_off = lr[q].v_off;
        it.ld = nb;
        it.r0 = r0;
        it.nr = r1 - r0;
        it.l0 = l0;
        it.nl = nl;
        it.xrow = lr[q].b.cb + r0;
        it.trow = toff[q] + l0;
        it.part = part;
        it.pidx = c;
        it.nparts = nch;
        it.counter = nch > 1 ? counters1 - 1 : 0;
        P.p1.push_back(it);
        item_bytes1.push_back((int64_t)(r1 - r0) * nl * 4);
      }
    }
  }
  // ---- tasks: consecutive items of at least TASK_BYTES
  auto pack = [](const std::vector<int64_t>& by, std::vector<int32_t>& task) {
    task.clear();
    task.push_back(0);
    int64_t acc = 0;
    for (size_t k = 0; k < by.size(); ++k) {
      acc += by[k];
      if (acc >= TASK_BYTES) {
        task.push_back((int32_t)(k + 1));
        acc = 0;
      }
    }
    if (task.back() != (int32_t)by.size()) task.push_back((int32_t)by.size());
  };
  pack(item_bytes1, P.p1_task);
  pack(item_bytes2, P.p2_task);
  P.n_p1_parts = parts1;
  P.n_p2_parts = parts2;
  P.n_p1_counters = counters1;
  P.n_p2_counters = counters2;
  upload(P.d_p1, P.p1, s);
  upload(P.d_p1_task, P.p1_task, s);
  upload(P.d_p2, P.p2, s);
  upload(P.d_p2_task, P.p2_task, s);
  upload(P.d_segs, P.segs, s);
  HM_HIP(hipStreamSynchronize(s));
}

int64_t matrix_bytes(const hm_matrix& M, bool hi) {
  const size_t dsz = dtype_size(M.dense_dtype);
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
  int64_t tsz = 0, p1 = 0, p2 = 0, c1 = 0, c2 = 0;
  for (const auto* M : mats) {
    C->xoff.push_back(C->N);
    C->N += M->n;
    tsz += M->Ktot;
    p1 += M->plan.n_p1_parts;
    p2 += M->plan.n_p2_parts;
    c1 += M->plan.n_p1_counters;
    c2 += M->plan.n_p2_counters;
  }
  const int64_t eb = 8;  // buffers sized for FP64 so one composition serves both vector types
  C->t.alloc(std::max<int64_t>(1, tsz * nr) * eb);
  C->part1.alloc(std::max<int64_t>(1, p1 * KG * nr) * eb);
  C->part2.alloc(std::max<int64_t>(1, p2 * TILE * nr) * eb);
  C->cnt1.alloc(std::max<int64_t>(1, c1) * 4);
  C->cnt2.alloc(std::max<int64_t>(1, c2) * 4);
  HM_HIP(hipMemsetAsync(C->cnt1.get(), 0, C->cnt1.bytes(), s));
  HM_HIP(hipMemsetAsync(C->cnt2.get(), 0, C->cnt2.bytes(), s));
  int64_t to = 0;
  p1 = p2 = c1 = c2 = 0;
  int32_t t1 = 0, t2 = 0;
  for (size_t q = 0; q < mats.size(); ++q) {
    const hm_matrix& M = *mats[q];
    SlotDev d{};
    d.p1 = M.plan.d_p1.get<P1Item>();
    d.p1_task = M.plan.d_p1_task.get<int32_t>();
    d.p2 = M.plan.d_p2.get<P2Item>();
    d.p2_task = M.plan.d_p2_task.get<int32_t>();
    d.segs = M.plan.d_segs.get<Seg>();
    d.dense = M.dense.get();
    d.U = M.U.get();
    d.V = M.V.get();
    d.cnt1 = C->cnt1.get<unsigned>() + c1;
    d.cnt2 = C->cnt2.get<unsigned>() + c2;
    d.part1 = C->part1.get<char>() + p1 * KG * nr * eb;
    d.part2 = C->part2.get<char>() + p2 * TILE * nr * eb;
    d.t = C->t.get<char>() + to * nr * eb;
    d.ldt = std::max<int64_t>(1, M.Ktot);
    d.xoff = C->xoff[q];
    d.p1_task_begin = t1;
    d.p2_task_begin = t2;
    d.n = (int32_t)M.n;
    d.slot = (int32_t)q;
    t1 += (int32_t)M.plan.p1_task.size() - 1;
    t2 += (int32_t)M.plan.p2_task.size() - 1;
    to += M.Ktot;
    p1 += M.plan.n_p1_parts;
    p2 += M.plan.n_p2_parts;
    c1 += M.plan.n_p1_counters;
    c2 += M.plan.n_p2_counters;
    C->slots_lo.push_back(d);
    SlotDev h = d;
    if (M.has_hi) {
      h.U = M.U_hi.get();
      h.V = M.V_hi.get();
    }
    C->slots_hi.push_back(h);
    C->bytes_lo += matrix_bytes(M, false);
    C->bytes_hi += matrix_bytes(M, true);
  }
  C->p1_tasks = t1;
  C->p2_tasks = t2;
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
};

__device__ inline int find_slot(const SlotDev* __restrict__ slots, int nslots, int task, bool phase1) {
  int lo = 0, hi = nslots - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int b = phase1 ? slots[mid].p1_task_begin : slots[mid].p2_task_begin;
    if (b <= task) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// acc[j] += sum_c A(lane, c) * src[c + j*lds], lane = row of the tile
template <class MT, class VT, int NR>
__device__ __forceinline__ void seg_accumulate(const MT* __restrict__ a, int ld, int w, const VT* __restrict__ src,
                                               int64_t lds, bool act, int nrr, VT* acc) {
  int c = 0;
  for (; c + 8 <= w; c += 8) {
    VT v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = act ? ld_as<VT>(a + (int64_t)(c + q) * ld) : VT(0);
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int j = 0; j < NR; ++j)
        if (j < nrr) acc[j] += v[q] * src[c + q + j * lds];
  }
  for (; c < w; ++c) {
    const VT v = act ? ld_as<VT>(a + (int64_t)c * ld) : VT(0);
#pragma unroll
    for (int j = 0; j < NR; ++j)
      if (j < nrr) acc[j] += v * src[c + j * lds];
  }
}

template <class VT, int NR>
__device__ __forceinline__ void epilogue_store(int row, int lane, int m, int nrr, const VT* acc,
                                               const VT* __restrict__ X, int64_t ldx, VT* __restrict__ Y,
                                               int64_t ldy, const EpiDev<VT>& ep) {
  if (lane >= m) return;
  const VT w = ep.rowscale ? ep.rowscale[row] : VT(1);
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    if (j >= nrr) break;
    VT o = ep.a_acc * w * acc[j];
    if (ep.a_x != VT(0)) o += ep.a_x * X[row + j * ldx];
    if (ep.a_z != VT(0)) o += ep.a_z * ep.z[row + j * ep.ldz];
    Y[row + j * ldy] = o;
  }
}

template <class DT, class LT, class VT, int NR>
__global__ __launch_bounds__(256) void k_phase2(const SlotDev* __restrict__ slots, int nslots, int ntasks,
                                                const int* __restrict__ slot_active, int nrr, const VT* __restrict__ X,
                                                int64_t ldx, VT* __restrict__ Y, int64_t ldy, EpiDev<VT> ep) {
  const int lane = threadIdx.x & 63;
  const int task = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (task >= ntasks) return;
  const int si = find_slot(slots, nslots, task, false);
  const SlotDev& S = slots[si];
  if (slot_active && !slot_active[S.slot]) return;
  const int lt = task - S.p2_task_begin;
  const int ib = S.p2_task[lt], ie = S.p2_task[lt + 1];
  const VT* Xs = X + S.xoff;
  VT* Ys = Y + S.xoff;
  const VT* Ts = (const VT*)S.t;
  EpiDev<VT> e = ep;
  if (e.rowscale) e.rowscale += S.xoff;
  if (e.z) e.z += S.xoff;
  for (int it = ib; it < ie; ++it) {
    const P2Item item = S.p2[it];
    const bool act = lane < item.m;
    VT acc[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) acc[j] = VT(0);
    for (int sg = item.seg0; sg < item.seg0 + item.nseg; ++sg) {
      const Seg seg = S.segs[sg];
      const VT* src;
      int64_t lds;
      if (seg.src >= 0) {
        src = Xs + seg.src;
        lds = ldx;
      } else {
        src = Ts + (~seg.src);
        lds = S.ldt;
      }
      if (seg.kind == 0)
        seg_accumulate<DT, VT, NR>((const DT*)S.dense + seg.off + lane, seg.ld, seg.w, src, lds, act, nrr, acc);
      else
        seg_accumulate<LT, VT, NR>((const LT*)S.U + seg.off + lane, seg.ld, seg.w, src, lds, act, nrr, acc);
    }
    const int row = item.row0 + lane;
    if (item.nparts == 1) {
      epilogue_store<VT, NR>(row, lane, item.m, nrr, acc, Xs, ldx, Ys, ldy, e);
    } else {
      VT* P0 = (VT*)S.part2 + (int64_t)item.part * TILE * NR;
      VT* P = P0 + (int64_t)item.pidx * TILE * NR;
#pragma unroll
      for (int j = 0; j < NR; ++j) P[j * TILE + lane] = acc[j];
      __threadfence();
      unsigned old = 0;
      if (lane == 0) old = atomicAdd(&S.cnt2[item.counter], 1u);
      old = __shfl(old, 0, 64);
      if (old == (unsigned)(item.nparts - 1)) {
        __threadfence();
        VT sum[NR];
#pragma unroll
        for (int j = 0; j < NR; ++j) sum[j] = VT(0);
        for (int p = 0; p < item.nparts; ++p)
#pragma unroll
          for (int j = 0; j < NR; ++j) sum[j] += P0[(int64_t)p * TILE * NR + j * TILE + lane];
        epilogue_store<VT, NR>(row, lane, item.m, nrr, sum, Xs, ldx, Ys, ldy, e);
        if (lane == 0) S.cnt2[item.counter] = 0u;
      }
    }
  }
}

// Phase 1: t[trow + l] (+ j*ldt) = sum_r V(r0 + r, l0 + l) x(xrow + r), lane = row of V.
template <class LT, class VT, int NR>
__global__ __launch_bounds__(256) void k_phase1(const SlotDev* __restrict__ slots, int nslots, int ntasks,
                                                const int* __restrict__ slot_active, int nrr,
                                                const VT* __restrict__ X, int64_t ldx) {
  constexpr int SG = NR <= 2 ? KG : (NR <= 4 ? 4 : (NR <= 8 ? 2 : 1));  // rank columns per pass
  const int lane = threadIdx.x & 63;
  const int task = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (task >= ntasks) return;
  const int si = find_slot(slots, nslots, task, true);
  const SlotDev& S = slots[si];
  if (slot_active && !slot_active[S.slot]) return;
  const int lt = task - S.p1_task_begin;
  const int ib = S.p1_task[lt], ie = S.p1_task[lt + 1];
  const VT* Xs = X + S.xoff;
  VT* T = (VT*)S.t;
  for (int it = ib; it < ie; ++it) {
    const P1Item item = S.p1[it];
    const LT* Vb = (const LT*)S.V + item.v_off + item.r0;
    // destination of the (rank column l, right-hand side j) sums
    VT* P0 = (VT*)S.part1 + (int64_t)(item.part < 0 ? 0 : item.part) * KG * NR;
    VT* dst;
    int64_t sl, sj;
    if (item.nparts == 1) {
      dst = T + item.trow;
      sl = 1;
      sj = S.ldt;
    } else {
      dst = P0 + (int64_t)item.pidx * KG * NR;
      sl = NR;
      sj = 1;
    }
    for (int g0 = 0; g0 < item.nl; g0 += SG) {
      VT acc[SG][NR];
#pragma unroll
      for (int q = 0; q < SG; ++q)
#pragma unroll
        for (int j = 0; j < NR; ++j) acc[q][j] = VT(0);
      for (int r = lane; r < item.nr; r += 64) {
        VT xv[NR];
#pragma unroll
        for (int j = 0; j < NR; ++j) xv[j] = j < nrr ? Xs[item.xrow + r + j * ldx] : VT(0);
#pragma unroll
        for (int q = 0; q < SG; ++q) {
          if (g0 + q < item.nl) {
            const VT a = ld_as<VT>(Vb + (int64_t)(item.l0 + g0 + q) * item.ld + r);
#pragma unroll
            for (int j = 0; j < NR; ++j) acc[q][j] += a * xv[j];
          }
        }
      }
#pragma unroll
      for (int q = 0; q < SG; ++q)
#pragma unroll
        for (int j = 0; j < NR; ++j) {
          const VT v = wave_sum(acc[q][j]);
          if (lane == 0 && g0 + q < item.nl && j < nrr) dst[(g0 + q) * sl + j * sj] = v;
        }
    }
    if (item.nparts > 1) {
      __threadfence();
      unsigned old = 0;
      if (lane == 0) old = atomicAdd(&S.cnt1[item.counter], 1u);
      old = __shfl(old, 0, 64);
      if (old == (unsigned)(item.nparts - 1)) {
        __threadfence();
        const int tot = item.nl * NR;
        for (int q = lane; q < tot; q += 64) {
          VT sum = VT(0);
          for (int p = 0; p < item.nparts; ++p) sum += P0[(int64_t)p * KG * NR + q];
          const int l = q / NR, j = q % NR;
          if (j < nrr) T[item.trow + l + j * S.ldt] = sum;
        }
        if (lane == 0) S.cnt1[item.counter] = 0u;
      }
    }
  }
}

// ------------------------------------------------------------------ launch
namespace {

template <class DT, class LT, class VT, int NR>
void launch_typed(const Composition& C, int nrr, bool hi, const void* X, int64_t ldx, void* Y, int64_t ldy,
                  const Epilogue& ep, const int* slot_active, hipStream_t s, hipEvent_t* ev) {
  if (ev) HM_HIP(hipEventRecord(ev[0], s));
  const SlotDev* slots = (hi ? C.d_slots_hi : C.d_slots_lo).get<SlotDev>();
  const int ns = (int)C.mats.size();
  if (C.p1_tasks > 0) {
    hipLaunchKernelGGL((k_phase1<LT, VT, NR>), dim3((C.p1_tasks + 3) / 4), dim3(256), 0, s, slots, ns, C.p1_tasks,
                       slot_active, nrr, (const VT*)X, ldx);
  }
  if (ev) HM_HIP(hipEventRecord(ev[1], s));
  EpiDev<VT> e;
  e.rowscale = (const VT*)ep.rowscale;
  e.a_acc = (VT)ep.a_acc;
  e.a_x = (VT)ep.a_x;
  e.a_z = (VT)ep.a_z;
  e.z = (const VT*)ep.z;
  e.ldz = ep.ldz;
  if (C.p2_tasks > 0) {
    hipLaunchKernelGGL((k_phase2<DT, LT, VT, NR>), dim3((C.p2_tasks + 3) / 4), dim3(256), 0, s, slots, ns,
                       C.p2_tasks, slot_active, nrr, (const VT*)X, ldx, (VT*)Y, ldy, e);
  }
  if (ev) HM_HIP(hipEventRecord(ev[2], s));
  HM_HIP(hipGetLastError());
}

template <class DT, class LT, class VT>
void launch_nr(const Composition& C, int nrr, bool hi, const void* X, int64_t ldx, void* Y, int64_t ldy,
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
  HM_REQUIRE(nrr >= 1 && nrr <= C.nr, "matvec: more right-hand sides than the composition holds");
  const hm_matrix& M0 = *C.mats[0];
  for (const auto* M : C.mats)
    HM_REQUIRE(M->dense_dtype == M0.dense_dtype && M->lr_dtype == M0.lr_dtype && M->has_hi == M0.has_hi,
               "matvec: matrices of one batch must share storage types");
  const bool use_hi = hi && M0.has_hi;
  const hm_dtype lt = use_hi ? HM_F32 : M0.lr_dtype;
  const hm_dtype dt = M0.dense_dtype;
  if (vb == 8) {
    if (dt == HM_F64 && lt == HM_F64) return launch_nr<double, double, double>(C, nrr, use_hi, X, ldx, Y, ldy, ep, slot_active, s, ev);
    if (dt == HM_F32 && lt == HM_F32) return launch_nr<float, float, double>(C, nrr, use_hi, X, ldx, Y, ldy, ep, slot_active, s, ev);
    if (dt == HM_F32 && lt == HM_BF16) return launch_nr<float, bf16_t, double>(C, nrr, use_hi, X, ldx, Y, ldy, ep, slot_active, s, ev);
    if (dt == HM_F64 && lt == HM_F32) return launch_nr<double, float, double>(C, nrr, use_hi, X, ldx, Y, ldy, ep, slot_active, s, ev);
  } else {
    if (dt == HM_F32 && lt == HM_F32) return launch_nr<float, float, float>(C, nrr, use_hi, X, ldx, Y, ldy, ep, slot_active, s, ev);
    if (dt == HM_F32 && lt == HM_BF16) return launch_nr<float, bf16_t, float>(C, nrr, use_hi, X, ldx, Y, ldy, ep, slot_active, s, ev);
    if (dt == HM_F64 && lt == HM_F64) return launch_nr<double, double, float>(C, nrr, use_hi, X, ldx, Y, ldy, ep, slot_active, s, ev);
  }
  fail(HM_EINVAL, "matvec: unsupported combination of storage and vector types");
}

}  // namespace hm
