// Internal declarations of the hierarchical view-factor radiosity library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/hm.h"

namespace hm {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
  hm_status code;
  Error(hm_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(hm_status c, const std::string& m) { throw Error(c, m); }

#define HM_HIP(call)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      ::hm::fail(e_ == hipErrorOutOfMemory ? HM_ENOMEM : HM_EDEVICE,                        \
                 std::string(#call) + ": " + hipGetErrorString(e_));                        \
  } while (0)

#define HM_REQUIRE(cond, msg)                   \
  do {                                          \
    if (!(cond)) ::hm::fail(HM_EINVAL, (msg));  \
  } while (0)

// ---------------------------------------------------------------- device memory
// Caching device allocator: freed blocks are kept per (device, size class)
// and handed out again, so per-call workspaces do not pay hipMalloc/hipFree.
// Reuse is stream-ordered: a block freed while this thread's current stream
// is s is handed to an allocation on another stream only after that stream
// has been made to wait for the work queued on s before the free.
void* pool_alloc(size_t bytes, size_t* granted);
hipStream_t current_stream();
void set_current_stream(hipStream_t s);
// Sets the calling thread's current stream for its lifetime (restores the
// previous one at the end).
struct StreamScope {
  hipStream_t prev;
  explicit StreamScope(hipStream_t s) : prev(current_stream()) { set_current_stream(s); }
  ~StreamScope() { set_current_stream(prev); }
  StreamScope(const StreamScope&) = delete;
  StreamScope& operator=(const StreamScope&) = delete;
};
void pool_free(void* p, size_t granted);
int64_t pool_cached_bytes();
void pool_trim();

// Owning device allocation from the pool, move-only.
class DevBuf {
 public:
  DevBuf() = default;
  explicit DevBuf(size_t bytes) { alloc(bytes); }
  ~DevBuf() { release(); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p_(o.p_), n_(o.n_), g_(o.g_) { o.p_ = nullptr; o.n_ = o.g_ = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p_ = o.p_; n_ = o.n_; g_ = o.g_; o.p_ = nullptr; o.n_ = o.g_ = 0; }
    return *this;
  }
  void alloc(size_t bytes) {
    release();
    if (bytes == 0) return;
    p_ = pool_alloc(bytes, &g_);
    n_ = bytes;
  }
  void release() {
    if (p_) pool_free(p_, g_);
    p_ = nullptr;
    n_ = g_ = 0;
  }
  template <class T = void> T* get() const { return static_cast<T*>(p_); }
  size_t bytes() const { return n_; }
 private:
  void* p_ = nullptr;
  size_t n_ = 0, g_ = 0;
};

template <class T>
inline void upload(DevBuf& b, const std::vector<T>& v, hipStream_t s) {
  b.alloc(v.size() * sizeof(T) + (v.empty() ? 0 : 0));
  if (!v.empty()) HM_HIP(hipMemcpyAsync(b.get(), v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

inline size_t dtype_size(hm_dtype t) { return t == HM_F64 ? 8 : (t == HM_F32 ? 4 : 2); }

// ---------------------------------------------------------------- context
}  // namespace hm

struct hm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string last_error;
};

namespace hm {

// ---------------------------------------------------------------- tree (host)
struct ClusterNode {
  int32_t begin, end;   // permuted positions [begin, end)
  double lo[3], hi[3];  // bounding box of the centroids
  int32_t child[2];     // -1 for a leaf
  int32_t level;
};

struct BlockRef {
  int32_t rb, re, cb, ce;  // rows [rb, re) x cols [cb, ce), permuted positions
};

}  // namespace hm

struct hm_tree {
  int64_t n = 0;
  hm_tree_params params{};
  std::vector<double> c, nrm, area;     // original order (copied)
  std::vector<int32_t> perm;            // perm[k] = original index at position k
  std::vector<hm::ClusterNode> nodes;   // nodes[0] = root
  std::vector<int32_t> leaves;          // node indices of the leaves, in order
  std::vector<hm::BlockRef> dense, lowrank;
};

namespace hm {

void build_tree(hm_tree& t);  // fills perm, nodes, leaves, dense, lowrank from c, params
// The admissibility condition of Algorithm 2 (eq. (28) on the bounding boxes).
bool tree_admissible(const ClusterNode& s, const ClusterNode& t, double eta);

// ---------------------------------------------------------------- matvec plan
// Both phases stream panels laid out so that every lane loads 16 contiguous
// bytes (4 elements) and a wave's load covers one contiguous run:
//  * phase 2 item panel (m rows <= 64, w columns, w % 4 == 0): element
//    (r, c) at base + ((c / 4) * m + r) * 4 + c % 4  (lane = row);
//  * phase 1 group panel (gw <= 64 rank columns of the V factors of one
//    column cluster, rows padded to a multiple of 4): element (r, l) at
//    base + ((r / 4) * gw + l) * 4 + r % 4  (lane = rank column).
constexpr int QW = 4;          // elements per lane vector
constexpr int P2_MAXW = 256;   // padded columns per phase-2 item
constexpr int P1_GW = 64;      // rank columns per phase-1 group (one per lane)
constexpr int P1_XST = 256;    // rows of x staged in LDS at a time
constexpr int TILE = 64;       // rows per phase-2 tile (lane = row)
constexpr int P2_WAVES = 8;    // items per phase-2 tile; waves per phase-2 workgroup
constexpr int P2_MANY_TILES = 4096;  // from this many tiles, four waves per workgroup
constexpr int P2_MAXSEG = 64;  // input runs per phase-2 item

// Phase 1 item: t (or a partial of it) for the gw columns of one group over
// row quads [q0, q0 + nq) of its column cluster.
struct P1Item {
  int64_t base;     // element offset of the group panel
  int32_t gw;       // columns in the group
  int32_t q0, nq;   // row quads
  int32_t nrows;    // valid rows of the cluster (the rest is zero padding)
  int32_t xrow;     // permuted x row of the cluster's first row
  int32_t trow;     // t index of the group's first column
  int32_t part;     // partial slot of this item; -1: write t directly
  int32_t gs;       // stored columns of the group panel: gw rounded up to even
};

// Groups whose rows are split over several items: t = sum of their partials
// (added in item order by a separate kernel).
struct P1Red {
  int32_t trow, gw, part0, nparts;
};

// Phase 2 tile: rows [row0, row0+m) and its items [it0, it0+nit); wave w of
// the tile's workgroup takes items it0 + w, it0 + w + P2_WAVES, ...
struct P2Tile {
  int32_t row0, m, it0, nit;
};

// Phase 2 item: a panel of w columns (m rows of its tile).
struct P2Item {
  int64_t base;     // element offset of the panel in its arena
  int32_t w;        // padded column count (multiple of 4)
  int32_t seg0, nseg;
  int32_t kind;     // 0: dense arena, 1: U arena
};

// Input run of a phase-2 item: columns [col0, col0+w) take x (src >= 0) or
// t (index ~src) entries src.., src+w-1.
struct Seg {
  int32_t col0, w, src, pad;
};

// One column cluster tau of the low-rank blocks: its V factors form
// ceil(ktau / P1_GW) group panels of np rows (n rounded up to 4); a panel
// of odd width carries one zero column, so every panel row of two adjacent
// columns starts on a 16-byte boundary.
struct P1Tau {
  int64_t vbase;    // element offset of the first group panel
  int64_t trow;     // t index of rank column 0
  int32_t xrow, n, np, ktau;
};

// Phase-1 work split (tunable; the panel layout does not depend on it).
struct P1Params {
  int32_t rows = 128;          // rows per item (multiple of 64)
  int32_t task_bytes = 16384;  // minimum matrix bytes per wave task
};

struct Plan {
  std::vector<P1Tau> taus;
  P1Params p1p;
  double p1_us = 0.0;  // measured time of the chosen split (0: not timed)
  // waves per phase-2 workgroup for one or two right-hand sides: 2, 4 or 8
  // (the same bits in every case), 0 = by tile count (4 from P2_MANY_TILES)
  int32_t p2_waves = 0;
  double p2_us = 0.0;  // measured phase-2 time of that choice (0: not timed)
  std::vector<P1Item> p1;
  std::vector<int32_t> p1_task;  // item begin per task, size ntasks + 1
  std::vector<P1Red> p1red;
  std::vector<P2Tile> p2t;
  std::vector<P2Item> p2;
  std::vector<Seg> segs;
  int32_t n_p1_parts = 0;
  int64_t dense_elems = 0, u_elems = 0, v_elems = 0;  // panel arena sizes
  DevBuf d_p1, d_p1_task, d_p1red, d_p2t, d_p2, d_segs;
};

// Device descriptor of one slot of a batched product.
struct SlotDev {
  const P1Item* p1;
  const int32_t* p1_task;
  const P1Red* p1red;
  const P2Tile* p2t;
  const P2Item* p2;
  const Seg* segs;
  const void* dense;
  const void* U;
  const void* V;
  void* part1;
  void* t;
  int64_t ldt;
  int64_t xoff;
  int32_t p1_task_begin, p1red_begin, p2_tile_begin;
  int32_t n, slot, pad;
};

// Packing work lists produced with the plan (consumed once by assembly).
struct NfDev {     // dense segment: F(row0 + r, cb + c) -> item panel
  int64_t base;
  int32_t row0, m, cb, w, col0, pad;
};
struct URepack {   // U_b rows of a tile -> item panel
  int64_t src;     // stage element offset of U_b(row0 - rb, l0)
  int64_t base;
  int32_t stage, ld, m, k, col0;
  int32_t row0, cb, l0;  // first (permuted) row and rank index taken, first column of the block
};
struct VRepack {   // V_b -> group panels of its column cluster
  int64_t src;     // stage element offset of V_b
  int64_t tau_base;
  int32_t stage, n, k, lc0, ktau, np;
  int32_t cb, rb;  // first (permuted) column and row of the block
};
struct PackLists {
  std::vector<NfDev> nf;
  std::vector<URepack> ur;
  std::vector<VRepack> vr;
};

}  // namespace hm

struct hm_matrix {
  uint64_t id = 0;  // unique per process, keys cached batches
  int device = 0;
  int64_t n = 0;
  hm_dtype dense_dtype = HM_F32, lr_dtype = HM_F32;
  bool has_hi = false;  // FP32 copies of BF16 factors (and of a BF16 near field)
  std::vector<int32_t> perm;
  hm::DevBuf d_perm;                         // int32 perm
  hm::DevBuf dense, U, V, U_hi, V_hi;        // arenas
  hm::DevBuf dense_hi;                       // FP32 copy of a BF16 near field
  int64_t dense_entries = 0, lr_entries = 0, Ktot = 0;
  int64_t u_entries = 0, v_entries = 0;  // sum k*m and sum k*n over low-rank blocks
  int64_t n_dense_blocks = 0, n_lr_blocks = 0, n_fallback = 0, rank_sum = 0;
  int32_t max_rank = 0;
  hm::Plan plan;
  // cached per-(ctx) compositions and the flux helper g, keyed by eps
  std::mutex mu;
  std::shared_ptr<void> cache;
  int64_t bytes_device() const;
};

namespace hm {

// ---------------------------------------------------------------- batched product
// A set of matrices laid out one after another in a combined row space.
struct Composition {
  int nr = 1;                 // right-hand sides per row
  int vec_bytes = 8;          // 8: FP64 vectors, 4: FP32
  std::vector<const hm_matrix*> mats;
  std::vector<int64_t> xoff;  // row offset per slot
  int64_t N = 0;              // total rows
  int32_t p1_tasks = 0, p1_reds = 0, p2_tiles = 0;
  int32_t p2_waves = 0;       // the members' common tuned choice, else 0
  std::vector<SlotDev> slots_lo, slots_hi;  // hi: FP32 copies of BF16 factors
  DevBuf d_slots_lo, d_slots_hi;
  // slot of every phase-1 task, then of every reduction, then of every tile
  std::vector<int32_t> slot_of;
  DevBuf d_slot_of;
  DevBuf t, part1;
  // 16-column products on the matrix cores: the input rows copied to
  // row-major order (16 values a row, FP32 or FP64); t is then row-major too
  DevBuf xr;
  int64_t bytes_lo = 0, bytes_hi = 0;     // algorithmic matrix bytes per product
};

void build_plan(hm_matrix& M, const std::vector<struct LrInfo>& lr, const std::vector<BlockRef>& dn,
                const hm_tree& t, PackLists& pk, hipStream_t s);
// Phase-1 items, partial reductions and tasks of a plan for the given split.
void plan_phase1(Plan& P, const P1Params& pp);
// Re-split phase 1 and upload its lists (the matrix must not be in use).
void replan_phase1(hm_matrix& M, const P1Params& pp, hipStream_t s);
// Times the candidate phase-1 splits on M (FP32 vectors unless the factors
// are FP64; products of `width` columns, 1..16) and keeps the fastest; for
// one or two columns then times phase 2 with 2, 4 and 8 waves per
// workgroup and keeps the fastest.  Call before any composition of M exists.
void autotune_phase1(hm_matrix& M, hipStream_t s, int width = 1);
// The same for several matrices multiplied together: one split for all,
// timed on their batched product.
void autotune_phase1_joint(const std::vector<hm_matrix*>& mats, hipStream_t s, int width = 1);
// The host part of build_plan (no device calls): items, tasks, arena sizes.
void plan_host(hm_matrix& M, const std::vector<struct LrInfo>& lr, const std::vector<BlockRef>& dn,
               const hm_tree& t, PackLists& pk);

std::unique_ptr<Composition> make_composition(const std::vector<const hm_matrix*>& mats, int nr,
                                              int vec_bytes, hipStream_t s);

// y = epilogue(F x) on every active slot of a composition.
// Epilogue per row i, column j:  y = a_acc * w_i * (F x)_i + a_x * x_i + a_z * z_i
// (w = rowscale, 1 when NULL; z may be NULL when a_z == 0).
struct Epilogue {
  const void* rowscale = nullptr;
  double a_acc = 1.0, a_x = 0.0, a_z = 0.0;
  const void* z = nullptr;
  int64_t ldz = 0;
  void* acc_out = nullptr;  // optional: the plain product F x as well (leading dim ld_acc)
  int64_t ld_acc = 0;
};

// nrr: right-hand sides actually present (<= C.nr, the padded width).
// vb: vector element bytes (8: FP64, 4: FP32).
void launch_matvec(const Composition& C, int nrr, int vb, bool hi, const void* X, int64_t ldx, void* Y, int64_t ldy,
                   const Epilogue& ep, const int* slot_active, hipStream_t s, hipEvent_t* ev = nullptr);

// What the product kernels read of a composition: its device tables, the
// work counts and the storage types.  A Composition gives one over its own
// buffers; the allocation-free product builds one over a static buffer.
struct CompView {
  const SlotDev* slots_lo = nullptr;
  const SlotDev* slots_hi = nullptr;
  const int32_t* slot_of = nullptr;
  void* xr = nullptr;  // row-major input rows (16-column products only)
  int64_t N = 0;
  int32_t p1_tasks = 0, p1_reds = 0, p2_tiles = 0;
  int32_t p2_waves = 0;
  int nr = 1;
  hm_dtype dense_dtype = HM_F32, lr_dtype = HM_F32;
  bool has_hi = false;
};
void launch_matvec_view(const CompView& V, int nrr, int vb, bool hi, const void* X, int64_t ldx, void* Y, int64_t ldy,
                        const Epilogue& ep, const int* slot_active, hipStream_t s, hipEvent_t* ev = nullptr);

inline int pad_width(int nrhs) { return nrhs <= 1 ? 1 : nrhs <= 2 ? 2 : nrhs <= 4 ? 4 : nrhs <= 8 ? 8 : 16; }
int64_t matrix_bytes(const hm_matrix& M, bool hi);

// ---------------------------------------------------------------- finite-element coupling
hm_fe* fe_create(hm_ctx& ctx, const hm_matrix& F, int64_t nn, const double* vtx, int64_t nf, const int32_t* tri,
                 const double* eps, const hm_fe_params& p);
void fe_cavity_load(hm_ctx& ctx, hm_fe& fe, const double* T, double* Q);
hm_fe_info fe_step(hm_ctx& ctx, hm_fe& fe, const double* Tn, const double* f_facet, double* T_out);
void fe_destroy(hm_fe* fe);
int fe_device(const hm_fe& fe);
const hm_matrix* fe_matrix(const hm_fe& fe);
int64_t fe_nodes(const hm_fe& fe);
int64_t fe_facets(const hm_fe& fe);

struct LrInfo {
  BlockRef b;
  int32_t k;
  int32_t stage;         // stage buffer holding the FP32/FP64 factors
  int64_t su, sv;        // element offsets of U_b (m x k) and V_b (n x k), column-major
};

// ---------------------------------------------------------------- block LU support
// One block of the reflection matrix for the block LU: dense (D, m x n) or
// low-rank (U m x k, V n x k), FP64, column-major.
struct BlockFactor {
  bool lowrank = false;
  int32_t k = 0;
  int64_t su = 0, sv = 0;  // staging offsets (internal to reflection_blocks)
  DevBuf D, U, V;
};
void reflection_blocks(hm_ctx& ctx, const hm_tree& t, const double* om, const std::vector<BlockRef>& blocks,
                       std::vector<uint8_t>& dense, const hm_assembly_params& p, std::vector<BlockFactor>& out);

hm_hlu* hlu_factor(hm_ctx& ctx, const hm_tree& t, const double* eps, const hm_assembly_params& p);
void hlu_solve(hm_ctx& ctx, const hm_hlu& H, int nrhs, const double* B, int64_t ldb, double* X, int64_t ldx);
void hlu_stats(const hm_hlu& H, int64_t* bytes, int64_t* entries, int32_t* max_rank, double* seconds);
int64_t hlu_rows(const hm_hlu& H);
int hlu_device(const hm_hlu& H);
void hlu_destroy(hm_hlu* H);  // waits for the device, then frees

// ---------------------------------------------------------------- misc helpers
const char* tl_error();
void set_tl_error(const std::string& m);

}  // namespace hm
