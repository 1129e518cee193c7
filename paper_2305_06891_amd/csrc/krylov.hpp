// Batched restarted GMRES on gfx950 for the radiosity system
// (I - diag(1 - eps) F) J = b, with F applied as an H-matrix product.
#pragma once

#include <memory>

#include "hm_internal.hpp"

namespace hm {

constexpr int MAXM = 64;       // largest restart length
constexpr int GS_T = 256;      // threads per reduction chunk
constexpr int GS_RPT = 8;      // rows per thread
constexpr int GS_ROWS = GS_T * GS_RPT;
constexpr int GS_MIN_CHUNKS = 64;  // chunks per system, where it has 256 rows a chunk

// One independent linear system: rows [row0, row0+n) of column col of the
// combined N x width vector block, belonging to slot `slot`.
struct SysDev {
  int64_t row0;
  int32_t n, col, slot, chunk0;  // chunk0: index of the system's first reduction chunk
};

struct ChunkDev {
  int32_t sys, r0, nr, part, pidx, nparts;
};

// Systems of a composition plus their reduction chunks (host + device).
struct SysSet {
  std::vector<SysDev> sys;
  std::vector<ChunkDev> chunks;
  int32_t nparts = 0;
  DevBuf d_sys, d_chunks;
  void build(const Composition& C, const std::vector<std::vector<int>>& cols_per_slot, hipStream_t s);
  int size() const { return (int)sys.size(); }
};

struct GmresStats {
  int iters = 0;       // Arnoldi steps (max over systems)
  int matvecs = 0;
  int64_t bytes = 0;
  std::vector<double> rel_res;  // final |b - Cx| / |b| per system
  bool converged = true;
};

// Copies a few kilobytes between pinned host memory (its device view) and
// device memory with a kernel on stream s: unlike a runtime copy it needs no
// DMA engine, whose hand-over to the next kernel costs tens of
// microseconds.  bytes and both addresses: multiples of 8.
void copy_small(const void* src, void* dst, size_t bytes, hipStream_t s);

// Pinned host memory, mapped for kernels and coherent, for small exchanges.
void* pinned_alloc(size_t bytes, void** dev);

// Pinned host memory for small host <-> device exchanges (copies from
// pageable memory go through a bounce buffer and take tens of microseconds
// each).  A lease takes a buffer of at least `need` bytes from a process-wide
// free list and returns it when it ends; the holder makes sure every copy
// from or to it has completed by then (a lease left by an exception keeps
// its buffer).  Buffers are never freed: a few per thread that solves.
struct PinnedLease {
  void* p = nullptr;    // host pointer
  void* dev = nullptr;  // the same memory as kernels see it
  size_t bytes = 0;
  explicit PinnedLease(size_t need);
  ~PinnedLease();
  PinnedLease(const PinnedLease&) = delete;
  PinnedLease& operator=(const PinnedLease&) = delete;
};

// Workspace of the Krylov iteration for one composition and vector type.
// A captured block of Arnoldi steps (kernels only) and what it was captured for.
struct StepGraph {
  bool hi = false;
  bool cgs1 = false;
  const void* omeps = nullptr;
  const void* x = nullptr;  // the iterate the block's update writes
  int nrr = 0, j0 = 0, nsteps = 0;
  hipGraphExec_t exec = nullptr;
};

struct Krylov {
  Krylov() = default;
  Krylov(const Krylov&) = delete;
  Krylov& operator=(const Krylov&) = delete;
  ~Krylov();
  const Composition* C = nullptr;
  SysSet* S = nullptr;
  int vb = 8;           // vector element bytes
  int m = 30;
  int64_t ld = 0;       // leading dimension of vector blocks (= C->N)
  int64_t blk = 0;      // elements per vector block (ld * width)
  DevBuf basis, w, r;   // basis: (m+1) blocks
  DevBuf H, cs, sn, hA, hB, hn, beta, part, cnt;
  // The scalars the host exchanges with the device every cycle, packed in
  // one buffer (the host's pinned staging has the same layout, so each
  // exchange is one copy):
  //   g[ns (MAXM+1)] tol[ns] bnorm[ns] (doubles), act[ns] steps[ns] slot_cnt[nslots] (ints)
  DevBuf xch;
  double *g = nullptr, *tol = nullptr, *bnorm = nullptr;
  int *act = nullptr, *steps = nullptr, *slot_cnt = nullptr;
  size_t xch_bytes = 0;  // a multiple of 8
  // pinned host side: the exchange block, then ns doubles of norms; the
  // kernels use its device view xch_hd.  Leased from the process-wide pool
  // (workspaces are built per serving round), never touched by the device
  // once a call on this workspace has returned.
  std::unique_ptr<PinnedLease> xch_lease;
  void* xch_h = nullptr;
  void* xch_hd = nullptr;
  // graphs of Arnoldi step blocks (valid while the buffers above and the
  // composition stay as they are; init drops them)
  std::vector<StepGraph> graphs;
  hipStream_t cap = nullptr;  // private stream used only to capture
  void drop_graphs();
  void init(const Composition& C, SysSet& S, int vec_bytes, int restart, hipStream_t s);
};

// Options of gmres().
enum : unsigned {
  // x is zero on entry: the first residual is b itself (no product).  For
  // the same number of products this searches a Krylov space that contains
  // the one of the start x = b, so it never ends with a larger residual.
  GM_X0_ZERO = 1u,
  // return as soon as every system's GMRES residual estimate (the last
  // Givens-rotated entry) meets the tolerance, without the closing product
  // for the true residual; rel_res then holds the estimates.  For inner
  // solves whose result the caller checks with its own residual.
  GM_TRUST_ESTIMATE = 2u,
  // one Gram-Schmidt pass per Arnoldi step (classical, without the second,
  // re-orthogonalising pass): for inner solves to a loose tolerance whose
  // result the caller checks with its own residual
  GM_CGS1 = 4u,
};

// Solve C x = b for every system of S.  b, x: vector blocks (ld = C.N) of
// the Krylov vector type; x holds the initial guess on entry.  omeps: per
// row (1 - eps) in the vector type.  hi selects the FP32 factor copy.
// bnorm: the per-system 2-norms of b when the caller has them (host array),
// else NULL (they are computed here, one host round trip).
GmresStats gmres(Krylov& K, bool hi, const void* omeps, const void* b, void* x, double rtol, int max_iter,
                 hipStream_t s, bool graphs = false, unsigned opts = 0, const double* bnorm = nullptr);



// Per-system 2-norms of a vector block (FP64 accumulation).
void block_norms(Krylov& K, const void* v, std::vector<double>& out, hipStream_t s);

}  // namespace hm
