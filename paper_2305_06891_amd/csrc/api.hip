// C entry points of the library (see include/hm.h): contexts, assembly,
// products, solves and the transient driver.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <map>

#include "convergence.hpp"
#include "dev_common.hpp"
#include "solve.hpp"

namespace hm {

namespace {
thread_local std::string g_tl_error;
std::atomic<uint64_t> g_next_id{1};
}  // namespace

const char* tl_error() { return g_tl_error.c_str(); }
void set_tl_error(const std::string& m) { g_tl_error = m; }

hm_matrix* assemble(hm_ctx& ctx, const hm_tree& t, const hm_assembly_params& p);
std::vector<hm_matrix*> assemble_batch(hm_ctx& ctx, const std::vector<const hm_tree*>& trees,
                                       const std::vector<hm_assembly_params>& ps, bool tune_jointly);

// Per-matrix cache: compositions for plain products, permuted vector
// buffers, and batched-solve state keyed by the ids of its matrices.
// Products leave their work queued when they return; `done` marks the end of
// the last product's work on `last`, and a product on another stream waits
// for it before it touches the shared buffers (xp, yp and the composition's
// scratch).
struct MatCache {
  std::map<int, std::unique_ptr<Composition>> comps;
  DevBuf xp, yp;
  std::map<std::vector<uint64_t>, std::unique_ptr<Batch>> batches;
  hipEvent_t done = nullptr;
  hipStream_t last = nullptr;
  bool pending = false;
  ~MatCache() {
    if (done) (void)hipEventDestroy(done);
  }
};

MatCache& cache_of(const hm_matrix& M) {
  auto& mm = const_cast<hm_matrix&>(M);
  if (!mm.cache) mm.cache = std::shared_ptr<void>(new MatCache(), [](void* p) { delete (MatCache*)p; });
  return *(MatCache*)mm.cache.get();
}

Batch& batch_for(const std::vector<const hm_matrix*>& mats, int nrhs, hipStream_t s) {
  std::vector<uint64_t> key;
  for (const auto* M : mats) key.push_back(M->id);
  key.push_back((uint64_t)nrhs);
  MatCache& mc = cache_of(*mats[0]);
  auto it = mc.batches.find(key);
  if (it != mc.batches.end()) return *it->second;
  auto b = std::make_unique<Batch>(mats, nrhs, s);
  Batch& r = *b;
  mc.batches[key] = std::move(b);
  return r;
}

template <class VT>
__global__ void k_perm_gather(const int32_t* __restrict__ perm, const VT* __restrict__ in, int64_t ldi,
                              VT* __restrict__ out, int64_t ldo, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i < n) out[i + j * ldo] = in[perm[i] + j * ldi];
}

template <class VT>
__global__ void k_perm_scatter(const int32_t* __restrict__ perm, const VT* __restrict__ in, int64_t ldi,
                               VT* __restrict__ out, int64_t ldo, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i < n) out[perm[i] + j * ldo] = in[i + j * ldi];
}

// Streams a buffer through the caches without writing it (evicts the
// last-level cache with clean lines); the sum is kept only if it is NaN.
__global__ void k_flush_read(const float4* __restrict__ p, int64_t n4, float* __restrict__ sink) {
  float acc = 0.f;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n4; k += (int64_t)gridDim.x * blockDim.x) {
    const float4 v = p[k];
    acc += v.x + v.y + v.z + v.w;
  }
  if (acc != acc) sink[0] = acc;
}

__global__ void k_check_range(const double* __restrict__ v, int64_t n, int64_t ld, int ncol, double lo, double hi,
                              int lo_open, int* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n || j >= ncol) return;
  const double x = v[i + j * ld];
  const bool ok = (lo_open ? x > lo : x >= lo) && x <= hi;  // false for NaN
  if (!ok) atomicOr(bad, 1);
}

// Device-side validation of caller vectors (no copy to the host).
void check_device_range(hm_ctx& c, const double* v, int64_t n, int64_t ld, int ncol, double lo, double hi,
                        bool lo_open, const char* what) {
  DevBuf flag(4);
  HM_HIP(hipMemsetAsync(flag.get(), 0, 4, c.stream));
  hipLaunchKernelGGL(k_check_range, dim3((unsigned)((n + 255) / 256), (unsigned)ncol), dim3(256), 0, c.stream, v, n,
                     ld, ncol, lo, hi, lo_open ? 1 : 0, flag.get<int>());
  HM_HIP(hipGetLastError());
  int bad = 0;
  HM_HIP(hipMemcpyAsync(&bad, flag.get(), 4, hipMemcpyDeviceToHost, c.stream));
  HM_HIP(hipStreamSynchronize(c.stream));
  if (bad) fail(HM_EINVAL, std::string(what) + " out of range or not finite");
}

}  // namespace hm

// ---------------------------------------------------------------- allocation-free product
// Device scratch of hm_hmatvec_noalloc: a fixed array in the library's code
// object, so the entry point needs no allocation.  Each device the library
// runs on holds its own copy until the process ends.  Host code never passes
// the array's name to a kernel or a copy (on the host it is only a stand-in
// symbol): it uses the device address that hipGetSymbolAddress returns for
// the current device, taken once per device when a context is created.
static __device__ __align__(256) unsigned char scratch[HM_NOALLOC_SCRATCH_BYTES];

namespace hm {
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The calling thread's current device must be `device`.
void scratch_setup(int device) {
  HM_REQUIRE(device >= 0 && device < kMaxDevices, "hm_ctx_create: device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* p = nullptr;
  HM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  HM_REQUIRE(p != nullptr, "hm_ctx_create: no device address for the product scratch");
  g_scratch_ptr[device] = p;
}

void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
}

// Writes the two slot descriptors (factors as stored, FP32 copies) and a
// zero slot index for every work item of a one-matrix product.
__global__ void k_noalloc_tables(SlotDev lo, SlotDev hi, SlotDev* __restrict__ slots, int32_t* __restrict__ slot_of,
                                 int32_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    slots[0] = lo;
    slots[1] = hi;
  }
  if (i < count) slot_of[i] = 0;
}

constexpr int64_t align256(int64_t b) { return (b + 255) & ~int64_t(255); }
}  // namespace
}  // namespace hm

int64_t hm_matrix::bytes_device() const {
  int64_t b = (int64_t)(dense.bytes() + dense_hi.bytes() + U.bytes() + V.bytes() + U_hi.bytes() + V_hi.bytes() +
                        d_perm.bytes());
  b += (int64_t)(plan.d_p1.bytes() + plan.d_p1_task.bytes() + plan.d_p1red.bytes() + plan.d_p2t.bytes() + plan.d_p2.bytes() +
                 plan.d_segs.bytes());
  return b;
}

using namespace hm;

namespace {

template <class F>
hm_status guarded(hm_ctx* ctx, F&& f) {
  try {
    if (ctx) HM_HIP(hipSetDevice(ctx->device));
    StreamScope scope(ctx ? ctx->stream : current_stream());
    f();
    return HM_OK;
  } catch (const Error& e) {
    if (ctx) ctx->last_error = e.what();
    set_tl_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->last_error = "out of host memory";
    set_tl_error("out of host memory");
    return HM_ENOMEM;
  } catch (const std::exception& e) {
    if (ctx) ctx->last_error = e.what();
    set_tl_error(e.what());
    return HM_EDEVICE;
  }
}

void check_params(const hm_solve_params* p) {
  HM_REQUIRE(p, "solve: NULL params");
  HM_REQUIRE(p->rtol > 0.0 && p->rtol < 1.0, "solve: rtol must be in (0, 1)");
  HM_REQUIRE(p->restart >= 1 && p->restart <= MAXM, "solve: restart must be in 1..64");
  HM_REQUIRE(p->max_iter >= 1, "solve: max_iter must be >= 1");
  HM_REQUIRE(!p->mixed_precision || (p->ir_inner_rtol > 0.0 && p->ir_inner_rtol < 1.0),
             "solve: ir_inner_rtol must be in (0, 1)");
  HM_REQUIRE(p->vec_dtype == HM_F64 || p->vec_dtype == HM_F32, "solve: vec_dtype must be HM_F64 or HM_F32");
  HM_REQUIRE(p->use_graphs == 0 || p->use_graphs == 1, "solve: use_graphs must be 0 or 1");
  HM_REQUIRE(p->open_cavity == 0 || p->open_cavity == 1, "solve: open_cavity must be 0 or 1");
  HM_REQUIRE(!p->open_cavity || (std::isfinite(p->ambient_temperature) && p->ambient_temperature > 0.0),
             "solve: ambient_temperature must be positive and finite for an open cavity");
}

}  // namespace

extern "C" {

const char* hm_version(void) { return "hmrad 1.0 gfx950"; }

const char* hm_status_string(hm_status s) {
  switch (s) {
    case HM_OK: return "ok";
    case HM_EINVAL: return "invalid argument";
    case HM_ENOMEM: return "out of memory";
    case HM_ENOTCONV: return "not converged";
    case HM_EDEVICE: return "device error";
    case HM_EBUSY: return "busy";
    case HM_ENOTFOUND: return "not found";
  }
  return "unknown status";
}

const char* hm_last_error(const hm_ctx* ctx) { return ctx ? ctx->last_error.c_str() : tl_error(); }

hm_status hm_ctx_create(int device, void* hip_stream, hm_ctx** out) {
  if (!out) {
    set_tl_error("hm_ctx_create: NULL out");
    return HM_EINVAL;
  }
  auto c = std::make_unique<hm_ctx>();
  c->device = device;
  hm_status st = guarded(nullptr, [&] {
    int nd = 0;
    HM_HIP(hipGetDeviceCount(&nd));
    HM_REQUIRE(device >= 0 && device < nd, "hm_ctx_create: no such device");
    HM_HIP(hipSetDevice(device));
    c->stream = (hipStream_t)hip_stream;  // NULL: the null stream
    scratch_setup(device);
  });
  if (st == HM_OK) *out = c.release();
  return st;
}

void hm_ctx_destroy(hm_ctx* ctx) {
  if (!ctx) return;
  if (ctx->own_stream) {
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipStreamDestroy(ctx->stream);
  }
  delete ctx;
}

hm_status hm_ctx_synchronize(hm_ctx* ctx) {
  if (!ctx) return HM_EINVAL;
  return guarded(ctx, [&] { HM_HIP(hipStreamSynchronize(ctx->stream)); });
}

namespace {
void check_assembly_params(const hm_assembly_params* p, const char* fn) {
  const std::string f(fn);
  HM_REQUIRE(p->aca_tol > 0.0 && p->aca_tol < 1.0, f + ": aca_tol must be in (0, 1)");
  HM_REQUIRE(p->k_max >= 1, f + ": k_max must be >= 1");
  HM_REQUIRE(p->lowrank_dtype == HM_F64 || p->lowrank_dtype == HM_F32 || p->lowrank_dtype == HM_BF16,
             f + ": bad lowrank_dtype");
  HM_REQUIRE(p->dense_dtype == HM_F64 || p->dense_dtype == HM_F32 || p->dense_dtype == HM_BF16,
             f + ": bad dense_dtype");
  HM_REQUIRE(!(p->dense_dtype == HM_F64 && p->lowrank_dtype == HM_BF16), f + ": BF16 factors need FP32 near field");
  HM_REQUIRE(p->dense_dtype != HM_BF16 || (p->lowrank_dtype == HM_BF16 && p->keep_f32_copy),
             f + ": a BF16 near field needs BF16 factors and keep_f32_copy (FP32 copies for FP64-vector products)");
  HM_REQUIRE(p->dense_dtype != HM_BF16 || !p->closed_row_scale, f + ": closed_row_scale needs an FP32 or FP64 near field");
  HM_REQUIRE(p->autotune >= 0 && p->autotune <= 16, f + ": autotune must be in 0..16");
  HM_REQUIRE(p->recompress == 0 || p->recompress == 1, f + ": recompress must be 0 or 1");
  HM_REQUIRE(p->aca_pivot == 0 || p->aca_pivot == 1, f + ": aca_pivot must be 0 or 1");
  HM_REQUIRE(p->lowrank_rounding == 0 || p->lowrank_rounding == 1, f + ": lowrank_rounding must be 0 or 1");
  HM_REQUIRE(p->lowrank_rounding == 0 || (p->lowrank_dtype == HM_BF16 && !p->closed_row_scale),
             f + ": dithered rounding needs BF16 factors and no closed_row_scale");
}
}  // namespace

hm_status hm_assemble_hmatrix(hm_ctx* ctx, const hm_tree* tree, const hm_assembly_params* p, hm_matrix** out) {
  if (!ctx) {
    set_tl_error("hm_assemble_hmatrix: NULL ctx");
    return HM_EINVAL;
  }
  return guarded(ctx, [&] {
    HM_REQUIRE(tree && p && out, "hm_assemble_hmatrix: NULL argument");
    check_assembly_params(p, "hm_assemble_hmatrix");
    hm_matrix* M = assemble(*ctx, *tree, *p);
    M->id = g_next_id++;
    *out = M;
  });
}

hm_status hm_assemble_hmatrix_batched(hm_ctx* ctx, int32_t count, const hm_tree* const* trees,
                                      const hm_assembly_params* params, hm_matrix** out) {
  if (!ctx) {
    set_tl_error("hm_assemble_hmatrix_batched: NULL ctx");
    return HM_EINVAL;
  }
  return guarded(ctx, [&] {
    HM_REQUIRE(count >= 1, "hm_assemble_hmatrix_batched: count must be >= 1");
    HM_REQUIRE(trees && params && out, "hm_assemble_hmatrix_batched: NULL argument");
    std::vector<const hm_tree*> ts(count);
    std::vector<hm_assembly_params> ps(count);
    for (int32_t i = 0; i < count; ++i) {
      HM_REQUIRE(trees[i], "hm_assemble_hmatrix_batched: NULL tree");
      check_assembly_params(params + i, "hm_assemble_hmatrix_batched");
      ts[i] = trees[i];
      ps[i] = params[i];
    }
    std::vector<hm_matrix*> ms = assemble_batch(*ctx, ts, ps, true);
    for (int32_t i = 0; i < count; ++i) {
      ms[i]->id = g_next_id++;
      out[i] = ms[i];
    }
  });
}

hm_status hm_matrix_stats(const hm_matrix* M, int64_t* bytes, int64_t* ed, int64_t* el, int32_t* maxr) {
  if (!M) {
    set_tl_error("hm_matrix_stats: NULL matrix");
    return HM_EINVAL;
  }
  if (bytes) *bytes = M->bytes_device();
  if (ed) *ed = M->dense_entries;
  if (el) *el = M->lr_entries;
  if (maxr) *maxr = M->max_rank;
  return HM_OK;
}

hm_status hm_matrix_info(const hm_matrix* M, int64_t* n, int64_t* nd, int64_t* nl, int64_t* nf, int64_t* rs) {
  if (!M) {
    set_tl_error("hm_matrix_info: NULL matrix");
    return HM_EINVAL;
  }
  if (n) *n = M->n;
  if (nd) *nd = M->n_dense_blocks;
  if (nl) *nl = M->n_lr_blocks;
  if (nf) *nf = M->n_fallback;
  if (rs) *rs = M->rank_sum;
  return HM_OK;
}

hm_status hm_matrix_tuning(const hm_matrix* M, int32_t* rows, int32_t* task_bytes, double* us) {
  if (!M) {
    set_tl_error("hm_matrix_tuning: NULL matrix");
    return HM_EINVAL;
  }
  if (rows) *rows = M->plan.p1p.rows;
  if (task_bytes) *task_bytes = M->plan.p1p.task_bytes;
  if (us) *us = M->plan.p1_us;
  return HM_OK;
}

hm_status hm_matrix_set_tuning(hm_ctx* ctx, hm_matrix* M, int32_t rows, int32_t task_bytes) {
  if (!ctx) {
    set_tl_error("hm_matrix_set_tuning: NULL ctx");
    return HM_EINVAL;
  }
  return guarded(ctx, [&] {
    HM_REQUIRE(M, "hm_matrix_set_tuning: NULL matrix");
    HM_REQUIRE(M->device == ctx->device, "hm_matrix_set_tuning: matrix lives on another device");
    HM_REQUIRE(rows >= 64 && rows % 64 == 0 && rows <= (1 << 20), "hm_matrix_set_tuning: p1_rows must be a positive multiple of 64");
    HM_REQUIRE(task_bytes >= 0, "hm_matrix_set_tuning: p1_task_bytes must be >= 0");
    P1Params pp;
    pp.rows = rows;
    pp.task_bytes = task_bytes;
    std::lock_guard<std::mutex> lk(M->mu);
    // every composition, batch and captured graph built on M copied the old
    // phase-1 lists and counts: wait for all work that may use them, drop
    // M's caches, and give M a new id so that batches cached under other
    // matrices (keyed by the ids of their members) no longer match it
    HM_HIP(hipDeviceSynchronize());
    M->cache.reset();
    replan_phase1(*M, pp, ctx->stream);
    HM_HIP(hipStreamSynchronize(ctx->stream));
    M->plan.p1_us = 0.0;
    M->id = g_next_id++;
  });
}

hm_status hm_matrix_tuning_phase2(const hm_matrix* M, int32_t* p2_waves, double* us) {
  if (!M) {
    set_tl_error("hm_matrix_tuning_phase2: NULL matrix");
    return HM_EINVAL;
  }
  if (p2_waves) *p2_waves = M->plan.p2_waves;
  if (us) *us = M->plan.p2_us;
  return HM_OK;
}

hm_status hm_matrix_set_tuning_phase2(hm_ctx* ctx, hm_matrix* M, int32_t p2_waves) {
  if (!ctx) {
    set_tl_error("hm_matrix_set_tuning_phase2: NULL ctx");
    return HM_EINVAL;
  }
  return guarded(ctx, [&] {
    HM_REQUIRE(M, "hm_matrix_set_tuning_phase2: NULL matrix");
    HM_REQUIRE(M->device == ctx->device, "hm_matrix_set_tuning_phase2: matrix lives on another device");
    HM_REQUIRE(p2_waves == 0 || p2_waves == 2 || p2_waves == 4 || p2_waves == 8,
               "hm_matrix_set_tuning_phase2: p2_waves must be 0, 2, 4 or 8");
    std::lock_guard<std::mutex> lk(M->mu);
    // compositions and captured graphs copied the old shape: drop them as
    // hm_matrix_set_tuning does
    HM_HIP(hipDeviceSynchronize());
    M->cache.reset();
    M->plan.p2_waves = p2_waves;
    M->plan.p2_us = 0.0;
    M->id = g_next_id++;
  });
}

void hm_matrix_destroy(hm_matrix* M) {
  if (!M) return;
  (void)hipSetDevice(M->device);
  (void)hipDeviceSynchronize();
  delete M;
}

hm_status hm_hmatvec_ex(hm_ctx* ctx, const hm_matrix* M, int32_t nrhs, hm_dtype vt, int32_t use_hi, const void* X,
                        int64_t ldx, void* Y, int64_t ldy, double alpha, double beta) {
  if (!ctx) {
    set_tl_error("hm_hmatvec: NULL ctx");
    return HM_EINVAL;
  }
  return guarded(ctx, [&] {
    HM_REQUIRE(M && X && Y, "hm_hmatvec: NULL argument");
    HM_REQUIRE(nrhs >= 1 && nrhs <= 16, "hm_hmatvec: nrhs must be in 1..16");
    HM_REQUIRE(vt == HM_F64 || vt == HM_F32, "hm_hmatvec: vec_dtype must be HM_F64 or HM_F32");
    HM_REQUIRE(ldx >= M->n && ldy >= M->n, "hm_hmatvec: leading dimension smaller than n");
    HM_REQUIRE(std::isfinite(alpha) && std::isfinite(beta), "hm_hmatvec: alpha/beta must be finite");
    std::lock_guard<std::mutex> lk(const_cast<hm_matrix*>(M)->mu);
    hipStream_t s = ctx->stream;
    MatCache& mc = cache_of(*M);
    if (mc.pending && mc.last != s) HM_HIP(hipStreamWaitEvent(s, mc.done, 0));
    const int W = pad_width(nrhs);
    auto& comp = mc.comps[W];
    if (!comp) comp = make_composition({M}, W, 8, s);
    const int64_t n = M->n;
    const size_t need = (size_t)n * W * 8;
    if (mc.xp.bytes() < need) {
      mc.xp.alloc(need);
      mc.yp.alloc(need);
    }
    const int vb = vt == HM_F64 ? 8 : 4;
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)nrhs);
    const int32_t* perm = M->d_perm.get<int32_t>();
    if (vb == 8) {
      hipLaunchKernelGGL(k_perm_gather<double>, grid, dim3(256), 0, s, perm, (const double*)X, ldx,
                         mc.xp.get<double>(), n, n);
      if (beta != 0.0)
        hipLaunchKernelGGL(k_perm_gather<double>, grid, dim3(256), 0, s, perm, (const double*)Y, ldy,
                           mc.yp.get<double>(), n, n);
    } else {
      hipLaunchKernelGGL(k_perm_gather<float>, grid, dim3(256), 0, s, perm, (const float*)X, ldx, mc.xp.get<float>(),
                         n, n);
      if (beta != 0.0)
        hipLaunchKernelGGL(k_perm_gather<float>, grid, dim3(256), 0, s, perm, (const float*)Y, ldy,
                           mc.yp.get<float>(), n, n);
    }
    HM_HIP(hipGetLastError());
    Epilogue ep;
    ep.a_acc = alpha;
    ep.a_z = beta;
    ep.z = beta != 0.0 ? mc.yp.get() : nullptr;
    ep.ldz = n;
    launch_matvec(*comp, nrhs, vb, use_hi != 0, mc.xp.get(), n, mc.yp.get(), n, ep, nullptr, s);
    if (vb == 8)
      hipLaunchKernelGGL(k_perm_scatter<double>, grid, dim3(256), 0, s, perm, mc.yp.get<double>(), n, (double*)Y, ldy, n);
    else
      hipLaunchKernelGGL(k_perm_scatter<float>, grid, dim3(256), 0, s, perm, mc.yp.get<float>(), n, (float*)Y, ldy, n);
    HM_HIP(hipGetLastError());
    if (!mc.done) HM_HIP(hipEventCreateWithFlags(&mc.done, hipEventDisableTiming));
    HM_HIP(hipEventRecord(mc.done, s));
    mc.last = s;
    mc.pending = true;
  });
}

hm_status hm_hmatvec(hm_ctx* ctx, const hm_matrix* M, int32_t nrhs, hm_dtype vt, const void* X, int64_t ldx,
                     void* Y, int64_t ldy, double alpha, double beta) {
  return hm_hmatvec_ex(ctx, M, nrhs, vt, 0, X, ldx, Y, ldy, alpha, beta);
}

hm_status hm_hmatvec_noalloc(hm_ctx* ctx, const hm_matrix* M, int32_t nrhs, hm_dtype vt, const void* X, int64_t ldx,
                             void* Y, int64_t ldy, double alpha, double beta) {
  if (!ctx) {
    set_tl_error("hm_hmatvec_noalloc: NULL ctx");
    return HM_EINVAL;
  }
  return guarded(ctx, [&] {
    HM_REQUIRE(M && X && Y, "hm_hmatvec_noalloc: NULL argument");
    HM_REQUIRE(nrhs >= 1 && nrhs <= 16, "hm_hmatvec_noalloc: nrhs must be in 1..16");
    HM_REQUIRE(vt == HM_F64 || vt == HM_F32, "hm_hmatvec_noalloc: vec_dtype must be HM_F64 or HM_F32");
    HM_REQUIRE(ldx >= M->n && ldy >= M->n, "hm_hmatvec_noalloc: leading dimension smaller than n");
    HM_REQUIRE(std::isfinite(alpha) && std::isfinite(beta), "hm_hmatvec_noalloc: alpha/beta must be finite");
    HM_REQUIRE(M->device == ctx->device, "hm_hmatvec_noalloc: matrix and context on different devices");
    char* base = (char*)scratch_ptr(ctx->device);
    HM_REQUIRE(base != nullptr, "hm_hmatvec_noalloc: no scratch address for this device");
    std::lock_guard<std::mutex> lk(const_cast<hm_matrix*>(M)->mu);
    const hipStream_t s = ctx->stream;
    const Plan& P = M->plan;
    const int W = pad_width(nrhs);
    const int64_t n = M->n;
    const int32_t p1_tasks = (int32_t)P.p1_task.size() - 1, p1_reds = (int32_t)P.p1red.size(),
                  p2_tiles = (int32_t)P.p2t.size();
    const int32_t count = p1_tasks + p1_reds + p2_tiles + 1;
    // scratch layout: slot tables, slot indices, permuted x and y, rank
    // intermediates t, phase-1 partial sums, row-major inputs (16 columns);
    // the vector buffers are sized for FP64 as in hm_hmatvec
    int64_t off = 0;
    const int64_t o_slots = off;
    off += align256(2 * (int64_t)sizeof(SlotDev));
    const int64_t o_sof = off;
    off += align256((int64_t)count * 4);
    const int64_t o_xp = off;
    off += align256(n * W * 8);
    const int64_t o_yp = off;
    off += align256(n * W * 8);
    const int64_t o_t = off;
    off += align256(std::max<int64_t>(1, M->Ktot * W) * 8);
    const int64_t o_p1 = off;
    off += align256(std::max<int64_t>(1, (int64_t)P.n_p1_parts * P1_GW * W) * 8);
    const int64_t o_xr = off;
    if (W == 16) off += align256(n * 16 * 8);
    if (off > (int64_t)HM_NOALLOC_SCRATCH_BYTES)
      fail(HM_ENOMEM, "hm_hmatvec_noalloc: this product needs " + std::to_string(off) +
                          " bytes of scratch, more than the fixed " + std::to_string((int64_t)HM_NOALLOC_SCRATCH_BYTES) +
                          " (use hm_hmatvec)");
    SlotDev d{};
    d.p1 = P.d_p1.get<P1Item>();
    d.p1_task = P.d_p1_task.get<int32_t>();
    d.p1red = P.d_p1red.get<P1Red>();
    d.p2t = P.d_p2t.get<P2Tile>();
    d.p2 = P.d_p2.get<P2Item>();
    d.segs = P.d_segs.get<Seg>();
    d.dense = M->dense.get();
    d.U = M->U.get();
    d.V = M->V.get();
    d.part1 = base + o_p1;
    d.t = base + o_t;
    d.ldt = std::max<int64_t>(1, M->Ktot);
    d.xoff = 0;
    d.n = (int32_t)n;
    SlotDev h = d;
    if (M->has_hi) {
      h.U = M->U_hi.get();
      h.V = M->V_hi.get();
      if (M->dense_dtype == HM_BF16) h.dense = M->dense_hi.get();
    }
    SlotDev* slots = (SlotDev*)(base + o_slots);
    int32_t* sof = (int32_t*)(base + o_sof);
    hipLaunchKernelGGL(k_noalloc_tables, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, d, h, slots, sof,
                       count);
    CompView V;
    V.slots_lo = slots;
    V.slots_hi = slots + 1;
    V.slot_of = sof;
    V.xr = W == 16 ? base + o_xr : nullptr;
    V.N = n;
    V.p1_tasks = p1_tasks;
    V.p1_reds = p1_reds;
    V.p2_tiles = p2_tiles;
    V.p2_waves = M->plan.p2_waves;
    V.nr = W;
    V.dense_dtype = M->dense_dtype;
    V.lr_dtype = M->lr_dtype;
    V.has_hi = M->has_hi;
    void* xp = base + o_xp;
    void* yp = base + o_yp;
    const int vb = vt == HM_F64 ? 8 : 4;
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)nrhs);
    const int32_t* perm = M->d_perm.get<int32_t>();
    if (vb == 8) {
      hipLaunchKernelGGL(k_perm_gather<double>, grid, dim3(256), 0, s, perm, (const double*)X, ldx, (double*)xp, n, n);
      if (beta != 0.0)
        hipLaunchKernelGGL(k_perm_gather<double>, grid, dim3(256), 0, s, perm, (const double*)Y, ldy, (double*)yp, n, n);
    } else {
      hipLaunchKernelGGL(k_perm_gather<float>, grid, dim3(256), 0, s, perm, (const float*)X, ldx, (float*)xp, n, n);
      if (beta != 0.0)
        hipLaunchKernelGGL(k_perm_gather<float>, grid, dim3(256), 0, s, perm, (const float*)Y, ldy, (float*)yp, n, n);
    }
    HM_HIP(hipGetLastError());
    Epilogue ep;
    ep.a_acc = alpha;
    ep.a_z = beta;
    ep.z = beta != 0.0 ? yp : nullptr;
    ep.ldz = n;
    launch_matvec_view(V, nrhs, vb, false, xp, n, yp, n, ep, nullptr, s);
    if (vb == 8)
      hipLaunchKernelGGL(k_perm_scatter<double>, grid, dim3(256), 0, s, perm, (const double*)yp, n, (double*)Y, ldy, n);
    else
      hipLaunchKernelGGL(k_perm_scatter<float>, grid, dim3(256), 0, s, perm, (const float*)yp, n, (float*)Y, ldy, n);
    HM_HIP(hipGetLastError());
  });
}

hm_status hm_hmatvec_profile(hm_ctx* ctx, int32_t count, const hm_matrix* const* Ms, int32_t nrhs, hm_dtype vt,
                             int32_t use_hi, int32_t reps, int64_t flush_bytes, double* ms1, double* ms2, double* mst,
                             int64_t* b1, int64_t* b2) {
  if (!ctx) {
    set_tl_error("hm_hmatvec_profile: NULL ctx");
    return HM_EINVAL;
  }
  return guarded(ctx, [&] {
    HM_REQUIRE(count >= 1 && Ms && reps >= 1 && nrhs >= 1 && nrhs <= 16 && flush_bytes >= 0,
               "hm_hmatvec_profile: bad arguments");
    HM_REQUIRE(vt == HM_F64 || vt == HM_F32, "hm_hmatvec_profile: vec_dtype must be HM_F64 or HM_F32");
    std::vector<const hm_matrix*> mats(Ms, Ms + count);
    for (const hm_matrix* M : mats) {
      HM_REQUIRE(M, "hm_hmatvec_profile: NULL matrix");
      HM_REQUIRE(M->device == ctx->device, "hm_hmatvec_profile: matrix lives on another device");
    }
    hipStream_t s = ctx->stream;
    const int W = pad_width(nrhs);
    const int vb = vt == HM_F64 ? 8 : 4;
    // a composition of its own: the matrices' cached compositions are left alone
    auto comp = make_composition(mats, W, vb, s);
    const int64_t N = comp->N;
    DevBuf X((size_t)N * W * vb), Y((size_t)N * W * vb), flush(flush_bytes > 0 ? (size_t)flush_bytes : 0), sink(16);
    if (flush_bytes > 0) HM_HIP(hipMemsetAsync(flush.get(), 0, (size_t)flush_bytes, s));
    {
      std::vector<char> h((size_t)N * W * vb);
      if (vb == 8) {
        double* d = (double*)h.data();
        for (int64_t k = 0; k < N * W; ++k) d[k] = 1.0;
      } else {
        float* f = (float*)h.data();
        for (int64_t k = 0; k < N * W; ++k) f[k] = 1.0f;
      }
      HM_HIP(hipMemcpyAsync(X.get(), h.data(), h.size(), hipMemcpyHostToDevice, s));
      HM_HIP(hipStreamSynchronize(s));
    }
    hipEvent_t ev[3];
    for (auto& e : ev) HM_HIP(hipEventCreate(&e));
    double t1 = 0, t2 = 0;
    const bool hi = use_hi != 0;
    try {
      for (int r = 0; r < reps; ++r) {
        if (flush_bytes > 0)
          hipLaunchKernelGGL(k_flush_read, dim3(1024), dim3(256), 0, s, flush.get<float4>(), flush_bytes / 16,
                             sink.get<float>());
        launch_matvec(*comp, nrhs, vb, hi, X.get(), N, Y.get(), N, Epilogue{}, nullptr, s, ev);
        HM_HIP(hipEventSynchronize(ev[2]));
        float a = 0, b = 0;
        HM_HIP(hipEventElapsedTime(&a, ev[0], ev[1]));
        HM_HIP(hipEventElapsedTime(&b, ev[1], ev[2]));
        t1 += a;
        t2 += b;
      }
    } catch (...) {
      for (auto& e : ev) (void)hipEventDestroy(e);
      throw;
    }
    for (auto& e : ev) HM_HIP(hipEventDestroy(e));
    int64_t by1 = 0, by2 = 0;
    const int64_t vecs = (int64_t)nrhs * vb;
    for (const hm_matrix* M : mats) {
      const bool use_f32 = hi && M->has_hi;
      const int64_t sl = use_f32 ? 4 : (int64_t)dtype_size(M->lr_dtype);
      const int64_t sd = use_f32 && M->dense_dtype == HM_BF16 ? 4 : (int64_t)dtype_size(M->dense_dtype);
      by1 += M->v_entries * sl + vecs * (M->n + M->Ktot);
      by2 += M->dense_entries * sd + M->u_entries * sl + vecs * (2 * M->n + M->Ktot);
    }
    if (ms1) *ms1 = t1 / reps;
    if (ms2) *ms2 = t2 / reps;
    if (mst) *mst = (t1 + t2) / reps;
    if (b1) *b1 = by1;
    if (b2) *b2 = by2;
  });
}

static void fill_info(hm_solve_info* info, const SolveResult& R, double secs, int sys_begin, int sys_end) {
  if (!info) return;
  info->iters = R.iters;
  info->outer_iters = R.outer;
  info->matvecs = R.matvecs;
  info->bytes_moved = R.bytes;
  info->seconds = secs;
  double rr = 0.0;
  for (int q = sys_begin; q < sys_end && q < (int)R.rel_res.size(); ++q) rr = max_keep_nan(rr, R.rel_res[q]);
  info->rel_residual = rr;
}

hm_status hm_solve_radiosity(hm_ctx* ctx, const hm_matrix* M, const double* eps, int32_t nrhs, const double* T,
                             int64_t ldT, double sigma, const hm_solve_params* p, double* J, int64_t ldJ, double* q,
                             int64_t ldq, hm_solve_info* info) {
  if (!ctx) {
    set_tl_error("hm_solve_radiosity: NULL ctx");
    return HM_EINVAL;
  }
  bool conv = true;
  hm_status st = guarded(ctx, [&] {
    const auto t0 = std::chrono::steady_clock::now();
    HM_REQUIRE(M && eps && T && J, "hm_solve_radiosity: NULL argument");
    HM_REQUIRE(nrhs >= 1 && nrhs <= 16, "hm_solve_radiosity: nrhs must be in 1..16");
    HM_REQUIRE(ldT >= M->n && ldJ >= M->n && (!q || ldq >= M->n), "hm_solve_radiosity: leading dimension < n");
    HM_REQUIRE(sigma > 0.0 && std::isfinite(sigma), "hm_solve_radiosity: sigma must be > 0");
    check_params(p);
    check_device_range(*ctx, eps, M->n, M->n, 1, 0.0, 1.0, true, "eps");
    check_device_range(*ctx, T, M->n, ldT, nrhs, 0.0, INFINITY, true, "T");
    std::lock_guard<std::mutex> lk(const_cast<hm_matrix*>(M)->mu);
    Batch& B = batch_for({M}, nrhs, ctx->stream);
    SolveResult R = B.solve({eps}, {T}, {ldT}, sigma, *p, {J}, {ldJ}, {q}, {ldq}, ctx->stream);
    HM_HIP(hipStreamSynchronize(ctx->stream));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_info(info, R, secs, 0, (int)R.rel_res.size());
    conv = R.converged;
  });
  if (st == HM_OK && !conv) {
    ctx->last_error = "hm_solve_radiosity: tolerance not reached within max_iter";
    return HM_ENOTCONV;
  }
  return st;
}

hm_status hm_solve_radiosity_batched(hm_ctx* ctx, int32_t count, const hm_matrix* const* M, const double* const* eps,
                                     const double* const* T, double sigma, const hm_solve_params* p,
                                     double* const* J, double* const* q, hm_solve_info* info_out) {
  if (!ctx) {
    set_tl_error("hm_solve_radiosity_batched: NULL ctx");
    return HM_EINVAL;
  }
  bool conv = true;
  hm_status st = guarded(ctx, [&] {
    const auto t0 = std::chrono::steady_clock::now();
    HM_REQUIRE(count >= 1 && M && eps && T && J, "hm_solve_radiosity_batched: bad arguments");
    HM_REQUIRE(sigma > 0.0 && std::isfinite(sigma), "hm_solve_radiosity_batched: sigma must be > 0");
    check_params(p);
    std::vector<const hm_matrix*> mats(M, M + count);
    std::vector<const double*> ev(eps, eps + count), Tv(T, T + count);
    std::vector<double*> Jv(J, J + count), qv(count, nullptr);
    if (q) qv.assign(q, q + count);
    std::vector<int64_t> ld(count);
    for (int i = 0; i < count; ++i) {
      HM_REQUIRE(mats[i] && ev[i] && Tv[i] && Jv[i], "hm_solve_radiosity_batched: NULL entry");
      HM_REQUIRE(mats[i]->device == ctx->device, "hm_solve_radiosity_batched: matrix on another device");
      ld[i] = mats[i]->n;
    }
    std::lock_guard<std::mutex> lk(const_cast<hm_matrix*>(mats[0])->mu);
    Batch& B = batch_for(mats, 1, ctx->stream);
    SolveResult R = B.solve(ev, Tv, ld, sigma, *p, Jv, ld, qv, ld, ctx->stream);
    HM_HIP(hipStreamSynchronize(ctx->stream));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info_out)
      for (int i = 0; i < count; ++i) fill_info(&info_out[i], R, secs, i, i + 1);
    conv = R.converged;
  });
  if (st == HM_OK && !conv) {
    ctx->last_error = "hm_solve_radiosity_batched: tolerance not reached within max_iter";
    return HM_ENOTCONV;
  }
  return st;
}

hm_status hm_hlu_factor(hm_ctx* ctx, const hm_tree* tree, const double* eps, const hm_assembly_params* p,
                        hm_hlu** out) {
  if (!ctx) {
    set_tl_error("hm_hlu_factor: NULL ctx");
    return HM_EINVAL;
  }
  return guarded(ctx, [&] {
    HM_REQUIRE(tree && eps && p && out, "hm_hlu_factor: NULL argument");
    check_assembly_params(p, "hm_hlu_factor");
    HM_REQUIRE(p->lowrank_dtype == HM_F64 && p->dense_dtype == HM_F64,
               "hm_hlu_factor: the block LU runs in FP64 (lowrank_dtype and dense_dtype HM_F64)");
    check_device_range(*ctx, eps, tree->n, tree->n, 1, 0.0, 1.0, true, "hm_hlu_factor: eps");
    *out = hlu_factor(*ctx, *tree, eps, *p);
  });
}

hm_status hm_hlu_solve(hm_ctx* ctx, const hm_hlu* lu, int32_t nrhs, const double* B, int64_t ldb, double* X,
                       int64_t ldx) {
  if (!ctx) {
    set_tl_error("hm_hlu_solve: NULL ctx");
    return HM_EINVAL;
  }
  return guarded(ctx, [&] {
    HM_REQUIRE(lu && B && X, "hm_hlu_solve: NULL argument");
    HM_REQUIRE(nrhs >= 1 && nrhs <= 65535, "hm_hlu_solve: nrhs must be in 1..65535");
    HM_REQUIRE(ldb >= hlu_rows(*lu) && ldx >= hlu_rows(*lu), "hm_hlu_solve: leading dimension smaller than n");
    HM_REQUIRE(hlu_device(*lu) == ctx->device, "hm_hlu_solve: factors and context on different devices");
    hlu_solve(*ctx, *lu, nrhs, B, ldb, X, ldx);
  });
}

hm_status hm_hlu_stats(const hm_hlu* lu, int64_t* bytes_device, int64_t* entries, int32_t* max_rank,
                       double* factor_seconds) {
  if (!lu) {
    set_tl_error("hm_hlu_stats: NULL factors");
    return HM_EINVAL;
  }
  hlu_stats(*lu, bytes_device, entries, max_rank, factor_seconds);
  return HM_OK;
}

void hm_hlu_destroy(hm_hlu* lu) {
  if (!lu) return;
  hlu_destroy(lu);
}

// ---- finite-element coupling
hm_status hm_fe_create(hm_ctx* ctx, const hm_matrix* F, int64_t n_nodes, const double* vertices,
                       int64_t n_facets, const int32_t* triangles, const double* eps, const hm_fe_params* p,
                       hm_fe** out) {
  if (!ctx) {
    set_tl_error("hm_fe_create: NULL ctx");
    return HM_EINVAL;
  }
  return guarded(ctx, [&] {
    HM_REQUIRE(F && vertices && triangles && eps && p && out, "hm_fe_create: NULL argument");
    HM_REQUIRE(p->conductance >= 0.0 && std::isfinite(p->conductance), "hm_fe_create: conductance must be >= 0");
    HM_REQUIRE(p->capacity > 0.0 && std::isfinite(p->capacity), "hm_fe_create: capacity must be > 0");
    HM_REQUIRE(p->dt > 0.0 && std::isfinite(p->dt), "hm_fe_create: dt must be > 0");
    HM_REQUIRE(p->newton_rtol > 0.0 && p->max_newton >= 1, "hm_fe_create: bad Newton parameters");
    HM_REQUIRE(p->krylov_restart >= 1 && p->krylov_restart <= 64 && p->max_krylov >= 1 && p->krylov_rtol > 0.0,
               "hm_fe_create: bad Krylov parameters");
    HM_REQUIRE(p->pc_rtol > 0.0 && p->pc_rtol < 1.0, "hm_fe_create: pc_rtol must be in (0, 1)");
    HM_REQUIRE(p->sigma > 0.0 && std::isfinite(p->sigma), "hm_fe_create: sigma must be > 0");
    check_params(&p->solve);
    HM_REQUIRE(F->device == ctx->device, "hm_fe_create: matrix and context on different devices");
    check_device_range(*ctx, eps, n_facets, n_facets, 1, 0.0, 1.0, true, "hm_fe_create: eps");
    *out = fe_create(*ctx, *F, n_nodes, vertices, n_facets, triangles, eps, *p);
  });
}

hm_status hm_fe_cavity_load(hm_ctx* c, hm_fe* fe, const double* T, double* Q) {
  if (!c) {
    set_tl_error("hm_fe_cavity_load: NULL ctx");
    return HM_EINVAL;
  }
  hm_ctx& ctx = *c;
  return guarded(c, [&] {
    HM_REQUIRE(fe && T && Q, "hm_fe_cavity_load: NULL argument");
    HM_REQUIRE(fe_device(*fe) == ctx.device, "hm_fe_cavity_load: object and context on different devices");
    check_device_range(ctx, T, fe_nodes(*fe), fe_nodes(*fe), 1, 0.0, INFINITY, true, "hm_fe_cavity_load: T");
    std::lock_guard<std::mutex> lk(const_cast<hm_matrix*>(fe_matrix(*fe))->mu);
    fe_cavity_load(ctx, *fe, T, Q);
  });
}

hm_status hm_fe_step(hm_ctx* c, hm_fe* fe, const double* T_n, const double* f_facet, double* T_out,
                     hm_fe_info* info) {
  if (!c) {
    set_tl_error("hm_fe_step: NULL ctx");
    return HM_EINVAL;
  }
  hm_ctx& ctx = *c;
  hm_fe_info r{};
  hm_status st = guarded(c, [&] {
    HM_REQUIRE(fe && T_n && T_out, "hm_fe_step: NULL argument");
    HM_REQUIRE(fe_device(*fe) == ctx.device, "hm_fe_step: object and context on different devices");
    check_device_range(ctx, T_n, fe_nodes(*fe), fe_nodes(*fe), 1, 0.0, INFINITY, true, "hm_fe_step: T_n");
    if (f_facet)
      check_device_range(ctx, f_facet, fe_facets(*fe), fe_facets(*fe), 1, -INFINITY, INFINITY, false,
                         "hm_fe_step: f_facet");
    std::lock_guard<std::mutex> lk(const_cast<hm_matrix*>(fe_matrix(*fe))->mu);
    r = fe_step(ctx, *fe, T_n, f_facet, T_out);
  });
  if (info) *info = r;
  if (st == HM_OK && r.status != HM_OK) {
    ctx.last_error = "hm_fe_step: Newton did not reach newton_rtol";
    return HM_ENOTCONV;
  }
  return st;
}

void hm_fe_destroy(hm_fe* fe) {
  if (!fe) return;
  fe_destroy(fe);
}

hm_status hm_transient_run(hm_ctx* ctx, const hm_matrix* M, const double* eps, int32_t nrhs, double* T, int64_t ldT,
                           const double* src, int64_t ldS, double sigma, const hm_transient_params* tp,
                           const hm_solve_params* sp, double* history, hm_transient_info* info) {
  if (!ctx) {
    set_tl_error("hm_transient_run: NULL ctx");
    return HM_EINVAL;
  }
  bool nonfinite = false;
  hm_status st = guarded(ctx, [&] {
    const auto t0 = std::chrono::steady_clock::now();
    HM_REQUIRE(M && eps && T && src && tp, "hm_transient_run: NULL argument");
    HM_REQUIRE(nrhs >= 1 && nrhs <= 16, "hm_transient_run: nrhs must be in 1..16");
    HM_REQUIRE(ldT >= M->n && ldS >= M->n, "hm_transient_run: leading dimension < n");
    HM_REQUIRE(tp->mc > 0 && tp->dt > 0 && tp->steps >= 0 && tp->max_newton >= 1 && tp->newton_rtol > 0,
               "hm_transient_run: bad transient parameters");
    HM_REQUIRE(sigma > 0.0 && std::isfinite(sigma), "hm_transient_run: sigma must be > 0");
    check_params(sp);
    check_device_range(*ctx, eps, M->n, M->n, 1, 0.0, 1.0, true, "eps");
    check_device_range(*ctx, T, M->n, ldT, nrhs, 0.0, INFINITY, true, "T");
    std::lock_guard<std::mutex> lk(const_cast<hm_matrix*>(M)->mu);
    Batch& B = batch_for({M}, nrhs, ctx->stream);
    TransientResult R = B.transient({eps}, T, ldT, src, ldS, sigma, *tp, *sp, history, ctx->stream);
    if (info) {
      info->steps_done = R.steps_done;
      info->newton_total = R.newton_total;
      info->newton_max = R.newton_max;
      info->matvecs = R.matvecs;
      info->max_rel_residual = R.max_rel_residual;
      info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    nonfinite = R.nonfinite;
  });
  if (st == HM_OK && nonfinite) {
    ctx->last_error = "hm_transient_run: a Newton residual was not finite (the run stopped at that step)";
    return HM_ENOTCONV;
  }
  return st;
}

}  // extern "C"
