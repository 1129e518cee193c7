// Batched restarted GMRES (classical Gram-Schmidt with one re-orthogonalisation)
// for the radiosity system (I - diag(1 - eps) F) J = b of eq. (11).
// All systems of a batch advance in lockstep; a system leaves the cycle as
// soon as its residual estimate meets the tolerance, and an H-matrix slot is
// skipped once none of its systems is active.  Dot products and norms are
// accumulated in FP64 and reduced in a fixed order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <mutex>

#include "dev_common.hpp"
#include "convergence.hpp"
#include "krylov.hpp"

namespace hm {

void SysSet::build(const Composition& C, const std::vector<std::vector<int>>& cols_per_slot, hipStream_t s) {
  sys.clear();
  chunks.clear();
  nparts = 0;
  for (size_t q = 0; q < C.mats.size(); ++q) {
    for (int col : cols_per_slot[q]) {
      SysDev d{C.xoff[q], (int32_t)C.mats[q]->n, col, (int32_t)q, (int32_t)chunks.size()};
      const int32_t sid = (int32_t)sys.size();
      sys.push_back(d);
      // at most GS_ROWS rows a chunk, and at least GS_MIN_CHUNKS chunks of
      // at least 256 rows where the system has the rows: a small system's
      // vector kernels then run on more than a handful of workgroups (the
      // split depends on the system alone, so a batch member reduces in the
      // same order as the system solved alone)
      const int32_t nch = std::max<int32_t>((int32_t)((d.n + GS_ROWS - 1) / GS_ROWS),
                                            std::min<int32_t>(GS_MIN_CHUNKS, (int32_t)((d.n + 255) / 256)));
      for (int32_t c = 0; c < nch; ++c) {
        const int32_t r0 = (int32_t)((int64_t)d.n * c / nch);
        const int32_t r1 = (int32_t)((int64_t)d.n * (c + 1) / nch);
        chunks.push_back(ChunkDev{sid, r0, r1 - r0, nparts, c, nch});
      }
      nparts += nch;
    }
  }
  upload(d_sys, sys, s);
  upload(d_chunks, chunks, s);
}

void Krylov::drop_graphs() {
  for (auto& g : graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  graphs.clear();
}

Krylov::~Krylov() {
  drop_graphs();
  if (cap) (void)hipStreamDestroy(cap);
}

void Krylov::init(const Composition& Cm, SysSet& Ss, int vec_bytes, int restart, hipStream_t s) {
  HM_REQUIRE(restart >= 1 && restart <= MAXM, "gmres: restart must be in 1..64");
  drop_graphs();
  C = &Cm;
  S = &Ss;
  vb = vec_bytes;
  m = restart;
  ld = Cm.N;
  blk = ld * Cm.nr;
  const int ns = Ss.size();
  basis.alloc((size_t)(m + 1) * blk * vb);
  w.alloc((size_t)blk * vb);
  r.alloc((size_t)blk * vb);
  H.alloc((size_t)ns * MAXM * (MAXM + 1) * 8);
  cs.alloc((size_t)ns * MAXM * 8);
  sn.alloc((size_t)ns * MAXM * 8);
  hA.alloc((size_t)ns * (MAXM + 1) * 8);
  hB.alloc((size_t)ns * (MAXM + 1) * 8);
  hn.alloc((size_t)ns * 8);
  beta.alloc((size_t)ns * 8);
  const size_t nslots = std::max<size_t>(1, Cm.mats.size());
  xch_bytes = ((size_t)ns * (MAXM + 3)) * 8 + (((2 * (size_t)ns + nslots) * 4 + 7) & ~(size_t)7);
  xch.alloc(xch_bytes);
  const size_t hb = xch_bytes + (size_t)ns * 8;
  if (!xch_lease || xch_lease->bytes < hb) {
    xch_lease.reset();
    xch_lease = std::make_unique<PinnedLease>(hb);
  }
  xch_h = xch_lease->p;
  xch_hd = xch_lease->dev;
  g = xch.get<double>();
  tol = g + (size_t)ns * (MAXM + 1);
  bnorm = tol + ns;
  act = (int*)(bnorm + ns);
  steps = act + ns;
  slot_cnt = steps + ns;
  part.alloc((size_t)std::max(1, Ss.nparts) * (MAXM + 1) * 8);
  cnt.alloc((size_t)ns * 4);
  HM_HIP(hipMemsetAsync(cnt.get(), 0, cnt.bytes(), s));
  HM_HIP(hipMemsetAsync(basis.get(), 0, basis.bytes(), s));
  HM_HIP(hipMemsetAsync(w.get(), 0, w.bytes(), s));
  HM_HIP(hipMemsetAsync(r.get(), 0, r.bytes(), s));
}

// ------------------------------------------------------------------ kernels
struct GsArgs {
  const SysDev* sys;
  const ChunkDev* chunks;
  int mode;        // 0 dots, 1 update(hA)+dots, 2 update(hB)+norm+Givens, 3 norm -> beta
  int cgs1;        // mode 2 updates with hA (no mode 1 ran: one pass)
  int j;           // Arnoldi step
  void* w;         // vector block being orthogonalised / normed
  const void* basis;
  int64_t ld, blk;
  double* hA;
  double* hB;
  double* H;
  double* cs;
  double* sn;
  double* g;
  double* hn;
  double* beta;
  const double* tol;
  int* act;
  int* steps;
  int* slot_cnt;
  double* part;
  unsigned* cnt;
};

template <class VT>
__global__ __launch_bounds__(GS_T) void k_gs(GsArgs a) {
  __shared__ double coef[MAXM + 1];
  __shared__ double red[GS_T / 64][MAXM + 2];
  const ChunkDev c = a.chunks[blockIdx.x];
  const int s = c.sys;
  if (a.mode != 3 && !a.act[s]) return;
  const SysDev sy = a.sys[s];
  const int64_t base = (int64_t)sy.col * a.ld + sy.row0 + c.r0;
  VT* w = (VT*)a.w + base;
  const VT* Vb = (const VT*)a.basis + base;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int L = (a.mode <= 1) ? a.j + 1 : 0;
  if (a.mode == 1 || a.mode == 2) {
    const double* src = (a.mode == 1 || a.cgs1) ? a.hA : a.hB;
    for (int l = tid; l <= a.j; l += GS_T) coef[l] = src[(int64_t)s * (MAXM + 1) + l];
    __syncthreads();
  }
  double wv[GS_RPT];
#pragma unroll
  for (int q = 0; q < GS_RPT; ++q) {
    const int r = tid + q * GS_T;
    wv[q] = r < c.nr ? (double)w[r] : 0.0;
  }
  if (a.mode == 1 || a.mode == 2) {
    for (int l = 0; l <= a.j; ++l) {
      const double cl = coef[l];
      const VT* v = Vb + (int64_t)l * a.blk;
#pragma unroll
      for (int q = 0; q < GS_RPT; ++q) {
        const int r = tid + q * GS_T;
        if (r < c.nr) wv[q] -= cl * (double)v[r];
      }
    }
#pragma unroll
    for (int q = 0; q < GS_RPT; ++q) {
      const int r = tid + q * GS_T;
      if (r < c.nr) {
        w[r] = (VT)wv[q];
        wv[q] = (double)(VT)wv[q];  // continue with the stored value
      }
    }
  }
  // partial sums: L dot products, or one squared norm
  const int nv = L > 0 ? L : 1;
  for (int l = 0; l < nv; ++l) {
    double d = 0.0;
    if (L > 0) {
      const VT* v = Vb + (int64_t)l * a.blk;
#pragma unroll
      for (int q = 0; q < GS_RPT; ++q) {
        const int r = tid + q * GS_T;
        if (r < c.nr) d += (double)v[r] * wv[q];
      }
    } else {
#pragma unroll
      for (int q = 0; q < GS_RPT; ++q) d += wv[q] * wv[q];
    }
    d = wave_sum(d);
    if (lane == 0) red[wid][l] = d;
  }
  __syncthreads();
  double* P0 = a.part + (int64_t)c.part * (MAXM + 1);
  if (tid < nv) {
    double t = red[0][tid];
    for (int q = 1; q < GS_T / 64; ++q) t += red[q][tid];
    P0[(int64_t)c.pidx * (MAXM + 1) + tid] = t;
  }
}

// One wave per system: the chunk partials of k_gs added in a fixed order
// (lane i sums partials i, i + 64, ..., then a fixed butterfly over the
// lanes; the order depends only on the system's own partial count), then the
// step's bookkeeping (Hessenberg entries, norm, Givens rotation).
__global__ __launch_bounds__(64) void k_gs_final(GsArgs a, int nsys) {
  __shared__ double red[MAXM + 1];
  const int s = blockIdx.x;
  if (s >= nsys) return;
  if (a.mode != 3 && !a.act[s]) return;
  const SysDev sy = a.sys[s];
  const ChunkDev c0 = a.chunks[sy.chunk0];
  const int L = (a.mode <= 1) ? a.j + 1 : 0;
  const int nv = L > 0 ? L : 1;
  const double* P0 = a.part + (int64_t)c0.part * (MAXM + 1);
  for (int l = 0; l < nv; ++l) {
    double t = 0.0;
    for (int p = threadIdx.x; p < c0.nparts; p += 64) t += P0[(int64_t)p * (MAXM + 1) + l];
    t = wave_sum(t);
    if (threadIdx.x == 0) red[l] = t;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double* hs = a.mode == 0 ? a.hA : a.hB;
  if (a.mode <= 1) {
    for (int l = 0; l < L; ++l) hs[(int64_t)s * (MAXM + 1) + l] = red[l];
  } else if (a.mode == 3) {
    a.beta[s] = sqrt(red[0]);
  } else {
    // finish column j of the Hessenberg matrix and its Givens rotation
    const int j = a.j;
    const double hnrm = sqrt(red[0]);
    double col[MAXM + 1];
    for (int i = 0; i <= j; ++i)
      col[i] = a.hA[(int64_t)s * (MAXM + 1) + i] + (a.cgs1 ? 0.0 : a.hB[(int64_t)s * (MAXM + 1) + i]);
    col[j + 1] = hnrm;
    double* cs = a.cs + (int64_t)s * MAXM;
    double* sn = a.sn + (int64_t)s * MAXM;
    for (int i = 0; i < j; ++i) {
      const double t0 = cs[i] * col[i] + sn[i] * col[i + 1];
      col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
      col[i] = t0;
    }
    const double x0 = col[j], x1 = col[j + 1];
    const double rr = hypot(x0, x1);
    double cj = 1.0, sj = 0.0;
    if (rr > 0.0) {
      cj = x0 / rr;
      sj = x1 / rr;
    }
    col[j] = rr;
    col[j + 1] = 0.0;
    cs[j] = cj;
    sn[j] = sj;
    double* gs = a.g + (int64_t)s * (MAXM + 1);
    const double gj = gs[j];
    gs[j] = cj * gj;
    gs[j + 1] = -sj * gj;
    double* Hc = a.H + ((int64_t)s * MAXM + j) * (MAXM + 1);
    for (int i = 0; i <= j + 1; ++i) Hc[i] = col[i];
    a.steps[s] = j + 1;
    a.hn[s] = hnrm;
    const double res = fabs(gs[j + 1]);
    if (res <= a.tol[s] || !(hnrm > 0.0) || rr == 0.0) {
      a.act[s] = 0;
      atomicSub(&a.slot_cnt[sy.slot], 1);
    }
  }
}

// dst = src / div[s] on the active systems (div = hn or beta).
template <class VT>
__global__ __launch_bounds__(GS_T) void k_scale(const SysDev* __restrict__ sys, const ChunkDev* __restrict__ chunks,
                                                const int* __restrict__ act, const double* __restrict__ div,
                                                const VT* __restrict__ src, VT* __restrict__ dst, int64_t ld) {
  const ChunkDev c = chunks[blockIdx.x];
  if (!act[c.sys]) return;
  const SysDev sy = sys[c.sys];
  const int64_t base = (int64_t)sy.col * ld + sy.row0 + c.r0;
  const double inv = 1.0 / div[c.sys];
  for (int r = threadIdx.x; r < c.nr; r += GS_T) dst[base + r] = (VT)((double)src[base + r] * inv);
}

// x += V y with H(0:k,0:k) y = g(0:k) (k = steps of the system).  With
// when_done (the slot counts, launched at the end of a block of Arnoldi
// steps) only once no system is left active, else nothing: the cycle's
// update then needs no host round trip.
template <class VT>
__global__ __launch_bounds__(GS_T) void k_xupdate(const SysDev* __restrict__ sys, const ChunkDev* __restrict__ chunks,
                                                  const int* __restrict__ steps, const double* __restrict__ H,
                                                  const double* __restrict__ g, const VT* __restrict__ basis,
                                                  int64_t ld, int64_t blk, VT* __restrict__ x,
                                                  const int* __restrict__ when_done, int nslots) {
  __shared__ double y[MAXM];
  __shared__ int left;
  if (when_done) {
    if (threadIdx.x == 0) {
      int t = 0;
      for (int q = 0; q < nslots; ++q) t += when_done[q];
      left = t;
    }
    __syncthreads();
    if (left) return;  // uniform over the workgroup
  }
  const ChunkDev c = chunks[blockIdx.x];
  const int s = c.sys;
  const int k = steps[s];
  if (k <= 0) return;
  if (threadIdx.x == 0) {
    const double* gs = g + (int64_t)s * (MAXM + 1);
    for (int i = k - 1; i >= 0; --i) {
      double t = gs[i];
      for (int l = i + 1; l < k; ++l) t -= H[((int64_t)s * MAXM + l) * (MAXM + 1) + i] * y[l];
      y[i] = t / H[((int64_t)s * MAXM + i) * (MAXM + 1) + i];
    }
  }
  __syncthreads();
  const SysDev sy = sys[s];
  const int64_t base = (int64_t)sy.col * ld + sy.row0 + c.r0;
  for (int r = threadIdx.x; r < c.nr; r += GS_T) {
    double acc = (double)x[base + r];
    for (int l = 0; l < k; ++l) acc += (double)basis[(int64_t)l * blk + base + r] * y[l];
    x[base + r] = (VT)acc;
  }
}

// ------------------------------------------------------------------ pinned leases
namespace {
std::mutex& lease_mu() {
  static std::mutex* m = new std::mutex();
  return *m;
}
struct FreeLease {
  void* p;
  void* dev;
  size_t bytes;
};
std::vector<FreeLease>& lease_free() {
  static auto* v = new std::vector<FreeLease>();
  return *v;
}
}  // namespace

PinnedLease::PinnedLease(size_t need) {
  {
    std::lock_guard<std::mutex> lk(lease_mu());
    auto& fl = lease_free();
    for (size_t i = 0; i < fl.size(); ++i)
      if (fl[i].bytes >= need) {
        p = fl[i].p;
        dev = fl[i].dev;
        bytes = fl[i].bytes;
        fl.erase(fl.begin() + (std::ptrdiff_t)i);
        return;
      }
  }
  size_t b = 4096;
  while (b < need) b <<= 1;
  p = pinned_alloc(b, &dev);
  bytes = b;
}

void* pinned_alloc(size_t bytes, void** dev) {
  void* p = nullptr;
  HM_HIP(hipHostMalloc(&p, bytes, hipHostMallocMapped | hipHostMallocCoherent));
  std::memset(p, 0, bytes);
  if (dev) HM_HIP(hipHostGetDevicePointer(dev, p, 0));
  return p;
}

__global__ void k_words(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

void copy_small(const void* src, void* dst, size_t bytes, hipStream_t s) {
  HM_REQUIRE(bytes % 8 == 0 && (uintptr_t)src % 8 == 0 && (uintptr_t)dst % 8 == 0, "copy_small: misaligned copy");
  const int64_t n = (int64_t)(bytes / 8);
  if (n == 0) return;
  const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 64);
  hipLaunchKernelGGL(k_words, dim3(nb), dim3(256), 0, s, (const uint64_t*)src, (uint64_t*)dst, n);
  HM_HIP(hipGetLastError());
}

PinnedLease::~PinnedLease() {
  if (std::uncaught_exceptions() > 0) return;
  std::lock_guard<std::mutex> lk(lease_mu());
  lease_free().push_back(FreeLease{p, dev, bytes});
}

// ------------------------------------------------------------------ driver
namespace {

GsArgs gs_args(Krylov& K, int mode, int j, void* wvec, bool cgs1 = false) {
  GsArgs a;
  a.cgs1 = cgs1 ? 1 : 0;
  a.sys = K.S->d_sys.get<SysDev>();
  a.chunks = K.S->d_chunks.get<ChunkDev>();
  a.mode = mode;
  a.j = j;
  a.w = wvec;
  a.basis = K.basis.get();
  a.ld = K.ld;
  a.blk = K.blk;
  a.hA = K.hA.get<double>();
  a.hB = K.hB.get<double>();
  a.H = K.H.get<double>();
  a.cs = K.cs.get<double>();
  a.sn = K.sn.get<double>();
  a.g = K.g;
  a.hn = K.hn.get<double>();
  a.beta = K.beta.get<double>();
  a.tol = K.tol;
  a.act = K.act;
  a.steps = K.steps;
  a.slot_cnt = K.slot_cnt;
  a.part = K.part.get<double>();
  a.cnt = K.cnt.get<unsigned>();
  return a;
}

template <class VT>
void run_gs(Krylov& K, int mode, int j, void* wvec, hipStream_t s, bool cgs1 = false) {
  const unsigned nb = (unsigned)K.S->chunks.size();
  if (nb == 0) return;
  const GsArgs a = gs_args(K, mode, j, wvec, cgs1);
  hipLaunchKernelGGL(k_gs<VT>, dim3(nb), dim3(GS_T), 0, s, a);
  hipLaunchKernelGGL(k_gs_final, dim3((unsigned)K.S->size()), dim3(64), 0, s, a, K.S->size());
  HM_HIP(hipGetLastError());
}

template <class VT>
void run_scale(Krylov& K, const double* div, const void* src, void* dst, hipStream_t s) {
  const unsigned nb = (unsigned)K.S->chunks.size();
  hipLaunchKernelGGL(k_scale<VT>, dim3(nb), dim3(GS_T), 0, s, K.S->d_sys.get<SysDev>(),
                     K.S->d_chunks.get<ChunkDev>(), K.act, div, (const VT*)src, (VT*)dst, K.ld);
  HM_HIP(hipGetLastError());
}

// The graph of a block of Arnoldi steps j0 .. j0 + nsteps - 1 for these
// arguments (body(j0, nsteps, stream) launches it), captured on the
// workspace's private stream at first use; nullptr when capture is not
// possible (the caller then launches the block directly).
template <class F>
hipGraphExec_t block_graph(Krylov& K, bool hi, bool cgs1, const void* omeps, const void* x, int nrr, int j0,
                           int nsteps, F&& body) {
  for (const auto& g : K.graphs)
    if (g.hi == hi && g.cgs1 == cgs1 && g.omeps == omeps && g.x == x && g.nrr == nrr && g.j0 == j0 &&
        g.nsteps == nsteps)
      return g.exec;
  if (!K.cap && hipStreamCreateWithFlags(&K.cap, hipStreamNonBlocking) != hipSuccess) {
    K.cap = nullptr;
    return nullptr;
  }
  if (hipStreamBeginCapture(K.cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
  bool ok = true;
  try {
    body(j0, nsteps, K.cap);
  } catch (const Error&) {
    ok = false;
  }
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(K.cap, &g) != hipSuccess || !g) ok = false;
  hipGraphExec_t ge = nullptr;
  if (ok && hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) ge = nullptr;
  if (g) (void)hipGraphDestroy(g);
  (void)hipGetLastError();
  if (!ge) return nullptr;
  StepGraph sg;
  sg.hi = hi;
  sg.cgs1 = cgs1;
  sg.omeps = omeps;
  sg.x = x;
  sg.nrr = nrr;
  sg.j0 = j0;
  sg.nsteps = nsteps;
  sg.exec = ge;
  K.graphs.push_back(sg);
  return ge;
}

template <class VT>
GmresStats gmres_t(Krylov& K, bool hi, const void* omeps, const void* b, void* x, double rtol, int max_iter,
                   hipStream_t s, bool use_graphs, unsigned opts, const double* bnorm_in) {
  const Composition& C = *K.C;
  const int ns = K.S->size();
  const int nslots = (int)C.mats.size();
  GmresStats st;
  st.rel_res.assign(ns, 0.0);
  const int64_t mbytes = hi ? C.bytes_hi : C.bytes_lo;
  // host side of the exchange block (same layout as K.xch), then the
  // residual norms read back after a product
  const size_t g0n = (size_t)ns * (MAXM + 1);
  double* g0 = (double*)K.xch_h;
  double* tolv = g0 + g0n;
  double* bn = tolv + ns;
  int* act = (int*)(bn + ns);
  int* stp = act + ns;
  int* cnt = stp + ns;
  double* beta = (double*)((char*)K.xch_h + K.xch_bytes);
  void* beta_d = (char*)K.xch_hd + K.xch_bytes;  // its device view
  std::memset(K.xch_h, 0, K.xch_bytes);
  // |b| per system
  if (bnorm_in) {
    std::copy(bnorm_in, bnorm_in + ns, bn);
  } else {
    run_gs<VT>(K, 3, 0, const_cast<void*>(b), s);
    copy_small(K.beta.get(), beta_d, (size_t)ns * 8, s);
    HM_HIP(hipStreamSynchronize(s));
    std::copy(beta, beta + ns, bn);
  }
  for (int q = 0; q < ns; ++q) tolv[q] = rtol * bn[q];
  Epilogue res_ep;  // r = b - (x - (1-eps) F x) = b - x + (1-eps) F x
  res_ep.rowscale = omeps;
  res_ep.a_acc = 1.0;
  res_ep.a_x = -1.0;
  res_ep.a_z = 1.0;
  res_ep.z = b;
  res_ep.ldz = K.ld;
  Epilogue op_ep;   // w = v - (1-eps) F v
  op_ep.rowscale = omeps;
  op_ep.a_acc = -1.0;
  op_ep.a_x = 1.0;
  const int nrr = C.nr;
  const bool cgs1 = (opts & GM_CGS1) != 0;
  int iters = 0;
  bool first = true;
  for (;;) {
    // true residual and its norm (b itself for a zero start: its norms are
    // bn, and the first basis vector is b / bn)
    const bool from_b = first && (opts & GM_X0_ZERO);
    if (from_b) {
      std::copy(bn, bn + ns, beta);
    } else {
      launch_matvec(C, nrr, K.vb, hi, x, K.ld, K.basis.get(), K.ld, res_ep, nullptr, s);
      st.matvecs++;
      st.bytes += mbytes;
      run_gs<VT>(K, 3, 0, K.basis.get(), s);
      copy_small(K.beta.get(), beta_d, (size_t)ns * 8, s);
      HM_HIP(hipStreamSynchronize(s));
    }
    first = false;
    int nact = 0;
    std::fill(cnt, cnt + nslots, 0);
    for (int q = 0; q < ns; ++q) {
      st.rel_res[q] = rel_residual(beta[q], bn[q]);
      // a system whose residual is not finite stops (and fails the solve)
      const bool finite = std::isfinite(beta[q]) && std::isfinite(bn[q]);
      if (!finite) st.converged = false;
      act[q] = finite && beta[q] > tolv[q] ? 1 : 0;
      if (act[q]) {
        ++nact;
        cnt[K.S->sys[q].slot]++;
      }
      g0[(size_t)q * (MAXM + 1)] = finite ? beta[q] : 0.0;
      stp[q] = 0;
    }
    if (nact == 0) break;
    if (iters >= max_iter) {
      st.converged = false;
      break;
    }
    // one copy: g (first entries), tol, |b|, active flags, step counts, slot counts
    copy_small(K.xch_hd, K.xch.get(), K.xch_bytes, s);
    if (from_b)
      run_scale<VT>(K, K.bnorm, b, K.basis.get(), s);
    else
      run_scale<VT>(K, K.beta.get<double>(), K.basis.get(), K.basis.get(), s);
    // one Arnoldi step on stream st (kernels only)
    auto step = [&](int j, hipStream_t st) {
      char* vj = K.basis.get<char>() + (size_t)j * K.blk * K.vb;
      char* vj1 = vj + (size_t)K.blk * K.vb;
      launch_matvec(C, nrr, K.vb, hi, vj, K.ld, K.w.get(), K.ld, op_ep, K.slot_cnt, st);
      run_gs<VT>(K, 0, j, K.w.get(), st);
      if (!cgs1) run_gs<VT>(K, 1, j, K.w.get(), st);
      run_gs<VT>(K, 2, j, K.w.get(), st, cgs1);
      run_scale<VT>(K, K.hn.get<double>(), K.w.get(), vj1, st);
    };
    // blocks of up to SYNC Arnoldi steps; after each the host reads the
    // whole exchange block back (the active counts decide whether to go on;
    // the step counts and the rotated right-hand sides are then at hand).
    // Steps launched after every system has converged find nothing active
    // and return at once; a block that ends with none active also applies
    // the update x += V y on the device.
    constexpr int SYNC = 4;
    const unsigned nchunks = (unsigned)K.S->chunks.size();
    auto update = [&](hipStream_t st, const int* when_done) {
      hipLaunchKernelGGL(k_xupdate<VT>, dim3(nchunks), dim3(GS_T), 0, st, K.S->d_sys.get<SysDev>(),
                         K.S->d_chunks.get<ChunkDev>(), K.steps, K.H.get<double>(), K.g,
                         (const VT*)K.basis.get(), K.ld, K.blk, (VT*)x, when_done, nslots);
      HM_HIP(hipGetLastError());
    };
    auto block = [&](int j0, int nsteps, hipStream_t st) {
      for (int q = 0; q < nsteps; ++q) step(j0 + q, st);
      update(st, K.slot_cnt);
      copy_small(K.xch.get(), K.xch_hd, K.xch_bytes, st);
    };
    int left = nact;
    for (int j = 0; j < K.m && iters + j < max_iter;) {
      const int nb = std::min(SYNC, std::min(K.m - j, max_iter - iters - j));
      hipGraphExec_t ge = use_graphs ? block_graph(K, hi, cgs1, omeps, x, nrr, j, nb, block) : nullptr;
      if (ge)
        HM_HIP(hipGraphLaunch(ge, s));
      else
        block(j, nb, s);
      j += nb;
      HM_HIP(hipStreamSynchronize(s));
      left = 0;
      for (int q = 0; q < nslots; ++q) left += cnt[q];
      if (left == 0) break;
    }
    // steps taken in this cycle: the most any system took
    const bool trusted = (opts & GM_TRUST_ESTIMATE) && left == 0;
    const int cyc = *std::max_element(stp, stp + ns);
    iters += cyc;
    st.matvecs += cyc;
    st.bytes += (int64_t)cyc * mbytes;
    // a cycle that ended with systems still active (restart or iteration
    // cap) applies its update here; otherwise the last block did
    if (left > 0) update(s, nullptr);
    if (trusted) {
      // every system met the tolerance by its residual estimate
      for (int q = 0; q < ns; ++q) {
        st.rel_res[q] = rel_residual(std::fabs(g0[(size_t)q * (MAXM + 1) + stp[q]]), bn[q]);
        if (std::isnan(st.rel_res[q])) st.converged = false;
      }
      break;
    }
  }
  st.iters = iters;
  return st;
}

}  // namespace

GmresStats gmres(Krylov& K, bool hi, const void* omeps, const void* b, void* x, double rtol, int max_iter,
                 hipStream_t s, bool graphs, unsigned opts, const double* bnorm) {
  if (K.vb == 8) return gmres_t<double>(K, hi, omeps, b, x, rtol, max_iter, s, graphs, opts, bnorm);
  return gmres_t<float>(K, hi, omeps, b, x, rtol, max_iter, s, graphs, opts, bnorm);
}

void block_norms(Krylov& K, const void* v, std::vector<double>& out, hipStream_t s) {
  if (K.vb == 8) run_gs<double>(K, 3, 0, const_cast<void*>(v), s);
  else run_gs<float>(K, 3, 0, const_cast<void*>(v), s);
  const int ns = K.S->size();
  // the norms come back through the workspace's pinned block (no gmres is
  // running on this workspace meanwhile)
  copy_small(K.beta.get(), (char*)K.xch_hd + K.xch_bytes, (size_t)ns * 8, s);
  HM_HIP(hipStreamSynchronize(s));
  const double* nr = (const double*)((const char*)K.xch_h + K.xch_bytes);
  out.assign(nr, nr + ns);
}

}  // namespace hm
