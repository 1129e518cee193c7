// Radiosity solves on top of the batched H-matrix product and GMRES:
// right-hand side sigma eps T^4 (eq. (4)), reflection operator of eq. (11),
// facet flux of eq. (12), optional mixed-precision iterative refinement and
// the lumped implicit-Euler transient (analogue of Sec. 3.3).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>

#include "convergence.hpp"
#include "dev_common.hpp"
#include "krylov.hpp"
#include "solve.hpp"

namespace hm {

// ------------------------------------------------------------------ kernels
__device__ inline int io_slot(const SlotIO* __restrict__ io, int ns, int64_t row) {
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (io[mid].xoff <= row) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// dst[row + j*N] = in_slot[perm[i] + j*ld] (permuted copy), j < ncol; 0 for j >= ncol_slot
__global__ void k_gather(const SlotIO* __restrict__ io, int ns, int64_t N, int ncol, double* __restrict__ dst) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (row >= N) return;
  const SlotIO s = io[io_slot(io, ns, row)];
  const int64_t i = row - s.xoff;
  dst[row + j * N] = (j < ncol && s.in) ? s.in[s.perm[i] + j * s.ld] : 0.0;
}

__global__ void k_scatter(const SlotIO* __restrict__ io, int ns, int64_t N, int ncol, const double* __restrict__ src) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (row >= N || j >= ncol) return;
  const SlotIO s = io[io_slot(io, ns, row)];
  if (!s.out) return;
  const int64_t i = row - s.xoff;
  s.out[s.perm[i] + j * s.ld] = src[row + j * N];
}

// b = sigma eps T^4 and its cast; zero in padded columns
template <class VT>
__global__ void k_rhs(const double* __restrict__ eps, const double* __restrict__ T, int64_t N, int ncol,
                      double sigma, double* __restrict__ b64, VT* __restrict__ bv, int power) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (row >= N) return;
  const int64_t k = row + j * N;
  double v = 0.0;
  if (j < ncol) {
    const double t = T[k];
    const double t2 = t * t;
    v = sigma * eps[row] * (power ? t : t2 * t2);
  }
  if (b64) b64[k] = v;
  if (bv) bv[k] = (VT)v;
}

template <class VT>
__global__ void k_omeps(const double* __restrict__ eps, int64_t N, VT* __restrict__ out) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row < N) out[row] = (VT)(1.0 - eps[row]);
}

template <class A, class B>
__global__ void k_cast(const A* __restrict__ a, B* __restrict__ b, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) b[k] = (B)a[k];
}

// Right-hand side of an inner correction solve from the FP64 residual src:
// b32 = (float) src and x32 = 0; with rcopy, also rcopy = src (the residual
// of a zero start is b itself).
__global__ void k_inner_rhs(const double* __restrict__ src, float* __restrict__ b32, float* __restrict__ x32,
                            double* __restrict__ rcopy, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double v = src[k];
  b32[k] = (float)v;
  x32[k] = 0.f;
  if (rcopy) rcopy[k] = v;
}

// b32 = 0 on the systems whose flag is 0 (those already converged take no
// correction); one workgroup per reduction chunk of a system.
__global__ void k_zero_done(const SysDev* __restrict__ sys, const ChunkDev* __restrict__ chunks,
                            const int* __restrict__ on, float* __restrict__ b32, int64_t ld) {
  const ChunkDev c = chunks[blockIdx.x];
  if (on[c.sys]) return;
  const SysDev sy = sys[c.sys];
  const int64_t base = (int64_t)sy.col * ld + sy.row0 + c.r0;
  for (int r = threadIdx.x; r < c.nr; r += blockDim.x) b32[base + r] = 0.f;
}

// y += (double) x
template <class VT>
__global__ void k_acc(const VT* __restrict__ x, double* __restrict__ y, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) y[k] += (double)x[k];
}

// q = eps (H - sigma T^4 g)  (eq. (12) through J and g = F C^-1 eps); for an
// open cavity (amb != NULL) plus the ambient exchange of eq. (35),
// -sigma (1 - c) (T^4 - T_amb^4) with amb = 1 - c
__global__ void k_flux(const double* __restrict__ eps, const double* __restrict__ T, const double* __restrict__ H,
                       const double* __restrict__ g, int64_t N, int ncol, double sigma, double* __restrict__ q,
                       const double* __restrict__ amb, double tamb4, int power) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (row >= N || j >= ncol) return;
  const int64_t k = row + j * N;
  const double t = T[k];
  const double t2 = t * t;
  const double e = power ? t : t2 * t2;  // radiation power eta
  double v = eps[row] * (H[k] - sigma * e * g[row]);
  if (amb) v = v - sigma * amb[row] * (e - tamb4);
  q[k] = v;
}

// amb = 1 - clamp(s, 0, 1) for the row sums s = F 1 (eqs. (32)-(33))
__global__ void k_ambient(const double* __restrict__ rowsum, int64_t N, double* __restrict__ amb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double c = fmin(fmax(rowsum[i], 0.0), 1.0);
  amb[i] = 1.0 - c;
}

__global__ void k_fill(double* __restrict__ x, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

// Newton residual R = mc (T - Tn)/dt - q - s, and the update T <- T - R / D
// with D = mc/dt + 4 sigma eps g T^3 (mode 1), or only R (mode 0).
// (open cavity: D also holds the ambient term's 4 sigma (1 - c) T^3)
__global__ void k_newton(const double* __restrict__ eps, const double* __restrict__ g, const double* __restrict__ q,
                         const double* __restrict__ src, const double* __restrict__ Tn, double* __restrict__ T,
                         double* __restrict__ R, int64_t N, int ncol, double mc, double dt, double sigma,
                         const int* __restrict__ upd, const double* __restrict__ amb) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (row >= N || j >= ncol) return;
  const int64_t k = row + j * N;
  const double t = T[k];
  const double r = mc * (t - Tn[k]) / dt - q[k] - src[k];
  R[k] = r;
  if (upd && upd[j]) {
    const double a = eps[row] * g[row] + (amb ? amb[row] : 0.0);
    const double D = mc / dt + 4.0 * sigma * a * (t * t * t);
    T[k] = t - r / D;
  }
}

__global__ void k_differs(const double* __restrict__ a, const double* __restrict__ b, int64_t n, int* flag) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n && a[k] != b[k]) atomicOr(flag, 1);
}

namespace {

dim3 grid_rows(int64_t N, int cols = 1) { return dim3((unsigned)((N + 255) / 256), (unsigned)cols); }

}  // namespace

// ------------------------------------------------------------------ batch state
Batch::Batch(const std::vector<const hm_matrix*>& m, int nrhs_, hipStream_t s) : mats(m), nrhs(nrhs_) {
  W = pad_width(nrhs);
  C = make_composition(mats, W, 8, s);
  N = C->N;
  std::vector<std::vector<int>> cols(mats.size());
  for (auto& c : cols)
    for (int j = 0; j < nrhs; ++j) c.push_back(j);
  S.build(*C, cols, s);
  const size_t vb = (size_t)N * W * 8;
  Tp.alloc(vb);
  b64.alloc(vb);
  x64.alloc(vb);
  r64.alloc(vb);
  H64.alloc(vb);
  epsp.alloc(N * 8);
  omeps64.alloc(N * 8);
  HM_HIP(hipMemsetAsync(Tp.get(), 0, vb, s));
  HM_HIP(hipMemsetAsync(x64.get(), 0, vb, s));
  HM_HIP(hipMemsetAsync(r64.get(), 0, vb, s));
  for (const auto* M : mats) {
    SlotIO io{};
    io.perm = M->d_perm.get<int32_t>();
    io.n = M->n;
    ios.push_back(io);
  }
  int64_t off = 0;
  for (auto& io : ios) {
    io.xoff = off;
    off += io.n;
  }
  d_ios.alloc((size_t)IO_ROLES * ios.size() * sizeof(SlotIO));
}

Krylov& Batch::krylov(int vb, int restart, hipStream_t s) {
  Krylov& K = vb == 8 ? K64 : K32;
  bool& ok = vb == 8 ? k64 : k32;
  if (!ok || K.m != restart) {
    if (vb == 4 && !b32.get()) {
      const size_t by = (size_t)N * W * 4;
      b32.alloc(by);
      x32.alloc(by);
      omeps32.alloc(N * 4);
      HM_HIP(hipMemsetAsync(x32.get(), 0, by, s));
    }
    K.init(*C, S, vb, restart, s);
    ok = true;
  }
  return K;
}

Batch::~Batch() {
  for (hipEvent_t& e : io_ev)
    if (e) {
      (void)hipEventSynchronize(e);
      (void)hipEventDestroy(e);
    }
  if (eps_ev) {
    (void)hipEventSynchronize(eps_ev);
    (void)hipEventDestroy(eps_ev);
  }
  // the pinned tables go back to the pool: every upload from them and the
  // flag's read-back have completed (the events above)
}

void Batch::io(int role, const std::vector<const double*>& in, const std::vector<double*>& out,
               int64_t ld_in_default, const std::vector<int64_t>* lds, hipStream_t s) {
  HM_REQUIRE(role >= 0 && role < IO_ROLES, "batch: bad io role");
  const size_t ns = ios.size();
  static_assert(sizeof(SlotIO) % 8 == 0, "slot tables are copied in 8-byte words");
  if (!ios_lease) {
    ios_lease = std::make_unique<PinnedLease>((size_t)IO_ROLES * ns * sizeof(SlotIO));
    ios_h = (SlotIO*)ios_lease->p;
    ios_hd = (SlotIO*)ios_lease->dev;
  }
  if (io_ev[role])
    HM_HIP(hipEventSynchronize(io_ev[role]));  // the previous upload of this table has read it
  else
    HM_HIP(hipEventCreateWithFlags(&io_ev[role], hipEventDisableTiming));
  SlotIO* t = ios_h + (size_t)role * ns;
  for (size_t q = 0; q < ns; ++q) {
    t[q] = ios[q];
    t[q].in = q < in.size() ? in[q] : nullptr;
    t[q].out = q < out.size() ? out[q] : nullptr;
    t[q].ld = lds ? (*lds)[q] : (ld_in_default > 0 ? ld_in_default : ios[q].n);
  }
  copy_small(ios_hd + (size_t)role * ns, d_ios.get<SlotIO>() + (size_t)role * ns, ns * sizeof(SlotIO), s);
  HM_HIP(hipEventRecord(io_ev[role], s));
}

void Batch::gather(int role, double* dst, int ncol, int dst_cols, hipStream_t s) {
  // dst holds dst_cols columns of N rows: columns ncol..dst_cols-1 are zeroed
  HM_REQUIRE(ncol >= 1 && ncol <= dst_cols && dst_cols <= W, "gather: bad column counts");
  hipLaunchKernelGGL(k_gather, grid_rows(N, dst_cols), dim3(256), 0, s, d_ios.get<SlotIO>() + (size_t)role * ios.size(),
                     (int)ios.size(), N, ncol, dst);
  HM_HIP(hipGetLastError());
}

void Batch::scatter(int role, const double* src, int ncol, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter, grid_rows(N, ncol), dim3(256), 0, s, d_ios.get<SlotIO>() + (size_t)role * ios.size(),
                     (int)ios.size(), N, ncol, src);
  HM_HIP(hipGetLastError());
}

// g = F C^-1 eps per slot (the flux helper of eq. (12)); FP64 vectors with
// the most accurate stored factors, solved to 1e-13.
void Batch::compare_eps(hipStream_t s) {
  eps_pending = false;
  if (!g_ready) return;
  if (!eps_lease) {
    eps_lease = std::make_unique<PinnedLease>(64);
    eps_flag_h = (int*)eps_lease->p;
    eps_flag_hd = eps_lease->dev;
  }
  if (!eps_ev) HM_HIP(hipEventCreateWithFlags(&eps_ev, hipEventDisableTiming));
  HM_HIP(hipMemsetAsync(d_flag.get(), 0, 8, s));
  hipLaunchKernelGGL(k_differs, grid_rows(N), dim3(256), 0, s, epsp.get<double>(), g_eps.get<double>(), N,
                     d_flag.get<int>());
  copy_small(d_flag.get(), eps_flag_hd, 8, s);
  HM_HIP(hipEventRecord(eps_ev, s));
  eps_pending = true;
}

void Batch::ensure_g(const std::vector<const double*>& eps_user, hipStream_t s) {
  // epsp holds the permuted emissivities of this call; g is reused while they are unchanged
  if (g_ready) {
    if (!eps_pending) compare_eps(s);
    HM_HIP(hipEventSynchronize(eps_ev));
    eps_pending = false;
    if (!*eps_flag_h) return;
  }
  if (!gb) gb = std::make_unique<Batch>(mats, 1, s);
  Batch& B = *gb;
  B.io(IO_EPS, eps_user, {}, 0, nullptr, s);
  B.gather(IO_EPS, B.epsp.get<double>(), 1, 1, s);
  hipLaunchKernelGGL(k_omeps<double>, grid_rows(B.N), dim3(256), 0, s, B.epsp.get<double>(), B.N,
                     B.omeps64.get<double>());
  HM_HIP(hipMemcpyAsync(B.b64.get(), B.epsp.get(), B.N * 8, hipMemcpyDeviceToDevice, s));
  HM_HIP(hipMemcpyAsync(B.x64.get(), B.epsp.get(), B.N * 8, hipMemcpyDeviceToDevice, s));
  Krylov& K = B.krylov(8, 30, s);
  GmresStats st = gmres(K, true, B.omeps64.get(), B.b64.get(), B.x64.get(), 1e-13, 2000, s);
  (void)st;
  if (!g.get()) g.alloc(N * 8);
  if (!g_eps.get()) g_eps.alloc(N * 8);
  if (!d_flag.get()) d_flag.alloc(8);
  launch_matvec(*B.C, 1, 8, true, B.x64.get(), B.N, g.get(), B.N, Epilogue{}, nullptr, s);
  HM_HIP(hipMemcpyAsync(g_eps.get(), epsp.get(), N * 8, hipMemcpyDeviceToDevice, s));
  HM_HIP(hipStreamSynchronize(s));
  g_ready = true;
}

void Batch::set_ambient(const hm_solve_params& p, hipStream_t s) {
  open = p.open_cavity != 0;
  if (!open) return;
  const double t2 = p.ambient_temperature * p.ambient_temperature;
  tamb4 = t2 * t2;
  if (amb_ready) return;
  // row sums of the stored operator: one FP64 product with the most
  // accurate factors on a vector of ones
  if (!gb) gb = std::make_unique<Batch>(mats, 1, s);
  Batch& B = *gb;
  DevBuf ones(N * 8), rs(N * 8);
  hipLaunchKernelGGL(k_fill, grid_rows(N), dim3(256), 0, s, ones.get<double>(), N, 1.0);
  launch_matvec(*B.C, 1, 8, true, ones.get(), N, rs.get(), N, Epilogue{}, nullptr, s);
  amb.alloc(N * 8);
  hipLaunchKernelGGL(k_ambient, grid_rows(N), dim3(256), 0, s, rs.get<double>(), N, amb.get<double>());
  HM_HIP(hipGetLastError());
  HM_HIP(hipStreamSynchronize(s));
  amb_ready = true;
}

SolveResult Batch::solve(const std::vector<const double*>& eps_user, const std::vector<const double*>& T_user,
                         const std::vector<int64_t>& ldT, double sigma, const hm_solve_params& p,
                         const std::vector<double*>& J_user, const std::vector<int64_t>& ldJ,
                         const std::vector<double*>& q_user, const std::vector<int64_t>& ldq, hipStream_t s) {
  SolveResult R;
  const bool want_q = p.want_q && std::any_of(q_user.begin(), q_user.end(), [](double* v) { return v != nullptr; });
  // permuted inputs
  io(IO_EPS, eps_user, {}, 0, nullptr, s);
  gather(IO_EPS, epsp.get<double>(), 1, 1, s);
  hipLaunchKernelGGL(k_omeps<double>, grid_rows(N), dim3(256), 0, s, epsp.get<double>(), N, omeps64.get<double>());
  if (want_q) compare_eps(s);
  io(IO_T, T_user, {}, 0, &ldT, s);
  gather(IO_T, Tp.get<double>(), nrhs, W, s);
  prepare_rhs(sigma, p, s);
  R = solve_prepared(p, s, false, true, want_q);
  if (want_q) {
    ensure_g(eps_user, s);
    set_ambient(p, s);
    flux(sigma, s, R.fx);
  }
  io(IO_J, {}, J_user, 0, &ldJ, s);
  scatter(IO_J, x64.get<double>(), nrhs, s);
  if (want_q) {
    io(IO_Q, {}, q_user, 0, &ldq, s);
    scatter(IO_Q, H64.get<double>(), nrhs, s);
  }
  return R;
}

void Batch::prepare_rhs(double sigma, const hm_solve_params& p, hipStream_t s) {
  const bool f32 = p.mixed_precision || p.vec_dtype == HM_F32;
  if (f32) {
    krylov(4, p.restart, s);
    hipLaunchKernelGGL(k_omeps<float>, grid_rows(N), dim3(256), 0, s, epsp.get<double>(), N, omeps32.get<float>());
  }
  hipLaunchKernelGGL(k_rhs<float>, grid_rows(N, W), dim3(256), 0, s, epsp.get<double>(), Tp.get<double>(), N, nrhs,
                     sigma, b64.get<double>(), f32 ? b32.get<float>() : (float*)nullptr, power_in ? 1 : 0);
  HM_HIP(hipGetLastError());
}

SolveResult Batch::solve_prepared(const hm_solve_params& p, hipStream_t s, bool warm, bool report, bool keep_fx) {
  SolveResult R;
  const int64_t tot = N * W;
  const unsigned gb_ = (unsigned)((tot + 255) / 256);
  if (!p.mixed_precision && p.vec_dtype != HM_F32) {
    Krylov& K = krylov(8, p.restart, s);
    if (!warm) HM_HIP(hipMemcpyAsync(x64.get(), b64.get(), tot * 8, hipMemcpyDeviceToDevice, s));
    GmresStats st = gmres(K, false, omeps64.get(), b64.get(), x64.get(), p.rtol, p.max_iter, s, p.use_graphs != 0);
    R.iters = st.iters;
    R.matvecs = st.matvecs;
    R.bytes = st.bytes;
    R.rel_res = st.rel_res;
    R.converged = st.converged;
  } else if (!p.mixed_precision) {
    Krylov& K = krylov(4, p.restart, s);
    if (warm) hipLaunchKernelGGL((k_cast<double, float>), dim3(gb_), dim3(256), 0, s, x64.get<double>(), x32.get<float>(), tot);
    else HM_HIP(hipMemcpyAsync(x32.get(), b32.get(), tot * 4, hipMemcpyDeviceToDevice, s));
    GmresStats st = gmres(K, false, omeps32.get(), b32.get(), x32.get(), p.rtol, p.max_iter, s, p.use_graphs != 0);
    hipLaunchKernelGGL((k_cast<float, double>), dim3(gb_), dim3(256), 0, s, x32.get<float>(), x64.get<double>(), tot);
    R.iters = st.iters;
    R.matvecs = st.matvecs;
    R.bytes = st.bytes;
    R.converged = st.converged;
    R.rel_res = st.rel_res;  // FP32 GMRES's own residuals
    if (report) {
      // the residual in FP64 against the same stored operator; without FP32
      // copies that is also the flux's operator, so the product can leave
      // F x for it
      const bool fx = keep_fx && !C->mats[0]->has_hi;
      Krylov& K8 = krylov(8, p.restart, s);
      residual64(false, s, fx);
      R.fx = fx;
      R.matvecs++;
      R.bytes += C->bytes_lo;
      std::vector<double> rn, bn;
      block_norms(K8, r64.get(), rn, s);
      block_norms(K8, b64.get(), bn, s);
      R.rel_res.resize(rn.size());
      for (size_t q = 0; q < rn.size(); ++q) {
        R.rel_res[q] = rel_residual(rn[q], bn[q]);
        if (std::isnan(R.rel_res[q])) R.converged = false;
      }
    }
  } else {
    // iterative refinement: FP64 residual with the FP32 (hi) factors, inner
    // FP32 GMRES with the stored (BF16) factors on C d = r, J += d.
    Krylov& K8 = krylov(8, p.restart, s);
    Krylov& K4 = krylov(4, p.restart, s);
    if (!warm) HM_HIP(hipMemsetAsync(x64.get(), 0, tot * 8, s));
    std::vector<double> bn, rn, inner_bn;
    block_norms(K8, b64.get(), bn, s);
    R.converged = false;
    int outer = 0, inner_total = 0;
    const size_t nslots = mats.size();
    const size_t nsys = (size_t)S.size();
    bool masked = false;  // the last refinement step left some slots untouched
    int64_t masked_bytes = 0;
    // per system: still above the tolerance; then per slot: holds such a
    // system (the next residual product runs on those slots only).  One
    // pinned upload per step.
    const size_t flag_bytes = ((nsys + nslots) * 4 + 7) & ~(size_t)7;
    PinnedLease flags_h(flag_bytes);
    int* sys_on = (int*)flags_h.p;
    int* slot_on = sys_on + nsys;
    if (!res_mask.get() || res_mask.bytes() < flag_bytes) res_mask.alloc(flag_bytes);
    const int* slot_on_d = res_mask.get<int>() + nsys;
    for (;;) {
      const bool zero_start = outer == 0 && !warm;
      if (zero_start) {
        // x = 0: the residual is b itself, no product needed (the inner
        // right-hand side below copies b into r64)
        R.fx = false;
      } else {
        // with the flux wanted, the product also leaves F x in H64: the last
        // residual is taken at the final iterate, with the flux's operator.
        // Slots whose systems had all met the tolerance took a zero
        // correction (x unchanged), so their residual and F x from the
        // previous product stand and the product skips them.
        residual64(true, s, keep_fx, masked ? slot_on_d : nullptr);
        R.fx = keep_fx;
        R.matvecs++;
        R.bytes += masked ? masked_bytes : C->bytes_hi;
      }
      if (zero_start)
        rn = bn;  // r = b
      else
        block_norms(K8, r64.get(), rn, s);
      bool done = true, nonfinite = false;
      R.rel_res.resize(rn.size());
      for (size_t q = 0; q < rn.size(); ++q) {
        R.rel_res[q] = rel_residual(rn[q], bn[q]);
        if (!residual_met(rn[q], bn[q], p.rtol)) done = false;
        if (std::isnan(R.rel_res[q])) nonfinite = true;
      }
      if (done) {
        R.converged = true;
        break;
      }
      // a residual that is not finite cannot be refined: stop, not converged
      if (nonfinite || outer >= 30 || inner_total >= p.max_iter) break;
      // the correction starts from zero: x32 = 0, b32 = the residual in
      // FP32, zero on the systems already converged (no inner work)
      hipLaunchKernelGGL(k_inner_rhs, dim3(gb_), dim3(256), 0, s, (zero_start ? b64 : r64).get<double>(),
                         b32.get<float>(), x32.get<float>(), zero_start ? r64.get<double>() : nullptr, tot);
      std::fill(slot_on, slot_on + nslots, 0);
      inner_bn.assign(nsys, 0.0);
      size_t ndone = 0;
      for (size_t q = 0; q < nsys; ++q) {
        sys_on[q] = residual_met(rn[q], bn[q], p.rtol) ? 0 : 1;
        if (sys_on[q]) {
          slot_on[S.sys[q].slot] = 1;
          inner_bn[q] = rn[q];
        } else {
          ++ndone;
        }
      }
      masked_bytes = 0;
      for (size_t q = 0; q < nslots; ++q)
        if (slot_on[q]) masked_bytes += matrix_bytes(*mats[q], true);
      masked = masked_bytes < C->bytes_hi;
      if (ndone > 0 || masked) {
        copy_small(flags_h.dev, res_mask.get(), flag_bytes, s);
        if (ndone > 0)
          hipLaunchKernelGGL(k_zero_done, dim3((unsigned)S.chunks.size()), dim3(256), 0, s, S.d_sys.get<SysDev>(),
                             S.d_chunks.get<ChunkDev>(), res_mask.get<int>(), b32.get<float>(), N);
      }
      // the FP64 residual above checks the correction's progress, so the
      // inner solve stops on its own residual estimate; its right-hand
      // side's norms are the FP64 residual norms (zero where converged)
      GmresStats st = gmres(K4, false, omeps32.get(), b32.get(), x32.get(), p.ir_inner_rtol, p.max_iter, s,
                            p.use_graphs != 0, GM_X0_ZERO | GM_TRUST_ESTIMATE | GM_CGS1, inner_bn.data());
      hipLaunchKernelGGL(k_acc<float>, dim3(gb_), dim3(256), 0, s, x32.get<float>(), x64.get<double>(), tot);
      R.fx = false;  // x changed
      R.iters += st.iters;
      R.matvecs += st.matvecs;
      R.bytes += st.bytes;
      inner_total += st.iters;
      ++outer;
    }
    R.outer = outer;
  }
  return R;
}

// r64 = b64 - C x64 with FP64 vectors (hi: FP32 copy of BF16 factors)
void Batch::residual64(bool hi, hipStream_t s, bool keep_fx, const int* slot_active) {
  Epilogue ep;
  ep.rowscale = omeps64.get();
  ep.a_acc = 1.0;
  ep.a_x = -1.0;
  ep.a_z = 1.0;
  ep.z = b64.get();
  ep.ldz = N;
  if (keep_fx) {
    ep.acc_out = H64.get();
    ep.ld_acc = N;
  }
  launch_matvec(*C, nrhs, 8, hi, x64.get(), N, r64.get(), N, ep, slot_active, s);
}

// H64 <- q = eps (F J - sigma T^4 g), J = x64
void Batch::flux(double sigma, hipStream_t s, bool have_fx) {
  if (!have_fx) launch_matvec(*C, nrhs, 8, true, x64.get(), N, H64.get(), N, Epilogue{}, nullptr, s);
  hipLaunchKernelGGL(k_flux, grid_rows(N, nrhs), dim3(256), 0, s, epsp.get<double>(), Tp.get<double>(),
                     H64.get<double>(), g.get<double>(), N, nrhs, sigma, H64.get<double>(),
                     open ? (const double*)amb.get<double>() : (const double*)nullptr, tamb4, power_in ? 1 : 0);
  HM_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ transient
TransientResult Batch::transient(const std::vector<const double*>& eps_user, double* T_user, int64_t ldT,
                                 const double* src_user, int64_t ldS, double sigma, const hm_transient_params& tp,
                                 const hm_solve_params& sp, double* history, hipStream_t s) {
  TransientResult TR;
  io(IO_EPS, eps_user, {}, 0, nullptr, s);
  gather(IO_EPS, epsp.get<double>(), 1, 1, s);
  hipLaunchKernelGGL(k_omeps<double>, grid_rows(N), dim3(256), 0, s, epsp.get<double>(), N, omeps64.get<double>());
  ensure_g(eps_user, s);
  set_ambient(sp, s);
  const double* ambp = open ? amb.get<double>() : nullptr;
  std::vector<int64_t> ldv{ldT};
  io(IO_T, {T_user}, {}, 0, &ldv, s);
  gather(IO_T, Tp.get<double>(), nrhs, W, s);
  std::vector<int64_t> lds{ldS};
  DevBuf srcp(N * W * 8), Tn(N * W * 8), Rv(N * W * 8), d_upd(W * 4);
  io(IO_SRC, {src_user}, {}, 0, &lds, s);
  gather(IO_SRC, srcp.get<double>(), nrhs, W, s);
  std::vector<int64_t> ldh{ldT};
  if (history) {
    io(IO_HIST, {}, {history}, 0, &ldh, s);
    scatter(IO_HIST, Tp.get<double>(), nrhs, s);
  }
  Krylov& K8 = krylov(8, sp.restart, s);
  std::vector<int> upd(W, 0);
  bool have_J = false;
  // every step's Newton loop ends on an evaluation at the accepted
  // temperatures with no update after it, so J (x64) and q (H64) already hold
  // the next step's first evaluation, which is at the same temperatures
  bool have_q = false;
  for (int step = 0; step < tp.steps; ++step) {
    HM_HIP(hipMemcpyAsync(Tn.get(), Tp.get(), N * W * 8, hipMemcpyDeviceToDevice, s));
    std::vector<double> scale;
    block_norms(K8, Tn.get(), scale, s);
    for (auto& v : scale) v *= tp.mc / tp.dt;
    int it = 0;
    for (;;) {
      if (have_q) {
        have_q = false;
      } else {
        // q(T): radiosity solve (warm start from the previous iterate) and flux
        prepare_rhs(sigma, sp, s);
        // the Newton residual below checks the step: no FP64 report of the solve
        SolveResult R = solve_prepared(sp, s, have_J, false);
        have_J = true;
        TR.matvecs += R.matvecs + 1;
        flux(sigma, s);  // H64 = q
      }
      std::fill(upd.begin(), upd.end(), 0);
      hipLaunchKernelGGL(k_newton, grid_rows(N, nrhs), dim3(256), 0, s, epsp.get<double>(), g.get<double>(),
                         H64.get<double>(), srcp.get<double>(), Tn.get<double>(), Tp.get<double>(), Rv.get<double>(),
                         N, nrhs, tp.mc, tp.dt, sigma, (const int*)nullptr, ambp);
      HM_HIP(hipGetLastError());
      std::vector<double> rn;
      block_norms(K8, Rv.get(), rn, s);
      bool done = true, nonfinite = false;
      double worst = 0.0;
      for (int j = 0; j < nrhs; ++j) {
        const double rel = rel_residual(rn[j], scale[j]);
        worst = max_keep_nan(worst, rel);
        if (std::isnan(rel)) nonfinite = true;
        upd[j] = !rel_met(rel, tp.newton_rtol) && !std::isnan(rel) ? 1 : 0;
        if (upd[j]) done = false;
      }
      if (done || nonfinite || it >= tp.max_newton) {
        TR.max_rel_residual = max_keep_nan(TR.max_rel_residual, worst);
        if (nonfinite) TR.nonfinite = true;
        break;
      }
      HM_HIP(hipMemcpyAsync(d_upd.get(), upd.data(), W * 4, hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_newton, grid_rows(N, nrhs), dim3(256), 0, s, epsp.get<double>(), g.get<double>(),
                         H64.get<double>(), srcp.get<double>(), Tn.get<double>(), Tp.get<double>(), Rv.get<double>(),
                         N, nrhs, tp.mc, tp.dt, sigma, d_upd.get<int>(), ambp);
      HM_HIP(hipGetLastError());
      ++it;
    }
    TR.newton_total += it;
    TR.newton_max = std::max(TR.newton_max, it);
    TR.steps_done = step + 1;
    if (TR.nonfinite) break;
    have_q = true;
    if (history) {
      io(IO_HIST, {}, {history + (int64_t)(step + 1) * ldT * nrhs}, 0, &ldh, s);
      scatter(IO_HIST, Tp.get<double>(), nrhs, s);
    }
  }
  io(IO_J, {}, {T_user}, 0, &ldv, s);
  scatter(IO_J, Tp.get<double>(), nrhs, s);
  HM_HIP(hipStreamSynchronize(s));
  return TR;
}

}  // namespace hm
