// Finite-element coupling of conduction and cavity radiation on gfx950
// (Sec. 3.1-3.4): P1 triangles of a conducting shell that are the cavity's
// facets, the projection P (facet averages of the nodal basis functions),
// the radiation load Q = S eta with S = P^T R_bar P (eqs. (Rdef),
// (Rbardef), (S_def_matrix)), implicit Euler on the Galerkin equations
// (eq. (SVF_Galerkin_time)) solved by Newton-Krylov with the sparse part of
// the Jacobian as preconditioner (eq. (Jprec)).
//
// Every action of R_bar on a facet power eta is one cavity solve: with this
// library's normalised F, R_bar eta = A q, q = eps (F J - sigma eta g),
// J = C^-1 (sigma eps eta), g = F C^-1 eps (eq. (12)), which the batched
// solver computes with the H-matrix when its inputs are powers instead of
// temperatures.  Nodal and facet vectors are FP64 in the caller's order.
#include <algorithm>
#include <cmath>
#include <vector>

#include "dev_common.hpp"
#include "hm_internal.hpp"
#include "solve.hpp"

namespace hm {
namespace {

dim3 rows_grid(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

// eta_i = sum_a P_ia w_a over the facet's vertices (P_ia = 1/3), with
// w = T^4 (mode 0) or w = 4 T^3 x (mode 1: the Jacobian's argument).
__global__ void k_fe_facet(const int32_t* __restrict__ tri, int64_t nf, const double* __restrict__ T,
                           const double* __restrict__ x, int mode, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int32_t v = tri[3 * i + a];
    const double t = T[v], t2 = t * t;
    s += mode == 0 ? t2 * t2 : 4.0 * (t2 * t) * x[v];
  }
  out[i] = s / 3.0;
}

// out_N = sum over the facets i around node N (ascending i) of A_i q_i / 3:
// (P^T diag(A) q)_N.
__global__ void k_fe_nodal(const int32_t* __restrict__ ptr, const int32_t* __restrict__ fac,
                           const double* __restrict__ area, const double* __restrict__ q, int64_t nn,
                           double* __restrict__ out) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nn) return;
  double s = 0.0;
  for (int32_t e = ptr[v]; e < ptr[v + 1]; ++e) {
    const int32_t i = fac[e];
    s += area[i] * q[i];
  }
  out[v] = s / 3.0;
}

// res = M (T - Tn)/dt + K T - Q - f (CSR rows of M and K on one pattern)
__global__ void k_fe_residual(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                              const double* __restrict__ mv, const double* __restrict__ kv,
                              const double* __restrict__ T, const double* __restrict__ Tn,
                              const double* __restrict__ Q, const double* __restrict__ f, double inv_dt, int64_t nn,
                              double* __restrict__ res) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nn) return;
  double s = 0.0;
  for (int32_t e = rp[r]; e < rp[r + 1]; ++e) {
    const int32_t c = ci[e];
    s += mv[e] * (T[c] - Tn[c]) * inv_dt + kv[e] * T[c];
  }
  res[r] = s - Q[r] - (f ? f[r] : 0.0);
}

// y = A x (CSR)
__global__ void k_fe_spmv(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                          const double* __restrict__ av, const double* __restrict__ x, int64_t nn,
                          double* __restrict__ y) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nn) return;
  double s = 0.0;
  for (int32_t e = rp[r]; e < rp[r + 1]; ++e) s += av[e] * x[ci[e]];
  y[r] = s;
}

// y = a x + b y
__global__ void k_fe_axpby(double a, const double* __restrict__ x, double b, double* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}

// z = r / d (Jacobi)
__global__ void k_fe_div(const double* __restrict__ r, const double* __restrict__ d, double* __restrict__ z,
                         int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = r[i] / d[i];
}

// partial dot products per block of 256 (fixed order: the block's tree
// sum), added on the host in block order
__global__ __launch_bounds__(256) void k_fe_dot(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                                                double* __restrict__ part) {
  __shared__ double sh[4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double v = i < n ? a[i] * b[i] : 0.0;
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// ---- conjugate gradients of the preconditioner with device scalars: the
// current and next r.z (two slots, alternating with the iteration's
// parity), p.Ap, r.r, the stopping threshold (pc_rtol |r0|)^2, the done and
// error flags and the iteration count.  Every kernel after the start reads
// the done flag first and does nothing once it is set, so iterations
// launched past convergence change nothing; the host looks at the scalars
// every few iterations.  Sums over a vector are block partials (fixed tree
// order) added by one workgroup in block order.
enum : int { CG_RZ = 0, CG_PAP = 2, CG_RR = 3, CG_TOL2 = 4, CG_DONE = 5, CG_ITS = 6, CG_ERR = 7, CG_N = 8 };

__device__ __forceinline__ double block_sum256(double v, double* sh) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  const double t = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return t;
}

// the npart sums of the partials part[q * stride + k], k = 0..npart-1
// (one workgroup of 256; thread t adds blocks t, t + 256, ... in order)
__device__ __forceinline__ void sum_partials(const double* __restrict__ part, int64_t nb, int npart, double* out) {
  __shared__ double sh[4];
  for (int k = 0; k < npart; ++k) {
    double v = 0.0;
    for (int64_t q = threadIdx.x; q < nb; q += 256) v += part[q * npart + k];
    out[k] = block_sum256(v, sh);
  }
}

// z = 0, res = r, zz = r / d, p = zz; partials of r.r and r.zz
__global__ __launch_bounds__(256) void k_cg_init(const double* __restrict__ r, const double* __restrict__ d,
                                                 int64_t n, double* __restrict__ z, double* __restrict__ res,
                                                 double* __restrict__ zz, double* __restrict__ p,
                                                 double* __restrict__ part) {
  __shared__ double sh[4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double rr = 0.0, rz = 0.0;
  if (i < n) {
    const double v = r[i], w = v / d[i];
    z[i] = 0.0;
    res[i] = v;
    zz[i] = w;
    p[i] = w;
    rr = v * v;
    rz = v * w;
  }
  rr = block_sum256(rr, sh);
  rz = block_sum256(rz, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = rr;
    part[2 * blockIdx.x + 1] = rz;
  }
}

__global__ __launch_bounds__(256) void k_cg_fin_init(const double* __restrict__ part, int64_t nb, double rtol2,
                                                     double* __restrict__ cg) {
  double t[2];
  sum_partials(part, nb, 2, t);
  if (threadIdx.x == 0) {
    cg[CG_RR] = t[0];
    cg[CG_RZ] = t[1];
    cg[CG_RZ + 1] = 0.0;
    cg[CG_PAP] = 0.0;
    cg[CG_TOL2] = rtol2 * t[0];
    cg[CG_DONE] = t[0] == 0.0 ? 1.0 : 0.0;
    cg[CG_ITS] = 0.0;
    cg[CG_ERR] = 0.0;
  }
}

// ap = A p and partials of p.ap
__global__ __launch_bounds__(256) void k_cg_ap(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                               const double* __restrict__ av, const double* __restrict__ p,
                                               int64_t n, double* __restrict__ ap, const double* __restrict__ cg,
                                               double* __restrict__ part) {
  __shared__ double sh[4];
  if (cg[CG_DONE] != 0.0) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    double s = 0.0;
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) s += av[e] * p[ci[e]];
    ap[i] = s;
    v = p[i] * s;
  }
  v = block_sum256(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

__global__ __launch_bounds__(256) void k_cg_fin_pap(const double* __restrict__ part, int64_t nb,
                                                    double* __restrict__ cg) {
  if (cg[CG_DONE] != 0.0) return;
  double t;
  sum_partials(part, nb, 1, &t);
  if (threadIdx.x == 0) {
    if (t > 0.0 && isfinite(t)) {
      cg[CG_PAP] = t;
    } else {  // not positive definite (or not finite): stop with an error
      cg[CG_ERR] = 1.0;
      cg[CG_DONE] = 1.0;
    }
  }
}

// z += alpha p, res -= alpha ap, zz = res / d (alpha = r.z / p.Ap);
// partials of res.res and res.zz
__global__ __launch_bounds__(256) void k_cg_step(const double* __restrict__ cg, int par, const double* __restrict__ p,
                                                 const double* __restrict__ ap, const double* __restrict__ d,
                                                 int64_t n, double* __restrict__ z, double* __restrict__ res,
                                                 double* __restrict__ zz, double* __restrict__ part) {
  __shared__ double sh[4];
  if (cg[CG_DONE] != 0.0) return;
  const double alpha = cg[CG_RZ + par] / cg[CG_PAP];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double rr = 0.0, rz = 0.0;
  if (i < n) {
    z[i] += alpha * p[i];
    const double v = res[i] - alpha * ap[i], w = v / d[i];
    res[i] = v;
    zz[i] = w;
    rr = v * v;
    rz = v * w;
  }
  rr = block_sum256(rr, sh);
  rz = block_sum256(rz, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = rr;
    part[2 * blockIdx.x + 1] = rz;
  }
}

__global__ __launch_bounds__(256) void k_cg_fin_step(const double* __restrict__ part, int64_t nb, int par,
                                                     double* __restrict__ cg) {
  if (cg[CG_DONE] != 0.0) return;
  double t[2];
  sum_partials(part, nb, 2, t);
  if (threadIdx.x == 0) {
    cg[CG_RR] = t[0];
    cg[CG_RZ + 1 - par] = t[1];
    cg[CG_ITS] += 1.0;
    if (t[0] <= cg[CG_TOL2]) cg[CG_DONE] = 1.0;
  }
}

// p = zz + beta p, beta = (new r.z) / (old r.z)
__global__ __launch_bounds__(256) void k_cg_dir(const double* __restrict__ cg, int par,
                                                const double* __restrict__ zz, int64_t n, double* __restrict__ p) {
  if (cg[CG_DONE] != 0.0) return;
  const double beta = cg[CG_RZ + 1 - par] / cg[CG_RZ + par];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = zz[i] + beta * p[i];
}

// out = the sum of the partials of k_fe_dot (fixed order)
__global__ __launch_bounds__(256) void k_fe_dot_fin(const double* __restrict__ part, int64_t nb,
                                                    double* __restrict__ out) {
  double t;
  sum_partials(part, nb, 1, &t);
  if (threadIdx.x == 0) out[0] = t;
}

}  // namespace
}  // namespace hm

using hm::Batch;
using hm::DevBuf;

struct hm_fe {
  int device = 0;
  const hm_matrix* F = nullptr;
  int64_t nn = 0, nf = 0;
  hm_fe_params p{};
  DevBuf tri, nptr, nfac, area, eps, rp, ci, mv, kv, pcv, pcd;  // mesh, CSR of M, K and M/dt + K
  std::unique_ptr<Batch> B;
  // work vectors; device scalars of the conjugate gradients and of dot
  // products, read back through mapped pinned memory
  DevBuf eta, qf, Jf, part, cg;
  std::unique_ptr<hm::PinnedLease> cg_h;
  int cavity_solves = 0, pc_iterations = 0;
};

namespace hm {

namespace {

// The device scalars (CG_N doubles) on the host.
const double* fetch_scalars(hm_fe& fe, hipStream_t s) {
  copy_small(fe.cg.get(), fe.cg_h->dev, CG_N * 8, s);
  HM_HIP(hipStreamSynchronize(s));
  return (const double*)fe.cg_h->p;
}

double fe_dot(hm_fe& fe, const double* a, const double* b, hipStream_t s) {
  const int64_t nb = (fe.nn + 255) / 256;
  hipLaunchKernelGGL(k_fe_dot, dim3((unsigned)nb), dim3(256), 0, s, a, b, fe.nn, fe.part.get<double>());
  hipLaunchKernelGGL(k_fe_dot_fin, dim3(1), dim3(256), 0, s, fe.part.get<double>(), nb, fe.cg.get<double>() + CG_N);
  HM_HIP(hipGetLastError());
  copy_small(fe.cg.get<double>() + CG_N, fe.cg_h->dev, 8, s);
  HM_HIP(hipStreamSynchronize(s));
  return *(const double*)fe.cg_h->p;
}

void axpby(hm_fe& fe, double a, const double* x, double b, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_fe_axpby, rows_grid(fe.nn), dim3(256), 0, s, a, x, b, y, fe.nn);
  HM_HIP(hipGetLastError());
}

// out = S w_nodal for the facet power eta (already in fe.eta): out =
// P^T diag(A) q(eta), one cavity solve to the relative residual rtol
void apply_rbar(hm_fe& fe, double* out, double rtol, hipStream_t s) {
  hm_solve_params sp = fe.p.solve;
  sp.rtol = rtol;
  sp.want_q = 1;
  sp.open_cavity = 0;
  SolveResult R = fe.B->solve({fe.eps.get<double>()}, {fe.eta.get<double>()}, {fe.nf}, fe.p.sigma, sp,
                              {fe.Jf.get<double>()}, {fe.nf}, {fe.qf.get<double>()}, {fe.nf}, s);
  HM_REQUIRE(R.converged, "fe: a cavity solve did not reach its tolerance");
  ++fe.cavity_solves;
  hipLaunchKernelGGL(k_fe_nodal, rows_grid(fe.nn), dim3(256), 0, s, fe.nptr.get<int32_t>(), fe.nfac.get<int32_t>(),
                     fe.area.get<double>(), fe.qf.get<double>(), fe.nn, out);
  HM_HIP(hipGetLastError());
}

// Q = S T^4
void cavity_load(hm_fe& fe, const double* T, double* Q, hipStream_t s) {
  hipLaunchKernelGGL(k_fe_facet, rows_grid(fe.nf), dim3(256), 0, s, fe.tri.get<int32_t>(), fe.nf, T,
                     (const double*)nullptr, 0, fe.eta.get<double>());
  HM_HIP(hipGetLastError());
  apply_rbar(fe, Q, fe.p.solve.rtol, s);
}

// z = (M/dt + K)^-1 r by conjugate gradients with the diagonal as
// preconditioner, from z = 0, to |r - A z| <= pc_rtol |r|.  The scalars stay
// on the device; the host launches blocks of CG_BLOCK iterations and reads
// them back after each.
void pc_solve(hm_fe& fe, const double* r, double* z, std::vector<DevBuf>& w, hipStream_t s) {
  constexpr int CG_BLOCK = 8, CG_MAX = 2000;
  const int64_t n = fe.nn, nb = (n + 255) / 256;
  double* res = w[0].get<double>();
  double* zz = w[1].get<double>();
  double* pp = w[2].get<double>();
  double* ap = w[3].get<double>();
  double* cg = fe.cg.get<double>();
  double* part = fe.part.get<double>();
  const dim3 g((unsigned)nb);
  const double rtol2 = fe.p.pc_rtol * fe.p.pc_rtol;
  hipLaunchKernelGGL(k_cg_init, g, dim3(256), 0, s, r, fe.pcd.get<double>(), n, z, res, zz, pp, part);
  hipLaunchKernelGGL(k_cg_fin_init, dim3(1), dim3(256), 0, s, part, nb, rtol2, cg);
  HM_HIP(hipGetLastError());
  for (int it = 0; it < CG_MAX; it += CG_BLOCK) {
    for (int q = 0; q < CG_BLOCK; ++q) {
      const int par = q & 1;  // CG_BLOCK is even: every block starts at parity 0
      hipLaunchKernelGGL(k_cg_ap, g, dim3(256), 0, s, fe.rp.get<int32_t>(), fe.ci.get<int32_t>(),
                         fe.pcv.get<double>(), pp, n, ap, cg, part);
      hipLaunchKernelGGL(k_cg_fin_pap, dim3(1), dim3(256), 0, s, part, nb, cg);
      hipLaunchKernelGGL(k_cg_step, g, dim3(256), 0, s, cg, par, pp, ap, fe.pcd.get<double>(), n, z, res, zz, part);
      hipLaunchKernelGGL(k_cg_fin_step, dim3(1), dim3(256), 0, s, part, nb, par, cg);
      hipLaunchKernelGGL(k_cg_dir, g, dim3(256), 0, s, cg, par, zz, n, pp);
    }
    HM_HIP(hipGetLastError());
    const double* h = fetch_scalars(fe, s);
    if (h[CG_DONE] != 0.0) {
      fe.pc_iterations += (int)h[CG_ITS];
      HM_REQUIRE(h[CG_ERR] == 0.0, "fe: the preconditioner's matrix is not positive definite");
      return;
    }
  }
  fail(HM_ENOTCONV, "fe: conjugate gradients for the preconditioner did not converge");
}

// y = (M/dt + K)^-1 J v = v - (M/dt + K)^-1 S (4 T^3 v)
void prec_jacobian(hm_fe& fe, const double* T, const double* v, double* y, std::vector<DevBuf>& w, double* tmp,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_fe_facet, rows_grid(fe.nf), dim3(256), 0, s, fe.tri.get<int32_t>(), fe.nf, T, v, 1,
                     fe.eta.get<double>());
  HM_HIP(hipGetLastError());
  // a Jacobian product needs its cavity solve only two orders below the
  // Krylov tolerance (the product's relative error is about cond(C) times
  // the solve's residual); the residual's own solves keep solve.rtol
  apply_rbar(fe, tmp, std::max(fe.p.solve.rtol, 1e-2 * fe.p.krylov_rtol), s);
  pc_solve(fe, tmp, y, w, s);
  axpby(fe, 1.0, v, -1.0, y, s);
}

}  // namespace

hm_fe* fe_create(hm_ctx& ctx, const hm_matrix& F, int64_t nn, const double* vtx, int64_t nf, const int32_t* tri,
                 const double* eps, const hm_fe_params& p) {
  hipStream_t s = ctx.stream;
  HM_REQUIRE(nf == F.n, "hm_fe_create: n_facets differs from the H-matrix's size");
  HM_REQUIRE(nn >= 3 && nn < ((int64_t)1 << 30) && nf < ((int64_t)1 << 29), "hm_fe_create: bad mesh sizes");
  auto fe = std::make_unique<hm_fe>();
  fe->device = ctx.device;
  fe->F = &F;
  fe->nn = nn;
  fe->nf = nf;
  fe->p = p;
  // element matrices (FP64, host), CSR pattern of the node adjacency
  std::vector<double> area(nf);
  std::vector<std::vector<std::pair<int32_t, std::pair<double, double>>>> rows(nn);
  std::vector<std::vector<int32_t>> inc(nn);
  for (int64_t i = 0; i < nf; ++i) {
    int32_t t[3];
    double x[3][3];
    for (int a = 0; a < 3; ++a) {
      t[a] = tri[3 * i + a];
      HM_REQUIRE(t[a] >= 0 && t[a] < nn, "hm_fe_create: vertex index out of range");
      for (int c = 0; c < 3; ++c) x[a][c] = vtx[3 * (int64_t)t[a] + c];
    }
    double e[3][3];  // edge opposite vertex a: x[a+2] - x[a+1]
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) e[a][c] = x[(a + 2) % 3][c] - x[(a + 1) % 3][c];
    const double cx = e[2][1] * (-e[1][2]) - e[2][2] * (-e[1][1]);
    const double cy = e[2][2] * (-e[1][0]) - e[2][0] * (-e[1][2]);
    const double cz = e[2][0] * (-e[1][1]) - e[2][1] * (-e[1][0]);
    const double A = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
    HM_REQUIRE(A > 0.0 && std::isfinite(A), "hm_fe_create: degenerate triangle");
    area[i] = A;
    for (int a = 0; a < 3; ++a) {
      inc[t[a]].push_back((int32_t)i);
      for (int b = 0; b < 3; ++b) {
        const double m = p.capacity * A / 12.0 * (a == b ? 2.0 : 1.0);
        const double k = p.conductance * (e[a][0] * e[b][0] + e[a][1] * e[b][1] + e[a][2] * e[b][2]) / (4.0 * A);
        rows[t[a]].push_back({t[b], {m, k}});
      }
    }
  }
  std::vector<int32_t> rp(nn + 1, 0), ci;
  std::vector<double> mv, kv, pcv, pcd(nn, 0.0);
  for (int64_t r = 0; r < nn; ++r) {
    auto& R = rows[r];
    HM_REQUIRE(!R.empty(), "hm_fe_create: a node belongs to no triangle");
    std::sort(R.begin(), R.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
    for (size_t q = 0; q < R.size();) {
      const int32_t c = R[q].first;
      double m = 0.0, k = 0.0;
      for (; q < R.size() && R[q].first == c; ++q) {
        m += R[q].second.first;
        k += R[q].second.second;
      }
      ci.push_back(c);
      mv.push_back(m);
      kv.push_back(k);
      pcv.push_back(m / p.dt + k);
      if (c == r) pcd[r] = m / p.dt + k;
    }
    rp[r + 1] = (int32_t)ci.size();
  }
  std::vector<int32_t> nptr(nn + 1, 0), nfac;
  for (int64_t v = 0; v < nn; ++v) {
    nfac.insert(nfac.end(), inc[v].begin(), inc[v].end());
    nptr[v + 1] = (int32_t)nfac.size();
  }
  std::vector<int32_t> trv(tri, tri + 3 * nf);
  upload(fe->tri, trv, s);
  upload(fe->nptr, nptr, s);
  upload(fe->nfac, nfac, s);
  upload(fe->area, area, s);
  upload(fe->rp, rp, s);
  upload(fe->ci, ci, s);
  upload(fe->mv, mv, s);
  upload(fe->kv, kv, s);
  upload(fe->pcv, pcv, s);
  upload(fe->pcd, pcd, s);
  fe->eps.alloc(nf * 8);
  HM_HIP(hipMemcpyAsync(fe->eps.get(), eps, nf * 8, hipMemcpyDeviceToDevice, s));
  fe->eta.alloc(nf * 8);
  fe->qf.alloc(nf * 8);
  fe->Jf.alloc(nf * 8);
  fe->part.alloc(((nn + 255) / 256) * 2 * 8);
  fe->cg.alloc((CG_N + 8) * 8);
  fe->cg_h = std::make_unique<hm::PinnedLease>((CG_N + 8) * 8);
  fe->B = std::make_unique<Batch>(std::vector<const hm_matrix*>{&F}, 1, s);
  fe->B->power_in = true;
  HM_HIP(hipStreamSynchronize(s));
  return fe.release();
}

void fe_cavity_load(hm_ctx& ctx, hm_fe& fe, const double* T, double* Q) {
  hipStream_t s = ctx.stream;
  cavity_load(fe, T, Q, s);
  HM_HIP(hipStreamSynchronize(s));
}

hm_fe_info fe_step(hm_ctx& ctx, hm_fe& fe, const double* Tn_user, const double* f_facet, double* T_out) {
  hipStream_t s = ctx.stream;
  const int64_t n = fe.nn;
  hm_fe_info info{};
  fe.cavity_solves = 0;
  fe.pc_iterations = 0;
  const int m = fe.p.krylov_restart;
  DevBuf Tn(n * 8), T(n * 8), Q(n * 8), res(n * 8), fN(n * 8), tmp(n * 8), rhs(n * 8), d(n * 8), Vb((size_t)(m + 1) * n * 8);
  std::vector<DevBuf> w(4);
  for (auto& b : w) b.alloc(n * 8);
  HM_HIP(hipMemcpyAsync(Tn.get(), Tn_user, n * 8, hipMemcpyDeviceToDevice, s));
  HM_HIP(hipMemcpyAsync(T.get(), Tn_user, n * 8, hipMemcpyDeviceToDevice, s));
  const double* fptr = nullptr;
  if (f_facet) {
    hipLaunchKernelGGL(k_fe_nodal, rows_grid(n), dim3(256), 0, s, fe.nptr.get<int32_t>(), fe.nfac.get<int32_t>(),
                       fe.area.get<double>(), f_facet, n, fN.get<double>());
    fptr = fN.get<double>();
  }
  // scale = |M T^n / dt|
  hipLaunchKernelGGL(k_fe_spmv, rows_grid(n), dim3(256), 0, s, fe.rp.get<int32_t>(), fe.ci.get<int32_t>(),
                     fe.mv.get<double>(), Tn.get<double>(), n, tmp.get<double>());
  const double scale = std::sqrt(fe_dot(fe, tmp.get<double>(), tmp.get<double>(), s)) / fe.p.dt;
  auto residual = [&]() {
    cavity_load(fe, T.get<double>(), Q.get<double>(), s);
    hipLaunchKernelGGL(k_fe_residual, rows_grid(n), dim3(256), 0, s, fe.rp.get<int32_t>(), fe.ci.get<int32_t>(),
                       fe.mv.get<double>(), fe.kv.get<double>(), T.get<double>(), Tn.get<double>(), Q.get<double>(),
                       fptr, 1.0 / fe.p.dt, n, res.get<double>());
    HM_HIP(hipGetLastError());
    return std::sqrt(fe_dot(fe, res.get<double>(), res.get<double>(), s));
  };
  double rn = residual();
  info.status = HM_ENOTCONV;
  for (int it = 0;; ++it) {
    HM_REQUIRE(std::isfinite(rn), "fe: the residual is not finite");
    if (rn <= fe.p.newton_rtol * scale) {
      info.status = HM_OK;
      break;
    }
    if (it >= fe.p.max_newton) break;
    // GMRES(m) from d = 0 on (M/dt + K)^-1 J d = -(M/dt + K)^-1 res
    pc_solve(fe, res.get<double>(), rhs.get<double>(), w, s);
    axpby(fe, 0.0, rhs.get<double>(), -1.0, rhs.get<double>(), s);  // rhs = -(...)
    HM_HIP(hipMemsetAsync(d.get(), 0, n * 8, s));
    const double b0 = std::sqrt(fe_dot(fe, rhs.get<double>(), rhs.get<double>(), s));
    double* V = Vb.get<double>();
    HM_HIP(hipMemcpyAsync(V, rhs.get(), n * 8, hipMemcpyDeviceToDevice, s));
    double beta = b0;
    int kr = 0;
    while (beta > fe.p.krylov_rtol * b0 && kr < fe.p.max_krylov) {
      // one cycle from the current d: V_0 = r / |r|
      axpby(fe, 0.0, V, 1.0 / beta, V, s);
      std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1, 0.0);
      g[0] = beta;
      int j = 0;
      for (; j < m && kr < fe.p.max_krylov; ++j, ++kr) {
        double* vj = V + (int64_t)j * n;
        double* wj = V + (int64_t)(j + 1) * n;
        prec_jacobian(fe, T.get<double>(), vj, wj, w, tmp.get<double>(), s);
        for (int i = 0; i <= j; ++i) {  // modified Gram-Schmidt
          const double h = fe_dot(fe, V + (int64_t)i * n, wj, s);
          H[(size_t)i * m + j] = h;
          axpby(fe, -h, V + (int64_t)i * n, 1.0, wj, s);
        }
        const double hn = std::sqrt(fe_dot(fe, wj, wj, s));
        H[(size_t)(j + 1) * m + j] = hn;
        if (hn > 0.0) axpby(fe, 0.0, wj, 1.0 / hn, wj, s);
        for (int i = 0; i < j; ++i) {  // earlier rotations
          const double a = H[(size_t)i * m + j], b = H[(size_t)(i + 1) * m + j];
          H[(size_t)i * m + j] = cs[i] * a + sn[i] * b;
          H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
        }
        const double a = H[(size_t)j * m + j], b = H[(size_t)(j + 1) * m + j];
        const double r = std::hypot(a, b);
        cs[j] = r > 0.0 ? a / r : 1.0;
        sn[j] = r > 0.0 ? b / r : 0.0;
        H[(size_t)j * m + j] = r;
        H[(size_t)(j + 1) * m + j] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        if (std::fabs(g[j + 1]) <= fe.p.krylov_rtol * b0 || hn == 0.0) {
          ++j;
          ++kr;
          break;
        }
      }
      // d += V y, H y = g (upper triangular j x j)
      std::vector<double> y(j, 0.0);
      for (int i = j - 1; i >= 0; --i) {
        double v = g[i];
        for (int k = i + 1; k < j; ++k) v -= H[(size_t)i * m + k] * y[k];
        y[i] = v / H[(size_t)i * m + i];
      }
      for (int i = 0; i < j; ++i) axpby(fe, y[i], V + (int64_t)i * n, 1.0, d.get<double>(), s);
      info.krylov += j;
      beta = std::fabs(g[j]);
      if (beta > fe.p.krylov_rtol * b0 && kr < fe.p.max_krylov) {
        // restart: the true preconditioned residual rhs - (M/dt+K)^-1 J d
        prec_jacobian(fe, T.get<double>(), d.get<double>(), V, w, tmp.get<double>(), s);
        axpby(fe, 1.0, rhs.get<double>(), -1.0, V, s);
        beta = std::sqrt(fe_dot(fe, V, V, s));
      }
    }
    axpby(fe, 1.0, d.get<double>(), 1.0, T.get<double>(), s);
    ++info.newton;
    rn = residual();
  }
  HM_HIP(hipMemcpyAsync(T_out, T.get(), n * 8, hipMemcpyDeviceToDevice, s));
  HM_HIP(hipStreamSynchronize(s));
  info.residual = scale > 0.0 ? rn / scale : rn;
  info.cavity_solves = fe.cavity_solves;
  info.pc_iterations = fe.pc_iterations;
  return info;
}

void fe_destroy(hm_fe* fe) { delete fe; }
int fe_device(const hm_fe& fe) { return fe.device; }
const hm_matrix* fe_matrix(const hm_fe& fe) { return fe.F; }
int64_t fe_nodes(const hm_fe& fe) { return fe.nn; }
int64_t fe_facets(const hm_fe& fe) { return fe.nf; }

}  // namespace hm
