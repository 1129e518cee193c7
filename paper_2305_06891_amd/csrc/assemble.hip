// H-matrix assembly on gfx950: centroid-rule view factors (eq. (10)), the
// dense near field of the inadmissible leaves, and adaptive cross
// approximation (Sec. 4.3, eqs. (30)-(31)) of the admissible leaves.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "dev_common.hpp"
#include "hm_internal.hpp"

namespace hm {

struct Geo {
  const double *cx, *cy, *cz, *nx, *ny, *nz, *ar;  // permuted facet geometry (FP64)
};

// Centroid-rule view factor between permuted facets i and j (eq. (10) with
// one quadrature point per facet, per-area convention): both cosines are
// measured against the centroid segment and clamped at zero; F_ii = 0.
// Evaluated in FP64 without contraction in the fixed operation order
// d = c_j - c_i, r2 = (dx*dx + dy*dy) + dz*dz, ci = (n_i.d), cj = -(n_j.d),
// F = (max(ci,0) * max(cj,0) * A_j) / ((pi * r2) * r2).
#pragma clang fp contract(off)
__device__ __forceinline__ double view_factor(const Geo& g, int i, int j) {
  if (i == j) return 0.0;
  const double dx = g.cx[j] - g.cx[i];
  const double dy = g.cy[j] - g.cy[i];
  const double dz = g.cz[j] - g.cz[i];
  const double r2 = (dx * dx + dy * dy) + dz * dz;
  const double ci = (g.nx[i] * dx + g.ny[i] * dy) + g.nz[i] * dz;
  const double cj = -((g.nx[j] * dx + g.ny[j] * dy) + g.nz[j] * dz);
  const double num = fmax(ci, 0.0) * fmax(cj, 0.0) * g.ar[j];
  const double den = (3.141592653589793 * r2) * r2;
  return r2 > 0.0 ? num / den : 0.0;
}
#pragma clang fp contract(on)

struct DnDev {
  int32_t rb, re, cb, ce;
  int64_t off;
};

// One workgroup per dense block; column-major m x n output.
template <class OT>
__global__ __launch_bounds__(256) void k_nearfield(const DnDev* __restrict__ blocks, Geo g, OT* __restrict__ out) {
  const DnDev b = blocks[blockIdx.x];
  const int m = b.re - b.rb, n = b.ce - b.cb;
  const int64_t mn = (int64_t)m * n;
  OT* o = out + b.off;
  for (int64_t e = threadIdx.x; e < mn; e += blockDim.x) {
    const int r = (int)(e % m), c = (int)(e / m);
    o[e] = Cvt<OT>::from_f64(view_factor(g, b.rb + r, b.cb + c));
  }
}

struct AcaDev {
  int32_t rb, re, cb, ce;
  int32_t kcap, pad;
  int64_t u_off, v_off, f_off;  // scratch offsets (doubles, doubles, ints)
};

constexpr int ACA_T = 256;
constexpr int ACA_W = ACA_T / 64;
constexpr int ACA_KMAX = 1024;

// (|value|, index) maximum over the workgroup: larger magnitude wins, the
// smaller index breaks ties.  The signed value travels with the winner.
struct ArgMax {
  double mag;
  double val;
  int idx;
};

__device__ inline ArgMax better(ArgMax a, ArgMax b) {
  if (b.mag > a.mag || (b.mag == a.mag && b.idx < a.idx)) return b;
  return a;
}

__device__ ArgMax block_argmax(ArgMax v, ArgMax* sh) {
  for (int o = 32; o > 0; o >>= 1) {
    ArgMax w;
    w.mag = __shfl_xor(v.mag, o, 64);
    w.val = __shfl_xor(v.val, o, 64);
    w.idx = __shfl_xor(v.idx, o, 64);
    v = better(v, w);
  }
  const int wid = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[wid] = v;
  __syncthreads();
  ArgMax r = sh[0];
  for (int w = 1; w < ACA_W; ++w) r = better(r, sh[w]);
  return r;
}

// Sum of NV values over the workgroup, fixed order (waves 0..3).
template <int NV>
__device__ void block_sum(double* v, double* sh) {
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
  const int wid = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) sh[wid * NV + q] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = sh[q];
    for (int w = 1; w < ACA_W; ++w) s += sh[w * NV + q];
    v[q] = s;
  }
}

// Partial-pivoting ACA of one admissible block per workgroup, in FP64.
// U (m x kcap) and V (n x kcap) are column-major scratch; on exit rank[b]
// holds k and status[b] is 1 when the stop test |u||v| <= tol |sum u v^T|_F
// was met (0 when the rank cap was reached first).
#pragma clang fp contract(off)
__global__ __launch_bounds__(ACA_T) void k_aca(const AcaDev* __restrict__ blocks, Geo g, double tol,
                                               double* __restrict__ scratch, int* __restrict__ flags,
                                               int* __restrict__ rank, int* __restrict__ status) {
  __shared__ double coef[ACA_KMAX];
  __shared__ ArgMax sh_am[ACA_W];
  __shared__ double sh_sum[ACA_W * 16];
  const AcaDev b = blocks[blockIdx.x];
  const int m = b.re - b.rb, n = b.ce - b.cb;
  double* U = scratch + b.u_off;
  double* V = scratch + b.v_off;
  int* used = flags + b.f_off;
  const int tid = threadIdx.x;
  for (int i = tid; i < m; i += ACA_T) used[i] = 0;
  __syncthreads();

  int i = 0, k = 0;
  double s2 = 0.0;
  int conv = 0;
  for (;;) {
    // residual row i: r_j = F(i, j) - sum_l u_l(i) v_l(j), written to V[:, k]
    for (int l = tid; l < k; l += ACA_T) coef[l] = U[(int64_t)l * m + i];
    __syncthreads();
    ArgMax am{-1.0, 0.0, 0x7fffffff};
    double* vk = V + (int64_t)k * n;
    for (int j = tid; j < n; j += ACA_T) {
      double r = view_factor(g, b.rb + i, b.cb + j);
      for (int l = 0; l < k; ++l) r = r - coef[l] * V[(int64_t)l * n + j];
      vk[j] = r;
      const double a = fabs(r);
      if (a > am.mag || (a == am.mag && j < am.idx)) am = ArgMax{a, r, j};
    }
    am = block_argmax(am, sh_am);
    const int jp = am.idx;
    const double rj = am.val;
    if (rj == 0.0) {
      // zero residual row: mark it used and move to the smallest unused row
      if (tid == 0) used[i] = 1;
      __syncthreads();
      ArgMax nx{-1.0, 0.0, 0x7fffffff};
      for (int ii = tid; ii < m; ii += ACA_T)
        if (!used[ii] && ii < nx.idx) nx = ArgMax{0.0, 0.0, ii};
      nx = block_argmax(nx, sh_am);
      if (nx.idx == 0x7fffffff) { conv = 1; break; }
      i = nx.idx;
      continue;
    }
    // v = r / r(jp)
    for (int j = tid; j < n; j += ACA_T) vk[j] = vk[j] / rj;
    // residual column jp: u_i = F(i, jp) - sum_l v_l(jp) u_l(i), written to U[:, k]
    __syncthreads();
    for (int l = tid; l < k; l += ACA_T) coef[l] = V[(int64_t)l * n + jp];
    if (tid == 0) used[i] = 1;
    __syncthreads();
    double* uk = U + (int64_t)k * m;
    ArgMax nx{-1.0, 0.0, 0x7fffffff};
    double nu2 = 0.0, nv2 = 0.0;
    for (int ii = tid; ii < m; ii += ACA_T) {
      double u = view_factor(g, b.rb + ii, b.cb + jp);
      for (int l = 0; l < k; ++l) u = u - coef[l] * U[(int64_t)l * m + ii];
      uk[ii] = u;
      nu2 += u * u;
      if (!used[ii]) {
        const double a = fabs(u);
        if (a > nx.mag || (a == nx.mag && ii < nx.idx)) nx = ArgMax{a, u, ii};
      }
    }
    for (int j = tid; j < n; j += ACA_T) nv2 += vk[j] * vk[j];
    {
      double t2[2] = {nu2, nv2};
      block_sum<2>(t2, sh_sum);
      nu2 = t2[0];
      nv2 = t2[1];
    }
    // cross terms sum_l (u_l . u)(v_l . v), eight ranks at a time
    double cross = 0.0;
    for (int l0 = 0; l0 < k; l0 += 8) {
      double d[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) d[q] = 0.0;
      const int nl = min(8, k - l0);
      for (int ii = tid; ii < m; ii += ACA_T) {
        const double u = uk[ii];
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (q < nl) d[q] += U[(int64_t)(l0 + q) * m + ii] * u;
      }
      for (int j = tid; j < n; j += ACA_T) {
        const double v = vk[j];
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (q < nl) d[8 + q] += V[(int64_t)(l0 + q) * n + j] * v;
      }
      block_sum<16>(d, sh_sum);
      for (int q = 0; q < nl; ++q) cross += d[q] * d[8 + q];
    }
    s2 += nu2 * nv2 + 2.0 * cross;
    ++k;
    if (sqrt(nu2 * nv2) <= tol * sqrt(fmax(s2, 0.0))) { conv = 1; break; }
    if (k >= b.kcap) { conv = 0; break; }
    nx = block_argmax(nx, sh_am);
    if (nx.idx == 0x7fffffff) { conv = 1; break; }
    i = nx.idx;
  }
  if (tid == 0) {
    rank[blockIdx.x] = k;
    status[blockIdx.x] = conv;
  }
}
#pragma clang fp contract(on)

struct CompactDev {
  int64_t su, sv;   // scratch offsets of U, V (doubles)
  int64_t du, dv;   // destination offsets (elements) in the stage buffers
  int32_t m, n, k, pad;
};

// Copy the first k columns of the FP64 scratch factors into the storage
// type (and optionally an FP32 copy).
template <class OT>
__global__ __launch_bounds__(256) void k_compact(const CompactDev* __restrict__ cd, const double* __restrict__ scratch,
                                                 OT* __restrict__ U, OT* __restrict__ V, float* __restrict__ Uhi,
                                                 float* __restrict__ Vhi) {
  const CompactDev c = cd[blockIdx.x];
  const int64_t nu = (int64_t)c.m * c.k, nv = (int64_t)c.n * c.k;
  for (int64_t e = threadIdx.x; e < nu; e += blockDim.x) {
    const double x = scratch[c.su + e];
    U[c.du + e] = Cvt<OT>::from_f64(x);
    if (Uhi) Uhi[c.du + e] = (float)x;
  }
  for (int64_t e = threadIdx.x; e < nv; e += blockDim.x) {
    const double x = scratch[c.sv + e];
    V[c.dv + e] = Cvt<OT>::from_f64(x);
    if (Vhi) Vhi[c.dv + e] = (float)x;
  }
}

// Row scaling of the stored blocks (closed cavity, eqs. (32)-(34)): row i
// of every dense block and of every U factor is multiplied by scale[i].
struct ScaleDev {
  int64_t off;
  int32_t rb, m, w, kind;  // kind 0 dense (m x w), 1 U (m x w)
};

template <class DT, class LT>
__global__ __launch_bounds__(256) void k_rowscale(const ScaleDev* __restrict__ sd, const double* __restrict__ scale,
                                                  DT* __restrict__ dense, LT* __restrict__ U, float* __restrict__ Uhi) {
  const ScaleDev s = sd[blockIdx.x];
  const int64_t tot = (int64_t)s.m * s.w;
  for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
    const int r = (int)(e % s.m);
    const double f = scale[s.rb + r];
    if (s.kind == 0) {
      dense[s.off + e] = Cvt<DT>::from_f64(Cvt<DT>::to_f64(dense[s.off + e]) * f);
    } else {
      const int64_t q = s.off + e;
      if (Uhi) {
        const double x = (double)Uhi[q] * f;
        Uhi[q] = (float)x;
        U[q] = Cvt<LT>::from_f64(x);
      } else {
        U[q] = Cvt<LT>::from_f64(Cvt<LT>::to_f64(U[q]) * f);
      }
    }
  }
}

__global__ void k_closed_scale(const double* __restrict__ s, double* __restrict__ scale, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double c = fmin(fmax(s[i], 0.0), 1.0);
    scale[i] = c != 0.0 ? 1.0 / c : 1.0;
  }
}

namespace {

int64_t rank_cap(int m, int n, int kmax) {
  int64_t mn = (int64_t)m * n;
  int64_t c = (mn + (m + n) - 1) / (m + n);
  return std::max<int64_t>(1, std::min<int64_t>(kmax, c));
}

template <class F>
void dispatch_dtype(hm_dtype t, F&& f) {
  if (t == HM_F64) f((double*)nullptr);
  else if (t == HM_F32) f((float*)nullptr);
  else f((bf16_t*)nullptr);
}

}  // namespace

void closed_row_scale(hm_matrix& M, const std::vector<DnInfo>& dn, const std::vector<LrInfo>& lr, hipStream_t s);

hm_matrix* assemble(hm_ctx& ctx, const hm_tree& t, const hm_assembly_params& p) {
  hipStream_t s = ctx.stream;
  const int64_t n = t.n;
  auto M = std::make_unique<hm_matrix>();
  M->device = ctx.device;
  M->n = n;
  M->dense_dtype = p.dense_dtype;
  M->lr_dtype = p.lowrank_dtype;
  M->has_hi = p.lowrank_dtype == HM_BF16 && p.keep_f32_copy;
  M->perm = t.perm;
  upload(M->d_perm, M->perm, s);

  // permuted geometry, SoA FP64
  std::vector<double> geo(7 * n);
  for (int64_t k = 0; k < n; ++k) {
    const int64_t o = t.perm[k];
    for (int a = 0; a < 3; ++a) {
      geo[a * n + k] = t.c[3 * o + a];
      geo[(3 + a) * n + k] = t.nrm[3 * o + a];
    }
    geo[6 * n + k] = t.area[o];
  }
  DevBuf d_geo;
  upload(d_geo, geo, s);
  const double* gp = d_geo.get<double>();
  Geo g{gp, gp + n, gp + 2 * n, gp + 3 * n, gp + 4 * n, gp + 5 * n, gp + 6 * n};

  // ---- ACA on the admissible blocks, in batches bounded by a scratch budget
  const int kmax = std::min<int>(p.k_max, ACA_KMAX);
  size_t free_b = 0, total_b = 0;
  HM_HIP(hipMemGetInfo(&free_b, &total_b));
  const int64_t budget = std::max<int64_t>(256ll << 20, std::min<int64_t>(8ll << 30, (int64_t)free_b / 4));
  std::vector<int32_t> order(t.lowrank.size());
  for (size_t q = 0; q < order.size(); ++q) order[q] = (int32_t)q;
  std::vector<LrInfo> lr;
  std::vector<DnInfo> dn;
  for (const auto& b : t.dense) dn.push_back(DnInfo{b, 0});
  struct Stage { DevBuf U, V, Uhi, Vhi; int64_t nu, nv; };
  std::vector<Stage> stages;
  std::vector<int64_t> lr_stage_u, lr_stage_v;  // offsets inside the stage; fixed up below
  std::vector<int32_t> lr_stage;
  const size_t es = dtype_size(p.lowrank_dtype);
  DevBuf scratch, flags, d_blk, d_rank, d_status, d_cd;
  size_t pos = 0;
  while (pos < order.size()) {
    std::vector<AcaDev> batch;
    int64_t sd = 0, sf = 0;
    while (pos < order.size()) {
      const BlockRef& b = t.lowrank[order[pos]];
      const int m = b.re - b.rb, nn = b.ce - b.cb;
      const int64_t kc = rank_cap(m, nn, kmax);
      const int64_t need = kc * (m + nn) * 8 + m * 4;
      if (!batch.empty() && (sd * 8 + sf * 4 + need) > budget) break;
      AcaDev a{b.rb, b.re, b.cb, b.ce, (int32_t)kc, 0, sd, sd + kc * m, sf};
      sd += kc * (m + nn);
      sf += m;
      batch.push_back(a);
      ++pos;
    }
    // largest blocks first for the hardware dispatcher
    std::vector<int32_t> bidx(batch.size());
    for (size_t q = 0; q < bidx.size(); ++q) bidx[q] = (int32_t)q;
    std::vector<AcaDev> sorted(batch.size());
    std::stable_sort(bidx.begin(), bidx.end(), [&](int32_t x, int32_t y) {
      return (int64_t)(batch[x].re - batch[x].rb) * (batch[x].ce - batch[x].cb) >
             (int64_t)(batch[y].re - batch[y].rb) * (batch[y].ce - batch[y].cb);
    });
    for (size_t q = 0; q < bidx.size(); ++q) sorted[q] = batch[bidx[q]];
    if ((size_t)sd * 8 > scratch.bytes()) scratch.alloc((size_t)sd * 8);
    if ((size_t)sf * 4 > flags.bytes()) flags.alloc((size_t)sf * 4);
    upload(d_blk, sorted, s);
    d_rank.alloc(sorted.size() * 4);
    d_status.alloc(sorted.size() * 4);
    hipLaunchKernelGGL(k_aca, dim3((unsigned)sorted.size()), dim3(ACA_T), 0, s, d_blk.get<AcaDev>(), g, p.aca_tol,
                       scratch.get<double>(), flags.get<int>(), d_rank.get<int>(), d_status.get<int>());
    HM_HIP(hipGetLastError());
    std::vector<int> rk(sorted.size()), st(sorted.size());
    HM_HIP(hipMemcpyAsync(rk.data(), d_rank.get(), rk.size() * 4, hipMemcpyDeviceToHost, s));
    HM_HIP(hipMemcpyAsync(st.data(), d_status.get(), st.size() * 4, hipMemcpyDeviceToHost, s));
    HM_HIP(hipStreamSynchronize(s));
    // classify: low rank (k(m+n) < mn and converged), rank zero (dropped), dense fallback
    std::vector<CompactDev> cd;
    Stage stg;
    stg.nu = stg.nv = 0;
    for (size_t q = 0; q < sorted.size(); ++q) {
      const AcaDev& a = sorted[q];
      const int m = a.re - a.rb, nn = a.ce - a.cb;
      const int k = rk[q];
      BlockRef br{a.rb, a.re, a.cb, a.ce};
      if (!st[q] || (int64_t)k * (m + nn) >= (int64_t)m * nn) {
        dn.push_back(DnInfo{br, 0});
        M->n_fallback++;
        continue;
      }
      if (k == 0) continue;  // exactly zero block
      cd.push_back(CompactDev{a.u_off, a.v_off, stg.nu, stg.nv, m, nn, k, 0});
      lr.push_back(LrInfo{br, k, stg.nu, stg.nv});
      lr_stage.push_back((int32_t)stages.size());
      stg.nu += (int64_t)m * k;
      stg.nv += (int64_t)nn * k;
    }
    if (!cd.empty()) {
      stg.U.alloc(stg.nu * es);
      stg.V.alloc(stg.nv * es);
      if (M->has_hi) {
        stg.Uhi.alloc(stg.nu * 4);
        stg.Vhi.alloc(stg.nv * 4);
      }
      upload(d_cd, cd, s);
      dispatch_dtype(p.lowrank_dtype, [&](auto* tag) {
        using OT = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(k_compact<OT>, dim3((unsigned)cd.size()), dim3(256), 0, s, d_cd.get<CompactDev>(),
                           scratch.get<double>(), stg.U.get<OT>(), stg.V.get<OT>(), stg.Uhi.get<float>(),
                           stg.Vhi.get<float>());
      });
      HM_HIP(hipGetLastError());
      HM_HIP(hipStreamSynchronize(s));  // scratch is reused by the next batch
    }
    stages.push_back(std::move(stg));
  }
  scratch.release();
  flags.release();

  // ---- consolidate the factor stages into one U and one V arena
  std::vector<int64_t> su(stages.size() + 1, 0), sv(stages.size() + 1, 0);
  for (size_t q = 0; q < stages.size(); ++q) {
    su[q + 1] = su[q] + stages[q].nu;
    sv[q + 1] = sv[q] + stages[q].nv;
  }
  M->U.alloc(su.back() * es);
  M->V.alloc(sv.back() * es);
  if (M->has_hi) {
    M->U_hi.alloc(su.back() * 4);
    M->V_hi.alloc(sv.back() * 4);
  }
  for (size_t q = 0; q < stages.size(); ++q) {
    if (stages[q].nu == 0) continue;
    HM_HIP(hipMemcpyAsync(M->U.get<char>() + su[q] * es, stages[q].U.get(), stages[q].nu * es, hipMemcpyDeviceToDevice, s));
    HM_HIP(hipMemcpyAsync(M->V.get<char>() + sv[q] * es, stages[q].V.get(), stages[q].nv * es, hipMemcpyDeviceToDevice, s));
    if (M->has_hi) {
      HM_HIP(hipMemcpyAsync(M->U_hi.get<char>() + su[q] * 4, stages[q].Uhi.get(), stages[q].nu * 4, hipMemcpyDeviceToDevice, s));
      HM_HIP(hipMemcpyAsync(M->V_hi.get<char>() + sv[q] * 4, stages[q].Vhi.get(), stages[q].nv * 4, hipMemcpyDeviceToDevice, s));
    }
  }
  for (size_t q = 0; q < lr.size(); ++q) {
    lr[q].u_off += su[lr_stage[q]];
    lr[q].v_off += sv[lr_stage[q]];
  }
  HM_HIP(hipStreamSynchronize(s));
  stages.clear();

  // ---- dense near field (tree-dense blocks and ACA fallbacks)
  int64_t doff = 0;
  std::vector<DnDev> dd;
  for (auto& d : dn) {
    d.off = doff;
    doff += (int64_t)(d.b.re - d.b.rb) * (d.b.ce - d.b.cb);
    dd.push_back(DnDev{d.b.rb, d.b.re, d.b.cb, d.b.ce, d.off});
  }
  const size_t ds = dtype_size(p.dense_dtype);
  M->dense.alloc(doff * ds);
  if (!dd.empty()) {
    DevBuf d_dd;
    upload(d_dd, dd, s);
    if (p.dense_dtype == HM_F64)
      hipLaunchKernelGGL(k_nearfield<double>, dim3((unsigned)dd.size()), dim3(256), 0, s, d_dd.get<DnDev>(), g,
                         M->dense.get<double>());
    else
      hipLaunchKernelGGL(k_nearfield<float>, dim3((unsigned)dd.size()), dim3(256), 0, s, d_dd.get<DnDev>(), g,
                         M->dense.get<float>());
    HM_HIP(hipGetLastError());
    HM_HIP(hipStreamSynchronize(s));
  }

  // ---- statistics
  M->dense_entries = doff;
  M->n_dense_blocks = (int64_t)dn.size();
  M->n_lr_blocks = (int64_t)lr.size();
  int64_t ktot = 0, lre = 0;
  for (const auto& l : lr) {
    ktot += l.k;
    lre += (int64_t)l.k * ((l.b.re - l.b.rb) + (l.b.ce - l.b.cb));
    M->u_entries += (int64_t)l.k * (l.b.re - l.b.rb);
    M->v_entries += (int64_t)l.k * (l.b.ce - l.b.cb);
    M->max_rank = std::max(M->max_rank, l.k);
  }
  M->Ktot = ktot;
  M->rank_sum = ktot;
  M->lr_entries = lre;

  build_plan(*M, lr, dn, t, s);
  if (p.closed_row_scale) closed_row_scale(*M, dn, lr, s);
  HM_HIP(hipStreamSynchronize(s));
  return M.release();
}

void apply_row_scale(hm_matrix& M, const std::vector<DnInfo>& dn, const std::vector<LrInfo>& lr,
                     const double* d_scale, hipStream_t s) {
  std::vector<ScaleDev> sd;
  for (const auto& d : dn)
    sd.push_back(ScaleDev{d.off, d.b.rb, d.b.re - d.b.rb, d.b.ce - d.b.cb, 0});
  for (const auto& l : lr) sd.push_back(ScaleDev{l.u_off, l.b.rb, l.b.re - l.b.rb, l.k, 1});
  if (sd.empty()) return;
  DevBuf d_sd;
  upload(d_sd, sd, s);
  auto go = [&](auto* dt, auto* lt) {
    using DT = std::remove_pointer_t<decltype(dt)>;
    using LT = std::remove_pointer_t<decltype(lt)>;
    hipLaunchKernelGGL((k_rowscale<DT, LT>), dim3((unsigned)sd.size()), dim3(256), 0, s, d_sd.get<ScaleDev>(),
                       d_scale, M.dense.get<DT>(), M.U.get<LT>(), M.has_hi ? M.U_hi.get<float>() : nullptr);
  };
  if (M.dense_dtype == HM_F64) {
    if (M.lr_dtype == HM_F64) go((double*)0, (double*)0);
    else if (M.lr_dtype == HM_F32) go((double*)0, (float*)0);
    else go((double*)0, (bf16_t*)0);
  } else {
    if (M.lr_dtype == HM_F64) go((float*)0, (double*)0);
    else if (M.lr_dtype == HM_F32) go((float*)0, (float*)0);
    else go((float*)0, (bf16_t*)0);
  }
  HM_HIP(hipGetLastError());
  HM_HIP(hipStreamSynchronize(s));
}

// Closed-cavity treatment (eqs. (32)-(34)): s = F_H 1 (the per-area row sum),
// c = clamp(s, 0, 1), rows with c != 0 divided by c.
void closed_row_scale(hm_matrix& M, const std::vector<DnInfo>& dn, const std::vector<LrInfo>& lr, hipStream_t s) {
  const int64_t n = M.n;
  DevBuf ones(n * 8), rs(n * 8), scale(n * 8);
  std::vector<double> h(n, 1.0);
  HM_HIP(hipMemcpyAsync(ones.get(), h.data(), n * 8, hipMemcpyHostToDevice, s));
  auto comp = make_composition({&M}, 1, 8, s);
  // the row sum is the same in either order: x = 1 is permutation invariant
  launch_matvec(*comp, 1, 8, M.has_hi, ones.get(), n, rs.get(), n, Epilogue{}, nullptr, s);
  hipLaunchKernelGGL(k_closed_scale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rs.get<double>(),
                     scale.get<double>(), n);
  HM_HIP(hipGetLastError());
  apply_row_scale(M, dn, lr, scale.get<double>(), s);
}

}  // namespace hm
