// H-matrix assembly on gfx950: centroid-rule view factors (eq. (10)), the
// dense near field of the inadmissible leaves, and adaptive cross
// approximation (Sec. 4.3, eqs. (30)-(31)) of the admissible leaves.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "dev_common.hpp"
#include "hm_internal.hpp"
#include "recompress.hpp"

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

struct AcaDev {
  int32_t rb, re, cb, ce;
  int32_t kcap, out;            // rank cap; index of the block's rank/status outputs
  int64_t u_off, v_off, f_off;  // scratch offsets (doubles, doubles, ints)
  int64_t r_off;                // full pivoting: scratch offset of the m x n residual (doubles)
  double tol;                   // relative ACA tolerance of the block's cavity
};

constexpr int ACA_T = 256;        // threads per workgroup of k_aca
constexpr int ACA_T_HUGE = 512;   // ... for blocks with m + n >= ACA_HUGE
constexpr int64_t ACA_FULL_BIG = 1 << 18;  // fully pivoted ACA: blocks of this many entries and more
                                           // run each pass over many workgroups
constexpr int ACA_HUGE = 4096;
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

template <int W>
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
  for (int w = 1; w < W; ++w) r = better(r, sh[w]);
  return r;
}

// Sum of NV values over the W waves of the workgroup, fixed order.
template <int W, int NV>
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
    for (int w = 1; w < W; ++w) s += sh[w * NV + q];
    v[q] = s;
  }
}

#pragma clang fp contract(off)
// r - sum_{l < k} c[l] P[l ld + j], subtracted one term at a time in the order
// of l; the loads go out eight at a time so their latencies overlap (the
// same operations as the plain loop, so the same result bit for bit).
__device__ __forceinline__ double sub_terms(double r, const double* c, const double* __restrict__ P, int64_t ld,
                                            int j, int k) {
  int l = 0;
  for (; l + 8 <= k; l += 8) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = P[(int64_t)(l + q) * ld + j];
#pragma unroll
    for (int q = 0; q < 8; ++q) r = r - c[l + q] * v[q];
  }
  for (; l < k; ++l) r = r - c[l] * P[(int64_t)l * ld + j];
  return r;
}

// Partial-pivoting ACA of one admissible block per workgroup of T threads,
// in FP64.  U (m x kcap) and V (n x kcap) are column-major scratch; on exit
// rank[b] holds k and status[b] is 1 when the stop test |u||v| <= tol
// |sum u v^T|_F was met (0 when the rank cap was reached first).  The
// crosses of a block are sequential, so a launch lasts as long as its
// largest blocks: those get T = 512 (8 waves, two per SIMD; each cross's row
// and column work spread twice as wide; 1024 threads would spill at the
// 128 registers they leave a thread), the others T = 256.
template <int T>
__global__ __launch_bounds__(T) void k_aca(const AcaDev* __restrict__ blocks, Geo g,
                                           double* __restrict__ scratch, int* __restrict__ flags,
                                           int* __restrict__ rank, int* __restrict__ status) {
  constexpr int ACA_T = T, ACA_W = T / 64;
  __shared__ double coef[ACA_KMAX];
  __shared__ ArgMax sh_am[ACA_W];
  __shared__ double sh_sum[ACA_W * 16];
  const AcaDev b = blocks[blockIdx.x];
  const double tol = b.tol;
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
      const double r = sub_terms(view_factor(g, b.rb + i, b.cb + j), coef, V, n, j, k);
      vk[j] = r;
      const double a = fabs(r);
      if (a > am.mag || (a == am.mag && j < am.idx)) am = ArgMax{a, r, j};
    }
    am = block_argmax<ACA_W>(am, sh_am);
    const int jp = am.idx;
    const double rj = am.val;
    if (rj == 0.0) {
      // zero residual row: mark it used and move to the smallest unused row
      if (tid == 0) used[i] = 1;
      __syncthreads();
      ArgMax nx{-1.0, 0.0, 0x7fffffff};
      for (int ii = tid; ii < m; ii += ACA_T)
        if (!used[ii] && ii < nx.idx) nx = ArgMax{0.0, 0.0, ii};
      nx = block_argmax<ACA_W>(nx, sh_am);
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
      const double u = sub_terms(view_factor(g, b.rb + ii, b.cb + jp), coef, U, m, ii, k);
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
      block_sum<ACA_W, 2>(t2, sh_sum);
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
      block_sum<ACA_W, 16>(d, sh_sum);
      for (int q = 0; q < nl; ++q) cross += d[q] * d[8 + q];
    }
    s2 += nu2 * nv2 + 2.0 * cross;
    ++k;
    if (sqrt(nu2 * nv2) <= tol * sqrt(fmax(s2, 0.0))) { conv = 1; break; }
    if (k >= b.kcap) { conv = 0; break; }
    nx = block_argmax<ACA_W>(nx, sh_am);
    if (nx.idx == 0x7fffffff) { conv = 1; break; }
    i = nx.idx;
  }
  if (tid == 0) {
    rank[b.out] = k;
    status[b.out] = conv;
  }
}

// ---- one wave per small block (m, n <= 64, rank cap <= ACAW_K): the same
// steps as k_aca, lane = row for U and lane = column for V, the factors and
// the geometry of the lane's row and column in registers, the pivot row's
// and column's values handed to all lanes by broadcast.  For such blocks
// k_aca's data lives in its first wave (thread = row / column index) and its
// other waves add zeros, so both kernels take the same pivots and ranks and
// produce the same factors bit for bit.
constexpr int ACAW_K = 32;

__device__ __forceinline__ double bcast_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline ArgMax wave_argmax(ArgMax v) {
  for (int o = 32; o > 0; o >>= 1) {
    ArgMax w;
    w.mag = __shfl_xor(v.mag, o, 64);
    w.val = __shfl_xor(v.val, o, 64);
    w.idx = __shfl_xor(v.idx, o, 64);
    v = better(v, w);
  }
  return v;
}

// view_factor's operations in its order, on geometry held in registers
__device__ __forceinline__ double view_factor_r(double icx, double icy, double icz, double inx, double iny,
                                                double inz, double jcx, double jcy, double jcz, double jnx,
                                                double jny, double jnz, double jar, bool same) {
  if (same) return 0.0;
  const double dx = jcx - icx;
  const double dy = jcy - icy;
  const double dz = jcz - icz;
  const double r2 = (dx * dx + dy * dy) + dz * dz;
  const double ci = (inx * dx + iny * dy) + inz * dz;
  const double cj = -((jnx * dx + jny * dy) + jnz * dz);
  const double num = fmax(ci, 0.0) * fmax(cj, 0.0) * jar;
  const double den = (3.141592653589793 * r2) * r2;
  return r2 > 0.0 ? num / den : 0.0;
}

__global__ __launch_bounds__(256) void k_aca_wave(const AcaDev* __restrict__ blocks, int nblk, Geo g,
                                                  double* __restrict__ scratch, int* __restrict__ rank,
                                                  int* __restrict__ status) {
  const int lane = threadIdx.x & 63;
  const int bi = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (bi >= nblk) return;
  const AcaDev b = uniform_load(blocks + bi);
  const double tol = b.tol;
  const int m = b.re - b.rb, n = b.ce - b.cb;
  // geometry of the lane's row (rows past m repeat the last) and column
  const int ri = b.rb + min(lane, m - 1), cj = b.cb + min(lane, n - 1);
  const double rcx = g.cx[ri], rcy = g.cy[ri], rcz = g.cz[ri], rnx = g.nx[ri], rny = g.ny[ri], rnz = g.nz[ri];
  const double ccx = g.cx[cj], ccy = g.cy[cj], ccz = g.cz[cj], cnx = g.nx[cj], cny = g.ny[cj], cnz = g.nz[cj];
  const double car = g.ar[cj];
  double U[ACAW_K], V[ACAW_K];
#pragma unroll
  for (int l = 0; l < ACAW_K; ++l) U[l] = V[l] = 0.0;
  bool used = false;
  int i = 0, k = 0, conv = 0;
  double s2 = 0.0;
  for (;;) {
    // residual row i (lane = column j)
    const double icx = bcast_d(rcx, i), icy = bcast_d(rcy, i), icz = bcast_d(rcz, i);
    const double inx = bcast_d(rnx, i), iny = bcast_d(rny, i), inz = bcast_d(rnz, i);
    double r = view_factor_r(icx, icy, icz, inx, iny, inz, ccx, ccy, ccz, cnx, cny, cnz, car, b.rb + i == cj);
#pragma unroll
    for (int l = 0; l < ACAW_K; ++l)
      if (l < k) r = r - bcast_d(U[l], i) * V[l];
    ArgMax am = lane < n ? ArgMax{fabs(r), r, lane} : ArgMax{-1.0, 0.0, 0x7fffffff};
    am = wave_argmax(am);
    const int jp = __builtin_amdgcn_readfirstlane(am.idx);
    const double rj = am.val;
    if (rj == 0.0) {
      // zero residual row: mark it used and move to the smallest unused row
      if (lane == i) used = true;
      const unsigned long long bal = __ballot(lane < m && !used);
      if (bal == 0ull) {
        conv = 1;
        break;
      }
      i = __ffsll((long long)bal) - 1;
      continue;
    }
    const double v = lane < n ? r / rj : 0.0;
    // residual column jp (lane = row)
    const double jcx = bcast_d(ccx, jp), jcy = bcast_d(ccy, jp), jcz = bcast_d(ccz, jp);
    const double jnx = bcast_d(cnx, jp), jny = bcast_d(cny, jp), jnz = bcast_d(cnz, jp), jar = bcast_d(car, jp);
    double u = view_factor_r(rcx, rcy, rcz, rnx, rny, rnz, jcx, jcy, jcz, jnx, jny, jnz, jar, ri == b.cb + jp);
#pragma unroll
    for (int l = 0; l < ACAW_K; ++l)
      if (l < k) u = u - bcast_d(V[l], jp) * U[l];
    if (lane >= m) u = 0.0;
    if (lane == i) used = true;
    const double nu2 = wave_sum(u * u), nv2 = wave_sum(v * v);
    double cross = 0.0;
#pragma unroll
    for (int l = 0; l < ACAW_K; ++l)
      if (l < k) cross += wave_sum(U[l] * u) * wave_sum(V[l] * v);
    s2 += nu2 * nv2 + 2.0 * cross;
#pragma unroll
    for (int l = 0; l < ACAW_K; ++l)
      if (l == k) {
        U[l] = u;
        V[l] = v;
      }
    ++k;
    if (sqrt(nu2 * nv2) <= tol * sqrt(fmax(s2, 0.0))) {
      conv = 1;
      break;
    }
    if (k >= b.kcap) {
      conv = 0;
      break;
    }
    ArgMax nx = (lane < m && !used) ? ArgMax{fabs(u), u, lane} : ArgMax{-1.0, 0.0, 0x7fffffff};
    nx = wave_argmax(nx);
    if (nx.idx == 0x7fffffff) {
      conv = 1;
      break;
    }
    i = __builtin_amdgcn_readfirstlane(nx.idx);
  }
  double* Us = scratch + b.u_off;
  double* Vs = scratch + b.v_off;
#pragma unroll
  for (int l = 0; l < ACAW_K; ++l)
    if (l < k) {
      if (lane < m) Us[(int64_t)l * m + lane] = U[l];
      if (lane < n) Vs[(int64_t)l * n + lane] = V[l];
    }
  if (lane == 0) {
    rank[b.out] = k;
    status[b.out] = conv;
  }
}
#pragma clang fp contract(on)

// ---- fully pivoted ACA (the paper's pivoting), one workgroup per block:
// the block is evaluated into a column-major m x n residual R in scratch;
// each cross takes the entry of largest |R| (smallest row-major index i n + j
// on ties) as pivot, u = R(:, j), v = R(i, :) / R(i, j), and R <- R - u v^T
// entry by entry (one product and one subtraction, no contraction, as the
// oracle's R - outer(u, v)), while the same pass finds the next pivot and
// |R|_F^2.  The stop test is eq. (31) on the exact residual:
// |R|_F <= tol |X|_F (or a zero residual, or the rank cap).
#pragma clang fp contract(off)
constexpr int FULL_U = 8;  // residual entries per thread in flight
template <int T>
__global__ __launch_bounds__(T) void k_aca_full(const AcaDev* __restrict__ blocks, Geo g,
                                                double* __restrict__ scratch, int* __restrict__ rank,
                                                int* __restrict__ status) {
  constexpr int W = T / 64;
  __shared__ ArgMax sh_am[W];
  __shared__ double sh_sum[W];
  const AcaDev b = blocks[blockIdx.x];
  const int m = b.re - b.rb, n = b.ce - b.cb;
  const int64_t mn = (int64_t)m * n;
  double* R = scratch + b.r_off;
  double* U = scratch + b.u_off;
  double* V = scratch + b.v_off;
  const int tid = threadIdx.x;
  // a thread visits entries e = tid, tid + T, ... (i = e mod m, j = e / m):
  // its row and column advance by T mod m and T / m per visit
  const int di = T % m, dj = T / m;
  const int i0 = tid % m, j0 = tid / m;
  ArgMax am{-1.0, 0.0, 0x7fffffff};
  double s2 = 0.0;
  int i = i0, j = j0;
  for (int64_t e = tid; e < mn; e += T) {
    const double x = view_factor(g, b.rb + i, b.cb + j);
    R[e] = x;
    s2 += x * x;
    const double a = fabs(x);
    const int key = i * n + j;
    if (a > am.mag || (a == am.mag && key < am.idx)) am = ArgMax{a, x, key};
    i += di;
    j += dj;
    if (i >= m) {
      i -= m;
      ++j;
    }
  }
  {
    double t[1] = {s2};
    block_sum<W, 1>(t, sh_sum);
    s2 = t[0];
  }
  am = block_argmax<W>(am, sh_am);
  const double limit = b.tol * sqrt(s2);
  int k = 0, conv = 0;
  for (;;) {
    if (am.idx == 0x7fffffff || am.val == 0.0) {
      conv = 1;  // zero residual: the crosses so far are exact
      break;
    }
    const int ip = am.idx / n, jp = am.idx % n;
    const double piv = am.val;
    double* uk = U + (int64_t)k * m;
    double* vk = V + (int64_t)k * n;
    for (int r = tid; r < m; r += T) uk[r] = R[(int64_t)jp * m + r];
    for (int c = tid; c < n; c += T) vk[c] = R[(int64_t)c * m + ip] / piv;
    __syncthreads();
    am = ArgMax{-1.0, 0.0, 0x7fffffff};
    double r2 = 0.0;
    i = i0;
    j = j0;
    // FULL_U of the thread's entries at a time: all their loads go out
    // before the first is used (one workgroup streams a block of up to
    // millions of entries per cross); they are then taken in the same
    // order as one at a time, so sums and pivots do not change
    for (int64_t e = tid; e < mn; e += (int64_t)FULL_U * T) {
      double rv[FULL_U], uv[FULL_U], vv[FULL_U];
      int key[FULL_U];
#pragma unroll
      for (int u = 0; u < FULL_U; ++u) {
        const bool in = e + (int64_t)u * T < mn;  // then i < m and j < n
        key[u] = in ? i * n + j : 0;
        rv[u] = in ? R[e + (int64_t)u * T] : 0.0;
        uv[u] = in ? uk[i] : 0.0;
        vv[u] = in ? vk[j] : 0.0;
        i += di;
        j += dj;
        if (i >= m) {
          i -= m;
          ++j;
        }
      }
#pragma unroll
      for (int u = 0; u < FULL_U; ++u) {
        if (e + (int64_t)u * T >= mn) break;
        const double r = rv[u] - uv[u] * vv[u];
        R[e + (int64_t)u * T] = r;
        r2 += r * r;
        const double a = fabs(r);
        if (a > am.mag || (a == am.mag && key[u] < am.idx)) am = ArgMax{a, r, key[u]};
      }
    }
    {
      double t[1] = {r2};
      block_sum<W, 1>(t, sh_sum);
      r2 = t[0];
    }
    am = block_argmax<W>(am, sh_am);
    ++k;
    if (sqrt(r2) <= limit) {
      conv = 1;
      break;
    }
    if (k >= b.kcap) {
      conv = 0;
      break;
    }
  }
  if (tid == 0) {
    rank[b.out] = k;
    status[b.out] = conv;
  }
}

// ---- fully pivoted ACA of the largest blocks, each pass over a block's
// residual spread over many workgroups: slices of FULL_SLICE entries write
// their partial |R|_F^2 and pivot candidate, and one finishing workgroup
// per block adds the partials in slice order, takes the pivot, applies the
// stop test and copies the next cross.  These are k_aca_full's steps and
// entry arithmetic (so the same pivots); only the order in which the norm's
// partial sums are added differs.
constexpr int FULL_T = 256;
constexpr int FULL_SLICE = FULL_T * FULL_U * 16;  // entries per slice
struct FullState {
  double limit;  // tol |X|_F
  int32_t k;     // current cross (its u, v are column k of U, V)
  int32_t done;  // 1 once the block has finished (rank and status written)
};
struct FullSlice {
  int32_t blk, s;  // block (index in the launch's list) and slice within it
};

// Slice pass: the first evaluation of the block (EVAL) or the update of its
// residual by the current cross; partial |R|_F^2 and pivot candidate to
// part2[slice], pam[slice].
template <bool EVAL>
__global__ __launch_bounds__(FULL_T) void k_full_pass(const AcaDev* __restrict__ blocks,
                                                      const FullSlice* __restrict__ slices,
                                                      const FullState* __restrict__ state, Geo g,
                                                      double* __restrict__ scratch, double* __restrict__ part2,
                                                      ArgMax* __restrict__ pam) {
  constexpr int T = FULL_T, W = T / 64;
  __shared__ ArgMax sh_am[W];
  __shared__ double sh_sum[W];
  const FullSlice q = slices[blockIdx.x];
  if (!EVAL && state[q.blk].done) return;  // uniform over the workgroup
  const AcaDev b = blocks[q.blk];
  const int m = b.re - b.rb, n = b.ce - b.cb;
  const int64_t mn = (int64_t)m * n;
  const int64_t e0 = (int64_t)q.s * FULL_SLICE;
  const int64_t e1 = e0 + FULL_SLICE < mn ? e0 + FULL_SLICE : mn;
  double* R = scratch + b.r_off;
  const int tid = threadIdx.x;
  const int64_t et = e0 + tid;
  const int64_t ec = et < mn ? et : mn - 1;  // a thread past the slice visits nothing
  const int di = T % m, dj = T / m;
  int i = (int)(ec % m), j = (int)(ec / m);
  ArgMax am{-1.0, 0.0, 0x7fffffff};
  double s2 = 0.0;
  if (EVAL) {
    for (int64_t e = et; e < e1; e += T) {
      const double x = view_factor(g, b.rb + i, b.cb + j);
      R[e] = x;
      s2 += x * x;
      const double a = fabs(x);
      const int key = i * n + j;
      if (a > am.mag || (a == am.mag && key < am.idx)) am = ArgMax{a, x, key};
      i += di;
      j += dj;
      if (i >= m) {
        i -= m;
        ++j;
      }
    }
  } else {
    const int k = state[q.blk].k;
    const double* uk = scratch + b.u_off + (int64_t)k * m;
    const double* vk = scratch + b.v_off + (int64_t)k * n;
    for (int64_t e = et; e < e1; e += (int64_t)FULL_U * T) {
      double rv[FULL_U], uv[FULL_U], vv[FULL_U];
      int key[FULL_U];
#pragma unroll
      for (int u = 0; u < FULL_U; ++u) {
        const bool in = e + (int64_t)u * T < e1;  // then i < m and j < n
        key[u] = in ? i * n + j : 0;
        rv[u] = in ? R[e + (int64_t)u * T] : 0.0;
        uv[u] = in ? uk[i] : 0.0;
        vv[u] = in ? vk[j] : 0.0;
        i += di;
        j += dj;
        if (i >= m) {
          i -= m;
          ++j;
        }
      }
#pragma unroll
      for (int u = 0; u < FULL_U; ++u) {
        if (e + (int64_t)u * T >= e1) break;
        const double r = rv[u] - uv[u] * vv[u];
        R[e + (int64_t)u * T] = r;
        s2 += r * r;
        const double a = fabs(r);
        if (a > am.mag || (a == am.mag && key[u] < am.idx)) am = ArgMax{a, r, key[u]};
      }
    }
  }
  {
    double t[1] = {s2};
    block_sum<W, 1>(t, sh_sum);
    s2 = t[0];
  }
  am = block_argmax<W>(am, sh_am);
  if (tid == 0) {
    part2[blockIdx.x] = s2;
    pam[blockIdx.x] = am;
  }
}

// Finishing step of a block after a slice pass: the partials of its slices
// [first[b], first[b + 1]) added in a fixed order; after the first pass the
// limit tol |X|_F, after an update the cross count, the stop test of eq.
// (31) and the rank cap; then, unless finished, the next cross u = R(:, jp),
// v = R(ip, :) / R(ip, jp) into column k of U and V.
template <bool INIT>
__global__ __launch_bounds__(FULL_T) void k_full_fin(const AcaDev* __restrict__ blocks, const int* __restrict__ first,
                                                     FullState* __restrict__ state, double* __restrict__ scratch,
                                                     const double* __restrict__ part2,
                                                     const ArgMax* __restrict__ pam, int* __restrict__ rank,
                                                     int* __restrict__ status) {
  constexpr int T = FULL_T, W = T / 64;
  __shared__ ArgMax sh_am[W];
  __shared__ double sh_sum[W];
  const int qb = blockIdx.x;
  FullState st = state[qb];
  if (!INIT && st.done) return;  // uniform
  const AcaDev b = blocks[qb];
  const int m = b.re - b.rb, n = b.ce - b.cb;
  const int tid = threadIdx.x;
  double r2 = 0.0;
  ArgMax am{-1.0, 0.0, 0x7fffffff};
  for (int s = first[qb] + tid; s < first[qb + 1]; s += T) {
    r2 += part2[s];
    am = better(am, pam[s]);
  }
  {
    double t[1] = {r2};
    block_sum<W, 1>(t, sh_sum);
    r2 = t[0];
  }
  am = block_argmax<W>(am, sh_am);
  const int k = INIT ? 0 : st.k + 1;
  const double limit = INIT ? b.tol * sqrt(r2) : st.limit;
  int done = 0, conv = 0;
  if (!INIT && sqrt(r2) <= limit) {
    done = 1;
    conv = 1;
  } else if (!INIT && k >= b.kcap) {
    done = 1;
  } else if (am.idx == 0x7fffffff || am.val == 0.0) {
    done = 1;
    conv = 1;  // zero residual: the crosses so far are exact
  }
  if (!done) {
    const int ip = am.idx / n, jp = am.idx % n;
    const double piv = am.val;
    const double* R = scratch + b.r_off;
    double* uk = scratch + b.u_off + (int64_t)k * m;
    double* vk = scratch + b.v_off + (int64_t)k * n;
    for (int r = tid; r < m; r += T) uk[r] = R[(int64_t)jp * m + r];
    for (int c = tid; c < n; c += T) vk[c] = R[(int64_t)c * m + ip] / piv;
  }
  if (tid == 0) {
    state[qb] = FullState{limit, k, done};
    if (done) {
      rank[b.out] = k;
      status[b.out] = conv;
    }
  }
}
#pragma clang fp contract(on)

struct CompactDev {
  int64_t su, sv;   // scratch offsets of U, V (doubles)
  int64_t du, dv;   // destination offsets (elements) in the stage buffer
  int32_t m, n, k, pad;
};

// Copy the first k columns of the FP64 scratch factors into a stage buffer
// (FP64 for FP64 storage, FP32 otherwise).
template <class ST>
__global__ __launch_bounds__(256) void k_compact(const CompactDev* __restrict__ cd, const double* __restrict__ scratch,
                                                 ST* __restrict__ stage) {
  const CompactDev c = cd[blockIdx.x];
  const int64_t nu = (int64_t)c.m * c.k, nv = (int64_t)c.n * c.k;
  for (int64_t e = threadIdx.x; e < nu; e += blockDim.x) stage[c.du + e] = (ST)scratch[c.su + e];
  for (int64_t e = threadIdx.x; e < nv; e += blockDim.x) stage[c.dv + e] = (ST)scratch[c.sv + e];
}

// Near field straight into the phase-2 panels: element (r, c) of the segment
// goes to base + ((col / 4) * m + r) * 4 + col % 4 with col = col0 + c.
template <class OT>
__global__ __launch_bounds__(256) void k_nf_pack(const NfDev* __restrict__ nf, Geo g, OT* __restrict__ out) {
  const NfDev d = nf[blockIdx.x];
  const int64_t tot = (int64_t)d.m * d.w;
  for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
    const int r = (int)(e % d.m), c = (int)(e / d.m);
    const int col = d.col0 + c;
    out[d.base + ((int64_t)(col >> 2) * d.m + r) * 4 + (col & 3)] =
        Cvt<OT>::from_f64(view_factor(g, d.row0 + r, d.cb + c));
  }
}

// BF16 near field from its FP32 copy (round to nearest even), so that the
// two hold the same rounding of each view factor as the low-rank factors.
__global__ __launch_bounds__(256) void k_to_bf16(const float* __restrict__ in, bf16_t* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = f32_to_bf16(in[i]);
}

// U factor rows of one tile into a phase-2 panel (storage type and FP32 copy).
// Storage rounding of a factor entry: nearest even, or dithered (BF16
// storage only) with the draw keyed by the entry.
template <class OT>
__device__ __forceinline__ OT round_factor(double x, bool dither, uint32_t side, uint32_t idx, uint32_t other,
                                           uint32_t l) {
  if constexpr (std::is_same<OT, bf16_t>::value) {
    if (dither) return f32_to_bf16_dither((float)x, dither_draw16(side, idx, other, l));
  }
  return Cvt<OT>::from_f64(x);
}

template <class ST, class OT>
__global__ __launch_bounds__(256) void k_u_pack(const URepack* __restrict__ ur, const void* const* __restrict__ stages,
                                                OT* __restrict__ out, float* __restrict__ out_hi, int dither) {
  const URepack d = ur[blockIdx.x];
  const ST* src = (const ST*)stages[d.stage] + d.src;
  const int64_t tot = (int64_t)d.m * d.k;
  for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
    const int r = (int)(e % d.m), c = (int)(e / d.m);
    const int col = d.col0 + c;
    const double x = (double)src[(int64_t)c * d.ld + r];
    const int64_t o = d.base + ((int64_t)(col >> 2) * d.m + r) * 4 + (col & 3);
    out[o] = round_factor<OT>(x, dither != 0, 1u, (uint32_t)(d.row0 + r), (uint32_t)d.cb, (uint32_t)(d.l0 + c));
    if (out_hi) out_hi[o] = (float)x;
  }
}

// V factor of one block into the group panels of its column cluster:
// element (r, l) goes to group g = pc / 64 (pc = lc0 + l), at
// ((r / 4) * gw + pc % 64) * 4 + r % 4 inside the group.
template <class ST, class OT>
__global__ __launch_bounds__(256) void k_v_pack(const VRepack* __restrict__ vr, const void* const* __restrict__ stages,
                                                OT* __restrict__ out, float* __restrict__ out_hi, int dither) {
  const VRepack d = vr[blockIdx.x];
  const ST* src = (const ST*)stages[d.stage] + d.src;
  const int64_t tot = (int64_t)d.n * d.k;
  for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
    const int r = (int)(e % d.n), l = (int)(e / d.n);
    const int pc = d.lc0 + l;
    const int g = pc / P1_GW, lp = pc % P1_GW;
    const int gw = min(P1_GW, d.ktau - g * P1_GW);
    const int gs = gw + (gw & 1);  // stored columns (an odd panel carries a zero column)
    const int64_t o = d.tau_base + (int64_t)g * P1_GW * d.np + ((int64_t)(r >> 2) * gs + lp) * 4 + (r & 3);
    const double x = (double)src[e];
    out[o] = round_factor<OT>(x, dither != 0, 2u, (uint32_t)(d.cb + r), (uint32_t)d.rb, (uint32_t)l);
    if (out_hi) out_hi[o] = (float)x;
  }
}

// Row scaling of the phase-2 panels (closed cavity, eqs. (32)-(34)): every
// element of row row0 + r of a tile's items is multiplied by scale[row0 + r].
template <class DT, class LT>
__global__ __launch_bounds__(256) void k_panel_rowscale(const P2Tile* __restrict__ tiles, const P2Item* __restrict__ items,
                                                        const double* __restrict__ scale, DT* __restrict__ dense,
                                                        LT* __restrict__ U, float* __restrict__ Uhi) {
  const P2Tile tl = tiles[blockIdx.x];
  for (int k = 0; k < tl.nit; ++k) {
    const P2Item it = items[tl.it0 + k];
    const int64_t tot = (int64_t)tl.m * it.w;
    for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
      const int r = (int)((e >> 2) % tl.m);
      const double f = scale[tl.row0 + r];
      const int64_t o = it.base + e;
      if (it.kind == 0) {
        dense[o] = Cvt<DT>::from_f64(Cvt<DT>::to_f64(dense[o]) * f);
      } else if (Uhi) {
        const double x = (double)Uhi[o] * f;
        Uhi[o] = (float)x;
        U[o] = Cvt<LT>::from_f64(x);
      } else {
        U[o] = Cvt<LT>::from_f64(Cvt<LT>::to_f64(U[o]) * f);
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

void closed_row_scale(hm_matrix& M, hipStream_t s);

namespace {

// One cavity of an assembly call.
struct AsmJob {
  const hm_tree* t = nullptr;
  hm_assembly_params p{};
  std::unique_ptr<hm_matrix> M;
  int64_t goff = 0;  // first facet of the cavity in the shared geometry arrays
  Geo g{};           // the cavity's geometry (pointers into the shared arrays)
  std::vector<LrInfo> lr;
  std::vector<BlockRef> dn;
  size_t lr_done = 0;  // admissible blocks of the cavity whose ACA has finished
};

// Near-field packing, panel packing of the compacted factors, statistics and
// the product plan of a cavity whose ACA blocks are all done.
void finish_job(AsmJob& J, const std::vector<DevBuf>& stages, hipStream_t s) {
  hm_matrix* M = J.M.get();
  const hm_assembly_params& p = J.p;
  auto& dn = J.dn;
  auto& lr = J.lr;
  // blocks whose recompressed factors are all zero hold nothing
  lr.erase(std::remove_if(lr.begin(), lr.end(), [](const LrInfo& l) { return l.k == 0; }), lr.end());
  std::sort(dn.begin(), dn.end(), [](const BlockRef& x, const BlockRef& y) {
    return x.rb != y.rb ? x.rb < y.rb : x.cb < y.cb;
  });
  for (const auto& d : dn) M->dense_entries += (int64_t)(d.re - d.rb) * (d.ce - d.cb);
  M->n_dense_blocks = (int64_t)dn.size();
  M->n_lr_blocks = (int64_t)lr.size();
  for (const auto& l : lr) {
    M->rank_sum += l.k;
    M->u_entries += (int64_t)l.k * (l.b.re - l.b.rb);
    M->v_entries += (int64_t)l.k * (l.b.ce - l.b.cb);
    M->max_rank = std::max(M->max_rank, l.k);
  }
  M->lr_entries = M->u_entries + M->v_entries;

  // ---- plan, panel arenas, packing
  PackLists pk;
  build_plan(*M, lr, dn, *J.t, pk, s);
  const Plan& P = M->plan;
  const size_t ds = dtype_size(p.dense_dtype), ls = dtype_size(p.lowrank_dtype);
  M->dense.alloc(std::max<int64_t>(1, P.dense_elems) * ds);
  M->U.alloc(std::max<int64_t>(1, P.u_elems) * ls);
  M->V.alloc(std::max<int64_t>(1, P.v_elems) * ls);
  HM_HIP(hipMemsetAsync(M->dense.get(), 0, M->dense.bytes(), s));
  if (p.dense_dtype == HM_BF16) {
    M->dense_hi.alloc(std::max<int64_t>(1, P.dense_elems) * 4);
    HM_HIP(hipMemsetAsync(M->dense_hi.get(), 0, M->dense_hi.bytes(), s));
  }
  HM_HIP(hipMemsetAsync(M->U.get(), 0, M->U.bytes(), s));
  HM_HIP(hipMemsetAsync(M->V.get(), 0, M->V.bytes(), s));
  if (M->has_hi) {
    M->U_hi.alloc(std::max<int64_t>(1, P.u_elems) * 4);
    M->V_hi.alloc(std::max<int64_t>(1, P.v_elems) * 4);
    HM_HIP(hipMemsetAsync(M->U_hi.get(), 0, M->U_hi.bytes(), s));
    HM_HIP(hipMemsetAsync(M->V_hi.get(), 0, M->V_hi.bytes(), s));
  }
  if (!pk.nf.empty()) {
    DevBuf d_nf;
    upload(d_nf, pk.nf, s);
    if (p.dense_dtype == HM_F64)
      hipLaunchKernelGGL(k_nf_pack<double>, dim3((unsigned)pk.nf.size()), dim3(256), 0, s, d_nf.get<NfDev>(), J.g,
                         M->dense.get<double>());
    else if (p.dense_dtype == HM_F32)
      hipLaunchKernelGGL(k_nf_pack<float>, dim3((unsigned)pk.nf.size()), dim3(256), 0, s, d_nf.get<NfDev>(), J.g,
                         M->dense.get<float>());
    else {
      // FP32 copy first (also the padding zeros), then its BF16 rounding
      const int64_t ne = std::max<int64_t>(1, P.dense_elems);
      hipLaunchKernelGGL(k_nf_pack<float>, dim3((unsigned)pk.nf.size()), dim3(256), 0, s, d_nf.get<NfDev>(), J.g,
                         M->dense_hi.get<float>());
      hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, M->dense_hi.get<float>(),
                         M->dense.get<bf16_t>(), ne);
    }
    HM_HIP(hipGetLastError());
    HM_HIP(hipStreamSynchronize(s));
  }
  if (!lr.empty()) {
    std::vector<const void*> sp(stages.size());
    for (size_t q = 0; q < stages.size(); ++q) sp[q] = stages[q].get();
    DevBuf d_sp, d_ur, d_vr;
    upload(d_sp, sp, s);
    upload(d_ur, pk.ur, s);
    upload(d_vr, pk.vr, s);
    float* uh = M->has_hi ? M->U_hi.get<float>() : nullptr;
    float* vh = M->has_hi ? M->V_hi.get<float>() : nullptr;
    auto go = [&](auto* stag, auto* otag) {
      using ST = std::remove_pointer_t<decltype(stag)>;
      using OT = std::remove_pointer_t<decltype(otag)>;
      if (!pk.ur.empty())
        hipLaunchKernelGGL((k_u_pack<ST, OT>), dim3((unsigned)pk.ur.size()), dim3(256), 0, s, d_ur.get<URepack>(),
                           d_sp.get<const void*>(), M->U.get<OT>(), uh, (int)p.lowrank_rounding);
      if (!pk.vr.empty())
        hipLaunchKernelGGL((k_v_pack<ST, OT>), dim3((unsigned)pk.vr.size()), dim3(256), 0, s, d_vr.get<VRepack>(),
                           d_sp.get<const void*>(), M->V.get<OT>(), vh, (int)p.lowrank_rounding);
    };
    if (p.lowrank_dtype == HM_F64) go((double*)0, (double*)0);
    else if (p.lowrank_dtype == HM_F32) go((float*)0, (float*)0);
    else go((float*)0, (bf16_t*)0);
    HM_HIP(hipGetLastError());
    HM_HIP(hipStreamSynchronize(s));
  }
  if (p.closed_row_scale) closed_row_scale(*M, s);
}

}  // namespace

// Assembles every cavity of `trees` (Sec. 4.3): the admissible blocks of all
// of them go through shared ACA launches (largest blocks first, one wave per
// small block), then each cavity is packed as soon as its blocks are done.
// Each block's ACA depends only on the block, so a matrix is the same whether
// its cavity is assembled alone or with others.  With tune_jointly, the
// matrices whose autotune flag is set get one phase-1 split, timed on their
// batched product; otherwise each such matrix is tuned alone.
// A second stream (default priority) and the events that fork it from and
// join it to the caller's stream, for the launch of the largest ACA blocks,
// which then runs beside the launch of the others.
struct SideStream {
  hipStream_t st = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  SideStream() {
    HM_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    HM_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    HM_HIP(hipEventCreateWithFlags(&join, hipEventDisableTiming));
  }
  ~SideStream() {
    if (st) (void)hipStreamSynchronize(st);
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (st) (void)hipStreamDestroy(st);
  }
  SideStream(const SideStream&) = delete;
  SideStream& operator=(const SideStream&) = delete;
};

std::vector<hm_matrix*> assemble_batch(hm_ctx& ctx, const std::vector<const hm_tree*>& trees,
                                       const std::vector<hm_assembly_params>& ps, bool tune_jointly) {
  hipStream_t s = ctx.stream;
  std::unique_ptr<SideStream> side;  // created with the first launch of the largest blocks
  const size_t nj = trees.size();
  std::vector<AsmJob> jobs(nj);
  int64_t ntot = 0;
  for (size_t j = 0; j < nj; ++j) {
    AsmJob& J = jobs[j];
    J.t = trees[j];
    J.p = ps[j];
    J.goff = ntot;
    ntot += J.t->n;
    HM_REQUIRE(ntot < ((int64_t)1 << 31), "assemble: more than 2^31 facets in one call");
    J.M = std::make_unique<hm_matrix>();
    hm_matrix* M = J.M.get();
    M->device = ctx.device;
    M->n = J.t->n;
    M->dense_dtype = J.p.dense_dtype;
    M->lr_dtype = J.p.lowrank_dtype;
    M->has_hi = J.p.lowrank_dtype == HM_BF16 && J.p.keep_f32_copy;
    M->perm = J.t->perm;
    upload(M->d_perm, M->perm, s);
    J.dn.assign(J.t->dense.begin(), J.t->dense.end());
  }

  // permuted geometry of all cavities, SoA FP64, one array per quantity
  std::vector<double> geo(7 * std::max<int64_t>(1, ntot));
  for (const AsmJob& J : jobs) {
    const hm_tree& t = *J.t;
    for (int64_t k = 0; k < t.n; ++k) {
      const int64_t o = t.perm[k], d = J.goff + k;
      for (int a = 0; a < 3; ++a) {
        geo[a * ntot + d] = t.c[3 * o + a];
        geo[(3 + a) * ntot + d] = t.nrm[3 * o + a];
      }
      geo[6 * ntot + d] = t.area[o];
    }
  }
  DevBuf d_geo;
  upload(d_geo, geo, s);
  const double* gp = d_geo.get<double>();
  const Geo g{gp, gp + ntot, gp + 2 * ntot, gp + 3 * ntot, gp + 4 * ntot, gp + 5 * ntot, gp + 6 * ntot};
  for (AsmJob& J : jobs) {
    const int64_t o = J.goff;
    J.g = Geo{g.cx + o, g.cy + o, g.cz + o, g.nx + o, g.ny + o, g.nz + o, g.ar + o};
  }

  // ---- ACA on the admissible blocks of all cavities, in batches bounded by
  // a scratch budget; block indices address the shared geometry
  size_t free_b = 0, total_b = 0;
  HM_HIP(hipMemGetInfo(&free_b, &total_b));
  const int64_t budget = std::max<int64_t>(256ll << 20, std::min<int64_t>(8ll << 30, (int64_t)free_b / 4));
  std::vector<DevBuf> stages;
  std::vector<size_t> stage_last;  // last job with factors in each stage buffer
  DevBuf scratch, flags, d_blk, d_blk_small, d_blk_huge, d_blk_full, d_blk_full_big, d_rank, d_status, d_cd;
  DevBuf d_full_slices, d_full_first, d_full_state, d_full_part, d_full_pam;  // sliced full pivoting
  size_t jpos = 0, bpos = 0, next_finish = 0;
  auto finish_ready = [&]() {
    while (next_finish < nj && jobs[next_finish].lr_done == jobs[next_finish].t->lowrank.size()) {
      finish_job(jobs[next_finish], stages, s);
      // stage buffers no later cavity reads
      for (size_t q = 0; q < stages.size(); ++q)
        if (stage_last[q] <= next_finish) stages[q].release();
      ++next_finish;
    }
  };
  finish_ready();
  while (next_finish < nj) {
    std::vector<AcaDev> batch;
    std::vector<int32_t> bjob;  // job of each batch entry
    std::vector<uint8_t> bfull;  // 1: fully pivoted ACA
    int64_t sd = 0, sf = 0;
    while (jpos < nj) {
      const AsmJob& J = jobs[jpos];
      if (bpos == J.t->lowrank.size()) {
        ++jpos;
        bpos = 0;
        continue;
      }
      const BlockRef& b = J.t->lowrank[bpos];
      const int m = b.re - b.rb, nn = b.ce - b.cb;
      const int64_t kc = rank_cap(m, nn, std::min<int>(J.p.k_max, ACA_KMAX));
      const bool full = J.p.aca_pivot == 1;
      const int64_t rsz = full ? (int64_t)m * nn : 0;  // residual of full pivoting
      HM_REQUIRE(rsz < ((int64_t)1 << 31), "assemble: full pivoting needs admissible blocks of fewer than 2^31 entries");
      const int64_t need = (kc * (m + nn) + rsz) * 8 + m * 4;
      if (!batch.empty() && (sd * 8 + sf * 4 + need) > budget) break;
      const int32_t o = (int32_t)J.goff;
      batch.push_back(AcaDev{b.rb + o, b.re + o, b.cb + o, b.ce + o, (int32_t)kc, 0, sd, sd + kc * m, sf,
                             sd + kc * (m + nn), J.p.aca_tol});
      bjob.push_back((int32_t)jpos);
      bfull.push_back(full ? 1 : 0);
      sd += kc * (m + nn) + rsz;
      sf += m;
      ++bpos;
    }
    HM_REQUIRE(!batch.empty(), "assemble: empty ACA batch");
    // blocks of at most 64 x 64 (rank cap <= 32): one wave each; larger ones:
    // one workgroup each (512 threads from m + n >= ACA_HUGE), largest
    // first for the hardware dispatcher
    std::vector<AcaDev> small, large, huge, full, full_big;
    for (size_t q = 0; q < batch.size(); ++q) {
      batch[q].out = (int32_t)q;
      const AcaDev& a = batch[q];
      if (bfull[q] && (int64_t)(a.re - a.rb) * (a.ce - a.cb) >= ACA_FULL_BIG) full_big.push_back(a);
      else if (bfull[q]) full.push_back(a);
      else if (a.re - a.rb <= 64 && a.ce - a.cb <= 64 && a.kcap <= ACAW_K) small.push_back(a);
      else if ((a.re - a.rb) + (a.ce - a.cb) >= ACA_HUGE) huge.push_back(a);
      else large.push_back(a);
    }
    auto by_size = [](const AcaDev& x, const AcaDev& y) {
      return (int64_t)(x.re - x.rb) * (x.ce - x.cb) > (int64_t)(y.re - y.rb) * (y.ce - y.cb);
    };
    std::stable_sort(large.begin(), large.end(), by_size);
    std::stable_sort(huge.begin(), huge.end(), by_size);
    std::stable_sort(full.begin(), full.end(), by_size);
    std::stable_sort(full_big.begin(), full_big.end(), by_size);
    if ((size_t)sd * 8 > scratch.bytes()) scratch.alloc((size_t)sd * 8);
    if ((size_t)sf * 4 > flags.bytes()) flags.alloc((size_t)sf * 4);
    d_rank.alloc(batch.size() * 4);
    d_status.alloc(batch.size() * 4);
    if (!huge.empty() || !full_big.empty()) {
      // on the side stream, after everything queued so far on s (uploads,
      // scratch), joined back into s before the ranks are read
      if (!huge.empty()) upload(d_blk_huge, huge, s);
      // the largest fully pivoted blocks: slices of FULL_SLICE entries,
      // contiguous per block; as many crosses as the widest rank cap
      std::vector<int> ffirst(full_big.size() + 1, 0);
      int fkmax = 0;
      if (!full_big.empty()) {
        upload(d_blk_full_big, full_big, s);
        std::vector<FullSlice> fsl;
        for (size_t q = 0; q < full_big.size(); ++q) {
          const AcaDev& a = full_big[q];
          const int64_t mn = (int64_t)(a.re - a.rb) * (a.ce - a.cb);
          ffirst[q] = (int)fsl.size();
          for (int64_t e = 0, sq = 0; e < mn; e += FULL_SLICE, ++sq) fsl.push_back(FullSlice{(int32_t)q, (int32_t)sq});
          fkmax = std::max(fkmax, (int)a.kcap);
        }
        ffirst[full_big.size()] = (int)fsl.size();
        upload(d_full_slices, fsl, s);
        upload(d_full_first, ffirst, s);
        d_full_state.alloc(full_big.size() * sizeof(FullState));
        d_full_part.alloc(fsl.size() * sizeof(double));
        d_full_pam.alloc(fsl.size() * sizeof(ArgMax));
      }
      if (!side) side = std::make_unique<SideStream>();
      HM_HIP(hipEventRecord(side->fork, s));
      HM_HIP(hipStreamWaitEvent(side->st, side->fork, 0));
      if (!huge.empty())
        hipLaunchKernelGGL(k_aca<ACA_T_HUGE>, dim3((unsigned)huge.size()), dim3(ACA_T_HUGE), 0, side->st,
                           d_blk_huge.get<AcaDev>(), g, scratch.get<double>(), flags.get<int>(),
                           d_rank.get<int>(), d_status.get<int>());
      // fully pivoted blocks of ACA_FULL_BIG entries and more: each cross
      // streams the whole residual, so every pass over it is spread over
      // many workgroups, with a finishing step per block between passes
      if (!full_big.empty()) {
        const unsigned nsl = (unsigned)ffirst[full_big.size()], nbl = (unsigned)full_big.size();
        const AcaDev* fb = d_blk_full_big.get<AcaDev>();
        const FullSlice* fs = d_full_slices.get<FullSlice>();
        FullState* fst = d_full_state.get<FullState>();
        hipLaunchKernelGGL(k_full_pass<true>, dim3(nsl), dim3(FULL_T), 0, side->st, fb, fs, (const FullState*)fst, g,
                           scratch.get<double>(), d_full_part.get<double>(), d_full_pam.get<ArgMax>());
        hipLaunchKernelGGL(k_full_fin<true>, dim3(nbl), dim3(FULL_T), 0, side->st, fb, d_full_first.get<int>(), fst,
                           scratch.get<double>(), (const double*)d_full_part.get<double>(),
                           (const ArgMax*)d_full_pam.get<ArgMax>(), d_rank.get<int>(), d_status.get<int>());
        for (int c = 0; c < fkmax; ++c) {
          hipLaunchKernelGGL(k_full_pass<false>, dim3(nsl), dim3(FULL_T), 0, side->st, fb, fs, (const FullState*)fst,
                             g, scratch.get<double>(), d_full_part.get<double>(), d_full_pam.get<ArgMax>());
          hipLaunchKernelGGL(k_full_fin<false>, dim3(nbl), dim3(FULL_T), 0, side->st, fb, d_full_first.get<int>(),
                             fst, scratch.get<double>(), (const double*)d_full_part.get<double>(),
                             (const ArgMax*)d_full_pam.get<ArgMax>(), d_rank.get<int>(), d_status.get<int>());
        }
      }
      HM_HIP(hipGetLastError());
      HM_HIP(hipEventRecord(side->join, side->st));
    }
    if (!large.empty()) {
      upload(d_blk, large, s);
      hipLaunchKernelGGL(k_aca<ACA_T>, dim3((unsigned)large.size()), dim3(ACA_T), 0, s, d_blk.get<AcaDev>(), g,
                         scratch.get<double>(), flags.get<int>(), d_rank.get<int>(), d_status.get<int>());
      HM_HIP(hipGetLastError());
    }
    if (!full.empty()) {
      upload(d_blk_full, full, s);
      hipLaunchKernelGGL(k_aca_full<ACA_T>, dim3((unsigned)full.size()), dim3(ACA_T), 0, s, d_blk_full.get<AcaDev>(),
                         g, scratch.get<double>(), d_rank.get<int>(), d_status.get<int>());
      HM_HIP(hipGetLastError());
    }
    if (!small.empty()) {
      upload(d_blk_small, small, s);
      hipLaunchKernelGGL(k_aca_wave, dim3((unsigned)((small.size() + 3) / 4)), dim3(256), 0, s,
                         d_blk_small.get<AcaDev>(), (int)small.size(), g, scratch.get<double>(),
                         d_rank.get<int>(), d_status.get<int>());
      HM_HIP(hipGetLastError());
    }
    if (!huge.empty() || !full_big.empty()) HM_HIP(hipStreamWaitEvent(s, side->join, 0));
    std::vector<int> rk(batch.size()), st(batch.size());
    HM_HIP(hipMemcpyAsync(rk.data(), d_rank.get(), rk.size() * 4, hipMemcpyDeviceToHost, s));
    HM_HIP(hipMemcpyAsync(st.data(), d_status.get(), st.size() * 4, hipMemcpyDeviceToHost, s));
    HM_HIP(hipStreamSynchronize(s));
    // classify: low rank (converged and k(m+n) < mn), rank zero (dropped),
    // dense fallback; factors compacted per stored precision (FP64 stage for
    // FP64 factors, FP32 otherwise)
    std::vector<CompactDev> cd[2];
    // blocks truncated by recompression instead of compacted as they are,
    // with the job and the position in its low-rank list of each
    std::vector<RcDev> rc[2];
    std::vector<std::pair<AsmJob*, size_t>> rc_lr[2];
    int64_t off[2] = {0, 0};
    int32_t sidx[2] = {-1, -1};
    for (int w = 0; w < 2; ++w) {
      sidx[w] = (int32_t)stages.size();
      stages.emplace_back();
      stage_last.push_back(0);
    }
    for (size_t q = 0; q < batch.size(); ++q) {
      const AcaDev& a = batch[q];
      AsmJob& J = jobs[bjob[q]];
      const int32_t o = (int32_t)J.goff;
      const int m = a.re - a.rb, nn = a.ce - a.cb;
      const int k = rk[q];
      BlockRef br{a.rb - o, a.re - o, a.cb - o, a.ce - o};
      J.lr_done++;
      if (!st[q] || (int64_t)k * (m + nn) >= (int64_t)m * nn) {
        J.dn.push_back(br);
        J.M->n_fallback++;
        continue;
      }
      if (k == 0) continue;  // exactly zero block
      const int w = J.p.lowrank_dtype == HM_F64 ? 1 : 0;
      if (J.p.recompress && k >= 2 && k <= RC_KMAX) {
        // the stage keeps room for the ACA rank; the truncated factors
        // (rank r <= k) are written at the same offsets
        rc[w].push_back(RcDev{a.u_off, a.v_off, 0, off[w], off[w] + (int64_t)m * k, m, nn, k,
                              (int32_t)rc[w].size(), a.tol});
        rc_lr[w].emplace_back(&J, J.lr.size());
      } else {
        cd[w].push_back(CompactDev{a.u_off, a.v_off, off[w], off[w] + (int64_t)m * k, m, nn, k, 0});
      }
      J.lr.push_back(LrInfo{br, k, sidx[w], off[w], off[w] + (int64_t)m * k});
      off[w] += (int64_t)k * (m + nn);
      stage_last[sidx[w]] = std::max<size_t>(stage_last[sidx[w]], (size_t)bjob[q]);
    }
    for (int w = 0; w < 2; ++w) {
      if (cd[w].empty() && rc[w].empty()) continue;
      DevBuf& stg = stages[sidx[w]];
      stg.alloc(off[w] * (w ? 8 : 4));
      if (!cd[w].empty()) {
        upload(d_cd, cd[w], s);
        if (w)
          hipLaunchKernelGGL(k_compact<double>, dim3((unsigned)cd[w].size()), dim3(256), 0, s,
                             d_cd.get<CompactDev>(), scratch.get<double>(), stg.get<double>());
        else
          hipLaunchKernelGGL(k_compact<float>, dim3((unsigned)cd[w].size()), dim3(256), 0, s,
                             d_cd.get<CompactDev>(), scratch.get<double>(), stg.get<float>());
        HM_HIP(hipGetLastError());
      }
      if (!rc[w].empty()) {
        DevBuf d_nr(rc[w].size() * 4);
        recompress_blocks(rc[w], scratch.get<double>(), stg.get(), w == 1, d_nr.get<int>(), s);
        std::vector<int> nr(rc[w].size());
        HM_HIP(hipMemcpyAsync(nr.data(), d_nr.get(), nr.size() * 4, hipMemcpyDeviceToHost, s));
        HM_HIP(hipStreamSynchronize(s));
        for (size_t q = 0; q < nr.size(); ++q) {
          LrInfo& l = rc_lr[w][q].first->lr[rc_lr[w][q].second];
          HM_REQUIRE(nr[q] >= 0 && nr[q] <= l.k, "assemble: recompression raised a rank");
          l.k = nr[q];
        }
      }
      HM_HIP(hipStreamSynchronize(s));  // scratch is reused by the next batch
    }
    finish_ready();
  }
  scratch.release();
  flags.release();
  stages.clear();

  // ---- phase-1 split
  std::vector<hm_matrix*> tuned;
  int width = 1;  // the widest product the tuned matrices ask for
  for (AsmJob& J : jobs)
    if (J.p.autotune) {
      tuned.push_back(J.M.get());
      width = std::max(width, (int)J.p.autotune);
    }
  if (tune_jointly && tuned.size() > 1) autotune_phase1_joint(tuned, s, width);
  else
    for (size_t j = 0, t = 0; j < jobs.size(); ++j)
      if (jobs[j].p.autotune) autotune_phase1(*tuned[t++], s, (int)jobs[j].p.autotune);
  HM_HIP(hipStreamSynchronize(s));
  std::vector<hm_matrix*> out(nj);
  for (size_t j = 0; j < nj; ++j) out[j] = jobs[j].M.release();
  return out;
}

hm_matrix* assemble(hm_ctx& ctx, const hm_tree& t, const hm_assembly_params& p) {
  return assemble_batch(ctx, {&t}, {p}, false)[0];
}

// Closed-cavity treatment (eqs. (32)-(34)): s = F_H 1 (the per-area row sum),
// c = clamp(s, 0, 1), rows with c != 0 divided by c.
void closed_row_scale(hm_matrix& M, hipStream_t s) {
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
  const unsigned ni = (unsigned)M.plan.p2t.size();
  if (ni) {
    const P2Tile* tl = M.plan.d_p2t.get<P2Tile>();
    const P2Item* it = M.plan.d_p2.get<P2Item>();
    float* uh = M.has_hi ? M.U_hi.get<float>() : nullptr;
    auto go = [&](auto* dt, auto* lt) {
      using DT = std::remove_pointer_t<decltype(dt)>;
      using LT = std::remove_pointer_t<decltype(lt)>;
      hipLaunchKernelGGL((k_panel_rowscale<DT, LT>), dim3(ni), dim3(256), 0, s, tl, it, scale.get<double>(),
                         M.dense.get<DT>(), M.U.get<LT>(), uh);
    };
    if (M.dense_dtype == HM_F64) {
      if (M.lr_dtype == HM_F64) go((double*)0, (double*)0);
      else go((double*)0, (float*)0);
    } else {
      if (M.lr_dtype == HM_F32) go((float*)0, (float*)0);
      else if (M.lr_dtype == HM_BF16) go((float*)0, (bf16_t*)0);
      else go((float*)0, (double*)0);
    }
    HM_HIP(hipGetLastError());
  }
  HM_HIP(hipStreamSynchronize(s));
}


// ------------------------------------------------------------------ per-block factors for the block LU
namespace {
// Dense block of the reflection matrix C = I - diag(1 - eps) F (eq. (11)):
// D(i, j) = -om_i F(r0 + i, c0 + j), plus 1 on the diagonal of a diagonal
// block (F_ii = 0); column-major m x n.
__global__ void k_reflect_dense(Geo g, int32_t r0, int32_t c0, int32_t m, int32_t n, const double* __restrict__ om,
                                int diag, double* __restrict__ D) {
  const int64_t mn = (int64_t)m * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < mn; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % m), j = (int)(e / m);
    double v = -om[r0 + i] * view_factor(g, r0 + i, c0 + j);
    if (diag && i == j) v += 1.0;
    D[e] = v;
  }
}

// U(i, l) <- -om[r0 + i] U(i, l): the row scaling of C applied to a low-rank factor
__global__ void k_reflect_rows(double* __restrict__ U, int32_t m, int32_t k, const double* __restrict__ om,
                               int32_t r0) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (int64_t)m * k) U[e] = -om[r0 + (int)(e % m)] * U[e];
}
}  // namespace

// Blocks of the reflection matrix for the block LU (Sec. 5.1): every listed
// block (permuted positions) is either a dense block of C (dense[i] = 1 on
// input: evaluated in full) or an admissible block compressed by ACA with
// the parameters' pivoting and recompressed at aca_tol, its U rows scaled by
// -(1 - eps); an admissible block that ACA stores dense (cap reached, or
// k (m + n) >= m n) comes back dense.  om = 1 - eps in the permuted order
// (DEVICE).  FP64 throughout.
void reflection_blocks(hm_ctx& ctx, const hm_tree& t, const double* om, const std::vector<BlockRef>& blocks,
                       std::vector<uint8_t>& dense, const hm_assembly_params& p, std::vector<BlockFactor>& out) {
  hipStream_t s = ctx.stream;
  const int64_t n = t.n;
  std::vector<double> geo(7 * std::max<int64_t>(1, n));
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
  const Geo g{gp, gp + n, gp + 2 * n, gp + 3 * n, gp + 4 * n, gp + 5 * n, gp + 6 * n};
  out.clear();
  out.resize(blocks.size());
  // ACA of the admissible blocks, in batches bounded by a scratch budget
  std::vector<size_t> adm;
  for (size_t q = 0; q < blocks.size(); ++q)
    if (!dense[q]) adm.push_back(q);
  const int64_t budget = (int64_t)1 << 30;
  size_t pos = 0;
  DevBuf scratch, flags, d_blk, d_rank, d_status, d_nr, d_cd;
  while (pos < adm.size()) {
    std::vector<AcaDev> batch;
    std::vector<size_t> who;
    int64_t sd = 0, sf = 0;
    while (pos < adm.size()) {
      const BlockRef& b = blocks[adm[pos]];
      const int m = b.re - b.rb, nn = b.ce - b.cb;
      const int64_t kc = rank_cap(m, nn, std::min<int>(p.k_max, ACA_KMAX));
      const int64_t rsz = p.aca_pivot == 1 ? (int64_t)m * nn : 0;
      HM_REQUIRE(rsz < ((int64_t)1 << 31), "block LU: full pivoting needs blocks of fewer than 2^31 entries");
      const int64_t need = (kc * (m + nn) + rsz) * 8 + m * 4;
      if (!batch.empty() && sd * 8 + sf * 4 + need > budget) break;
      batch.push_back(AcaDev{b.rb, b.re, b.cb, b.ce, (int32_t)kc, (int32_t)batch.size(), sd, sd + kc * m, sf,
                             sd + kc * (m + nn), p.aca_tol});
      who.push_back(adm[pos]);
      sd += kc * (m + nn) + rsz;
      sf += m;
      ++pos;
    }
    if ((size_t)sd * 8 > scratch.bytes()) scratch.alloc((size_t)sd * 8);
    if ((size_t)sf * 4 > flags.bytes()) flags.alloc((size_t)sf * 4);
    d_rank.alloc(batch.size() * 4);
    d_status.alloc(batch.size() * 4);
    std::vector<AcaDev> small, large;
    for (const AcaDev& a : batch) {
      if (p.aca_pivot != 1 && a.re - a.rb <= 64 && a.ce - a.cb <= 64 && a.kcap <= ACAW_K) small.push_back(a);
      else large.push_back(a);
    }
    DevBuf d_small;
    if (!large.empty()) {
      upload(d_blk, large, s);
      if (p.aca_pivot == 1)
        hipLaunchKernelGGL(k_aca_full<ACA_T>, dim3((unsigned)large.size()), dim3(ACA_T), 0, s, d_blk.get<AcaDev>(),
                           g, scratch.get<double>(), d_rank.get<int>(), d_status.get<int>());
      else
        hipLaunchKernelGGL(k_aca<ACA_T>, dim3((unsigned)large.size()), dim3(ACA_T), 0, s, d_blk.get<AcaDev>(), g,
                           scratch.get<double>(), flags.get<int>(), d_rank.get<int>(), d_status.get<int>());
      HM_HIP(hipGetLastError());
    }
    if (!small.empty()) {
      upload(d_small, small, s);
      hipLaunchKernelGGL(k_aca_wave, dim3((unsigned)((small.size() + 3) / 4)), dim3(256), 0, s,
                         d_small.get<AcaDev>(), (int)small.size(), g, scratch.get<double>(), d_rank.get<int>(),
                         d_status.get<int>());
      HM_HIP(hipGetLastError());
    }
    std::vector<int> rk(batch.size()), st(batch.size());
    HM_HIP(hipMemcpyAsync(rk.data(), d_rank.get(), rk.size() * 4, hipMemcpyDeviceToHost, s));
    HM_HIP(hipMemcpyAsync(st.data(), d_status.get(), st.size() * 4, hipMemcpyDeviceToHost, s));
    HM_HIP(hipStreamSynchronize(s));
    // low-rank blocks: recompressed (rank >= 2) or copied (rank 1) into an FP64 stage
    std::vector<RcDev> rc;
    std::vector<CompactDev> cd;
    std::vector<size_t> rc_q, cd_q;
    int64_t off = 0;
    for (size_t q = 0; q < batch.size(); ++q) {
      const AcaDev& a = batch[q];
      const int m = a.re - a.rb, nn = a.ce - a.cb, k = rk[q];
      if (!st[q] || (int64_t)k * (m + nn) >= (int64_t)m * nn) {
        dense[who[q]] = 1;
        continue;
      }
      out[who[q]].lowrank = true;
      out[who[q]].k = k;
      if (k >= 2 && k <= RC_KMAX) {
        rc.push_back(RcDev{a.u_off, a.v_off, 0, off, off + (int64_t)m * k, m, nn, k, (int32_t)rc.size(), a.tol});
        rc_q.push_back(q);
      } else if (k >= 1) {
        cd.push_back(CompactDev{a.u_off, a.v_off, off, off + (int64_t)m * k, m, nn, k, 0});
        cd_q.push_back(q);
      }
      out[who[q]].su = off;
      out[who[q]].sv = off + (int64_t)m * k;
      off += (int64_t)k * (m + nn);
    }
    DevBuf stage(std::max<int64_t>(1, off) * 8);
    if (!cd.empty()) {
      upload(d_cd, cd, s);
      hipLaunchKernelGGL(k_compact<double>, dim3((unsigned)cd.size()), dim3(256), 0, s, d_cd.get<CompactDev>(),
                         scratch.get<double>(), stage.get<double>());
      HM_HIP(hipGetLastError());
    }
    if (!rc.empty()) {
      d_nr.alloc(rc.size() * 4);
      recompress_blocks(rc, scratch.get<double>(), stage.get(), true, d_nr.get<int>(), s);
      std::vector<int> nr(rc.size());
      HM_HIP(hipMemcpyAsync(nr.data(), d_nr.get(), nr.size() * 4, hipMemcpyDeviceToHost, s));
      HM_HIP(hipStreamSynchronize(s));
      for (size_t q = 0; q < rc.size(); ++q) out[who[rc_q[q]]].k = nr[q];
    }
    // each block's factors into buffers of its own (U m x k, V n x k, the
    // row scaling of C on U)
    for (size_t q = 0; q < batch.size(); ++q) {
      BlockFactor& f = out[who[q]];
      if (!f.lowrank || dense[who[q]]) continue;
      const AcaDev& a = batch[q];
      const int m = a.re - a.rb, nn = a.ce - a.cb;
      f.U.alloc(std::max<int64_t>(1, (int64_t)m * f.k) * 8);
      f.V.alloc(std::max<int64_t>(1, (int64_t)nn * f.k) * 8);
      if (f.k > 0) {
        HM_HIP(hipMemcpyAsync(f.U.get(), stage.get<double>() + f.su, (size_t)m * f.k * 8, hipMemcpyDeviceToDevice, s));
        HM_HIP(hipMemcpyAsync(f.V.get(), stage.get<double>() + f.sv, (size_t)nn * f.k * 8, hipMemcpyDeviceToDevice, s));
        const int64_t e = (int64_t)m * f.k;
        hipLaunchKernelGGL(k_reflect_rows, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, s, f.U.get<double>(), m,
                           f.k, om, a.rb);
        HM_HIP(hipGetLastError());
      }
    }
    HM_HIP(hipStreamSynchronize(s));
  }
  // dense blocks of C
  for (size_t q = 0; q < blocks.size(); ++q) {
    if (!dense[q]) continue;
    const BlockRef& b = blocks[q];
    const int m = b.re - b.rb, nn = b.ce - b.cb;
    BlockFactor& f = out[q];
    f.lowrank = false;
    f.D.alloc((size_t)m * nn * 8);
    const int64_t e = (int64_t)m * nn;
    const unsigned gr = (unsigned)std::min<int64_t>(4096, (e + 255) / 256);
    hipLaunchKernelGGL(k_reflect_dense, dim3(gr), dim3(256), 0, s, g, b.rb, b.cb, m, nn, om,
                       b.rb == b.cb && b.re == b.ce ? 1 : 0, f.D.get<double>());
    HM_HIP(hipGetLastError());
  }
  HM_HIP(hipStreamSynchronize(s));
}

}  // namespace hm
