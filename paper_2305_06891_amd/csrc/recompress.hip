// Recompression of ACA crosses into truncated-SVD form on gfx950 (Sec. 4.3:
// the cross approximation is post-processed into standard low-rank factors;
// Sec. 5.1: ranks follow the singular value decay at the relative accuracy
// eps_rel).  One workgroup per block, FP64 throughout:
//
//  1. column scaling: U = Uh diag(a), V = Vh diag(b) with unit columns
//     (a_l = |u_l|, b_l = |v_l|), so U V^T = Uh D Vh^T, D = diag(a b);
//  2. Gram matrices Gu = Uh^T Uh, Gv = Vh^T Vh (k x k);
//  3. pivoted Cholesky Gu ~ Ru^T Ru (largest remaining diagonal first,
//     stopped when it falls below RC_DROP: columns within 1e-8 of the span
//     of the selected ones add nothing), so Uh ~ Qu Ru with
//     Qu = Uh_sel Ru11^-1 orthonormal; the same for V;
//  4. core K = Ru D Rv^T (ru x rv);
//  5. its SVD: Householder QR with column pivoting K P = Q R, then
//     one-sided Jacobi on the columns of R^T (cyclic round-robin pairs):
//     R^T Z = W, whose column norms are the singular values s and whose
//     normalised columns, permuted back, the right singular vectors
//     x = P W S^-1 (Z and Q are never formed); the smallest rank r >= 1 with
//     sqrt(sum_{i>r} s_i^2) <= tol |s|_2 (Frobenius form of eq. (31));
//  6. the kept right vectors x_r and the left ones times s, K x_r;
//  7. U' = U Tu, V' = V Tv with Tu = diag(1/a) [Ru11^-1 K x_r] and
//     Tv = diag(1/b) [Rv11^-1 x_r] on the selected rows, so that
//     U' = (left vectors) S_r and V' has orthonormal columns; a second
//     kernel forms them straight into the staging buffer of the compacted
//     factors.
//
// Untruncated, the factors reproduce U V^T whatever the accuracy of the
// Cholesky factors (the same Ru, Rv are used on both sides), so rounding in
// the Gram matrices only perturbs the directions that are cut.
#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <cmath>
#include <climits>

#include "dev_common.hpp"
#include "hm_internal.hpp"
#include "recompress.hpp"

namespace hm {

namespace {

constexpr int RC_T = 256;                 // threads per workgroup
constexpr int RC_W = RC_T / 64;           // waves
constexpr int RC_LP = 16;                 // lanes per Jacobi pair
constexpr int RC_GROUPS = RC_T / RC_LP;   // Jacobi pairs in flight
constexpr int RC_PL = (RC_KMAX + RC_LP - 1) / RC_LP;  // column entries per lane
constexpr int RC_ROWS = 16;               // panel rows staged per Gram pass
constexpr int RC_SWEEPS = 40;             // Jacobi sweep limit
constexpr double RC_DROP = 1e-16;         // pivoted Cholesky stop (unit diagonal)
constexpr double RC_JTOL = 1e-13;         // Jacobi: |g| <= RC_JTOL sqrt(a b) counts as orthogonal
constexpr double RC_JFLOOR = 1e-30;       // ... and so does a pair of columns below RC_JFLOOR |K|_F^2

struct RcMax {
  double mag;
  int idx;
};

__device__ inline RcMax rc_better(RcMax a, RcMax b) {
  if (b.mag > a.mag || (b.mag == a.mag && b.idx < a.idx)) return b;
  return a;
}

__device__ RcMax rc_block_max(RcMax v, RcMax* sh) {
  for (int o = 32; o > 0; o >>= 1) {
    RcMax w;
    w.mag = __shfl_xor(v.mag, o, 64);
    w.idx = __shfl_xor(v.idx, o, 64);
    v = rc_better(v, w);
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  RcMax r = sh[0];
  for (int w = 1; w < RC_W; ++w) r = rc_better(r, sh[w]);
  return r;
}

__device__ double rc_block_sum(double v, double* sh) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = sh[0];
  for (int w = 1; w < RC_W; ++w) s += sh[w];
  return s;
}

__device__ inline double grp_sum(double v) {
#pragma unroll
  for (int o = RC_LP / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, RC_LP);
  return v;
}

// Column 2-norms of a len x k column-major panel (one wave per column).
__device__ void rc_colnorms(const double* __restrict__ P, int len, int k, double* __restrict__ nrm) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int l = wid; l < k; l += RC_W) {
    double s = 0.0;
    for (int i = lane; i < len; i += 64) {
      const double v = P[(int64_t)l * len + i];
      s += v * v;
    }
    s = wave_sum(s);
    if (lane == 0) nrm[l] = sqrt(s);
  }
}

// G = S^T S for S = P diag(inv) (len x k, column-major): 4 x 4 tiles of the
// upper triangle, one per thread per pass, over rows staged RC_ROWS at a
// time in LDS; both triangles of G (ld k) are written.
__device__ void rc_gram(const double* __restrict__ P, int len, int k, const double* __restrict__ inv,
                        double* __restrict__ G, double* __restrict__ stage, int sst) {
  const int nt = (k + 3) / 4, kc = 4 * nt;
  const int ntiles = nt * (nt + 1) / 2;
  for (int t0 = 0; t0 < ntiles; t0 += RC_T) {
    const int t = t0 + (int)threadIdx.x;
    const bool have = t < ntiles;
    int tp = 0, tq = 0;
    if (have) {
      int rem = t;
      while (rem >= nt - tp) {
        rem -= nt - tp;
        ++tp;
      }
      tq = tp + rem;
    }
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int i0 = 0; i0 < len; i0 += RC_ROWS) {
      const int rows = min(RC_ROWS, len - i0);
      __syncthreads();
      for (int e = threadIdx.x; e < RC_ROWS * kc; e += RC_T) {
        const int c = e / RC_ROWS, r = e % RC_ROWS;
        stage[r * sst + c] = (r < rows && c < k) ? P[(int64_t)c * len + i0 + r] * inv[c] : 0.0;
      }
      __syncthreads();
      if (have)
        for (int r = 0; r < rows; ++r) {
          const double* row = stage + r * sst;
          double x[4], y[4];
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            x[a] = row[4 * tp + a];
            y[a] = row[4 * tq + a];
          }
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] += x[a] * y[b];
        }
    }
    if (have)
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int p = 4 * tp + a, q = 4 * tq + b;
          if (p < k && q < k) {
            G[(int64_t)p * k + q] = acc[a][b];
            G[(int64_t)q * k + p] = acc[a][b];
          }
        }
  }
  __syncthreads();
}

// Pivoted Cholesky of the k x k Gram matrix G: rows s of R (ld k, all k
// columns; zero at the columns selected before step s), sel[s] = column of
// step s.  Returns the number of steps (the numerical rank).
// With weights w (the early mode), the step takes the column of largest
// w_j^2 d_j and the steps stop once sum_j w_j sqrt(d_j) over the columns not
// taken is at most lim.
__device__ int rc_pchol(const double* __restrict__ G, int k, double* __restrict__ R, int* __restrict__ sel,
                        double* __restrict__ d, int* __restrict__ taken, RcMax* sh, const double* __restrict__ w,
                        double lim, double* sh_sum) {
  for (int j = threadIdx.x; j < k; j += RC_T) {
    d[j] = G[(int64_t)j * k + j];
    taken[j] = 0;
  }
  __syncthreads();
  int rr = 0;
  for (int s = 0; s < k; ++s) {
    RcMax am{-1.0, INT_MAX};
    double rest = 0.0;
    for (int j = threadIdx.x; j < k; j += RC_T)
      if (!taken[j]) {
        am = rc_better(am, RcMax{w ? w[j] * w[j] * d[j] : d[j], j});
        if (w) rest += w[j] * sqrt(fmax(d[j], 0.0));
      }
    am = rc_block_max(am, sh);
    if (w && rc_block_sum(rest, sh_sum) <= lim) break;
    if (am.idx == INT_MAX) break;
    const int p = am.idx;
    if (!(d[p] > RC_DROP)) break;
    const double rpp = sqrt(d[p]);
    for (int j = threadIdx.x; j < k; j += RC_T) {
      double v;
      if (j == p) {
        v = rpp;
      } else if (taken[j]) {
        v = 0.0;
      } else {
        double x = G[(int64_t)p * k + j];
        for (int t = 0; t < s; ++t) x -= R[(int64_t)t * k + p] * R[(int64_t)t * k + j];
        v = x / rpp;
      }
      R[(int64_t)s * k + j] = v;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < k; j += RC_T)
      if (!taken[j] && j != p) d[j] -= R[(int64_t)s * k + j] * R[(int64_t)s * k + j];
    if (threadIdx.x == 0) {
      taken[p] = 1;
      sel[s] = p;
    }
    __syncthreads();
    rr = s + 1;
  }
  return rr;
}

// Back substitution R11 Y = B in place for r right-hand sides (Y column c
// at Y + c k), R11(s, s') = R(s, sel[s']) upper triangular (n x n): row by
// row from the last, each row's values then removed from the rows above it,
// all columns at once.
__device__ void rc_trsm(const double* __restrict__ R, int k, const int* __restrict__ sel, int n,
                        double* __restrict__ Y, int r) {
  for (int s = n - 1; s >= 0; --s) {
    const double piv = R[(int64_t)s * k + sel[s]];
    for (int c = threadIdx.x; c < r; c += RC_T) Y[(int64_t)c * k + s] /= piv;
    __syncthreads();
    // eight updates per thread at a time, all loads before the stores
    for (int e0 = threadIdx.x; e0 < s * r; e0 += 8 * RC_T) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * RC_T;
        if (e < s * r) {
          const int s2 = e % s, c = e / s;
          v[u] = Y[(int64_t)c * k + s2] - R[(int64_t)s2 * k + sel[s]] * Y[(int64_t)c * k + s];
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * RC_T;
        if (e < s * r) Y[(int64_t)(e / s) * k + e % s] = v[u];
      }
    }
    __syncthreads();
  }
}

}  // namespace

int64_t recompress_work_doubles(int k) { return 8 * (int64_t)k * k; }

namespace {

// The steps 1-7 for one block.  Work arrays (k x k, ld k) may be in LDS or
// in the global workspace: Gu and Gv (Gram matrices), Ru and Rv (Cholesky
// rows), K (core, then its QR, then Rv^T z products), W (R^T, rotated in
// place); Gv may share Gu's storage and K Gu's, W may share Ru's when
// Ru_keep is a copy of its own; ytmp, ztmp, Tu, Tv are global.
__device__ void rc_core(const RcDev& b, const double* __restrict__ scratch, int* __restrict__ newrank,
                        double* stage, int sst, double* Gu, double* Ru, double* Gv, double* Rv, double* K, double* W,
                        double* Ru_keep, double* ytmp, double* ztmp, double* Tu, double* Tv, double* ia, double* ib,
                        double* dd, double* sig, int* selu, int* selv, int* taken, int* order, RcMax* sh_max,
                        double* sh_sum, int* sh_rot) {
  const int m = b.m, n = b.n, k = b.k;
  const double* U = scratch + b.u_off;
  const double* V = scratch + b.v_off;
  const int tid = threadIdx.x;

  // 1. column scales (a zero column gets scale 0 and drops out)
  rc_colnorms(U, m, k, ia);
  rc_colnorms(V, n, k, ib);
  __syncthreads();
  for (int l = tid; l < k; l += RC_T) {
    const double a = ia[l], c = ib[l];
    dd[l] = a * c;  // D = diag(a b)
    ia[l] = a > 0.0 ? 1.0 / a : 0.0;
    ib[l] = c > 0.0 ? 1.0 / c : 0.0;
  }
  __syncthreads();
  // 2-3. Gram matrices and their pivoted Cholesky factors
  rc_gram(U, m, k, ia, Gu, stage, sst);
  double lim = 0.0;
  if (b.early) {
    // |U V^T|_F^2 = sum_{l,l'} d_l d_l' Gu(l,l') Gv(l,l') (Gu, Gv of the unit columns)
    rc_gram(V, n, k, ib, Gv, stage, sst);
    double x2 = 0.0;
    for (int e = tid; e < k * k; e += RC_T) {
      const int l = e % k, l2 = e / k;
      x2 += dd[l] * dd[l2] * Gu[e] * Gv[e];
    }
    x2 = rc_block_sum(x2, sh_sum);
    lim = RC_EARLY * b.tol * sqrt(fmax(x2, 0.0));
  }
  const int ru = rc_pchol(Gu, k, Ru, selu, sig, taken, sh_max, b.early ? dd : nullptr, lim, sh_sum);
  if (!b.early) rc_gram(V, n, k, ib, Gv, stage, sst);
  const int rv = rc_pchol(Gv, k, Rv, selv, sig, taken, sh_max, b.early ? dd : nullptr, lim, sh_sum);
  // 4. K = Ru D Rv^T (ru x rv, column t at K + t k)
  for (int e = tid; e < ru * rv; e += RC_T) {
    const int s = e % ru, t = e / ru;
    double x = 0.0;
    for (int l = 0; l < k; ++l) x += Ru[(int64_t)s * k + l] * dd[l] * Rv[(int64_t)t * k + l];
    K[(int64_t)t * k + s] = x;
  }
  __syncthreads();
  // Ru is kept where the last steps read it (W may take its place)
  if (Ru_keep != Ru)
    for (int e = tid; e < ru * k; e += RC_T) Ru_keep[e] = Ru[e];
  __syncthreads();
  // 5. Householder QR of K with column pivoting (largest remaining column
  // first, the first index on ties): R in the upper triangle of K, the
  // column order in perm; W = R^T.  One-sided Jacobi on the columns of R^T
  // (the preconditioning of Drmac and Veselic, SIAM J. Matrix Anal. Appl.
  // 29 (2008)) converges in about half the sweeps it takes on K itself, and
  // the rotations need not be kept: with R^T Z = W S', the right singular
  // vectors of K are P W, the left ones times s come from K (P W).
  int* perm = taken;  // free after the Cholesky steps
  const int lane = tid & 63, wid = tid >> 6;
  for (int j = tid; j < rv; j += RC_T) perm[j] = j;
  for (int j = wid; j < rv; j += RC_W) {  // column norms^2 (sig holds them during the QR)
    double s2 = 0.0;
    for (int i = lane; i < ru; i += 64) {
      const double x = K[(int64_t)j * k + i];
      s2 += x * x;
    }
    s2 = wave_sum(s2);
    if (lane == 0) sig[j] = s2;
  }
  __syncthreads();
  const int qmax = min(ru, rv);
  int kq = 0;
  for (int s = 0; s < qmax; ++s) {
    RcMax am{-1.0, INT_MAX};
    for (int j = s + tid; j < rv; j += RC_T) am = rc_better(am, RcMax{sig[j], j});
    am = rc_block_max(am, sh_max);
    if (!(am.mag > 0.0)) break;
    const int p = am.idx;
    double* ks = K + (int64_t)s * k;
    if (p != s) {
      double* kp = K + (int64_t)p * k;
      for (int i = tid; i < ru; i += RC_T) {
        const double x = ks[i];
        ks[i] = kp[i];
        kp[i] = x;
      }
      if (tid == 0) {
        const int t = perm[s];
        perm[s] = perm[p];
        perm[p] = t;
        sig[p] = sig[s];
      }
    }
    __syncthreads();
    // reflector I - beta v v^T with v = x - alpha e_1 (x: rows s.. of the
    // column, |x|^2 = am.mag), stored in place of the column
    const double x0 = ks[s];
    const double nx = sqrt(am.mag);
    const double alpha = x0 >= 0.0 ? -nx : nx;
    const double beta = 1.0 / (nx * (nx + fabs(x0)));  // 2 / |v|^2
    __syncthreads();
    if (tid == 0) ks[s] = x0 - alpha;
    __syncthreads();
    for (int j = s + 1 + wid; j < rv; j += RC_W) {
      double* kj = K + (int64_t)j * k;
      double dot = 0.0;
      for (int i = s + lane; i < ru; i += 64) dot += ks[i] * kj[i];
      dot = wave_sum(dot) * beta;
      double s2 = 0.0;
      for (int i = s + lane; i < ru; i += 64) {
        const double x = kj[i] - dot * ks[i];
        kj[i] = x;
        if (i > s) s2 += x * x;
      }
      s2 = wave_sum(s2);
      if (lane == 0) sig[j] = s2;  // the next step's norms (rows s+1..)
    }
    __syncthreads();
    if (tid == 0) ks[s] = alpha;
    __syncthreads();
    kq = s + 1;
  }
  // W = R^T (rv x kq): column i holds row i of R
  double fro2 = 0.0;  // |K|_F^2 = |R|_F^2, which the rotations keep
  if (W != K) {
    for (int e = tid; e < kq * rv; e += RC_T) {
      const int j = e % rv, i = e / rv;
      const double x = j >= i ? K[(int64_t)j * k + i] : 0.0;
      W[(int64_t)i * k + j] = x;
      fro2 += x * x;
    }
  } else {
    // in place: R(i, j), j > i, sits at K[j k + i] and goes to K[i k + j]
    // (below the diagonal of K: the Householder vectors, no longer needed);
    // then the places it came from are cleared
    for (int e = tid; e < kq * rv; e += RC_T) {
      const int j = e % rv, i = e / rv;
      if (j > i) W[(int64_t)i * k + j] = K[(int64_t)j * k + i];
    }
    __syncthreads();
    for (int e = tid; e < kq * rv; e += RC_T) {
      const int j = e % rv, i = e / rv;
      if (j < i) W[(int64_t)i * k + j] = 0.0;  // R(j, i) read above (j < i < kq)
      const double x = W[(int64_t)i * k + j];
      fro2 += x * x;
    }
  }
  fro2 = rc_block_sum(fro2, sh_sum);
  const double floor2 = RC_JFLOOR * fro2;
  // one-sided Jacobi on the columns of W: round-robin pairs over np
  // positions (np = kq rounded up to even; position kq is a dummy)
  const int np = (kq + 1) & ~1;
  const int g = tid / RC_LP, gl = tid % RC_LP;
  for (int sweep = 0; sweep < RC_SWEEPS && np >= 2; ++sweep) {
    if (tid == 0) *sh_rot = 0;
    __syncthreads();
    int rotated = 0;
    for (int step = 0; step < np - 1; ++step) {
      for (int pi = g; pi < np / 2; pi += RC_GROUPS) {
        auto pos = [&](int j) { return j == 0 ? 0 : ((j - 1 + step) % (np - 1)) + 1; };
        int p = pos(pi), q = pos(np - 1 - pi);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        if (q >= kq) continue;
        double* wp = W + (int64_t)p * k;
        double* wq = W + (int64_t)q * k;
        // the lane's slices of both columns in registers: every load is
        // issued before any store (the stores of a rotation would otherwise
        // hold up the next loads by a memory latency each)
        double xp[RC_PL], xq[RC_PL];
#pragma unroll
        for (int u = 0; u < RC_PL; ++u) {
          const int i = gl + u * RC_LP;
          xp[u] = i < rv ? wp[i] : 0.0;
          xq[u] = i < rv ? wq[i] : 0.0;
        }
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int u = 0; u < RC_PL; ++u) {
          al += xp[u] * xp[u];
          be += xq[u] * xq[u];
          ga += xp[u] * xq[u];
        }
        al = grp_sum(al);
        be = grp_sum(be);
        ga = grp_sum(ga);
        // a pair counts as orthogonal when |g| is below RC_JTOL of sqrt(a b),
        // or when both columns are rounding noise (such pairs would keep
        // rotating on it).  Every column above that floor is made
        // orthogonal to the others to RC_JTOL relative to the two norms:
        // the right vectors are the normalised columns, and a kept column
        // of norm s_t leaning toward one of norm s_1 by d would bring
        // d s_1 of the larger direction into K x_t.
        if (ga != 0.0 && fabs(ga) > RC_JTOL * sqrt(al * be) && fmax(al, be) > floor2) {
          const double zeta = (be - al) / (2.0 * ga);
          const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + tt * tt), sn = c * tt;
#pragma unroll
          for (int u = 0; u < RC_PL; ++u) {
            const int i = gl + u * RC_LP;
            if (i < rv) {
              wp[i] = c * xp[u] - sn * xq[u];
              wq[i] = sn * xp[u] + c * xq[u];
            }
          }
          rotated = 1;
        }
      }
      __syncthreads();
    }
    if (rotated) atomicOr(sh_rot, 1);
    __syncthreads();
    const int any = *sh_rot;
    __syncthreads();
    if (!any) break;
  }
  // singular values (column norms of W), their descending order and the rank
  for (int t = tid; t < kq; t += RC_T) {
    double s2 = 0.0;
    for (int i = 0; i < rv; ++i) s2 += W[(int64_t)t * k + i] * W[(int64_t)t * k + i];
    sig[t] = sqrt(s2);
  }
  __syncthreads();
  for (int t = tid; t < kq; t += RC_T) {
    int rank = 0;
    for (int u = 0; u < kq; ++u) rank += (sig[u] > sig[t] || (sig[u] == sig[t] && u < t)) ? 1 : 0;
    order[rank] = t;
  }
  __syncthreads();
  double tot = 0.0;
  for (int t = tid; t < kq; t += RC_T) tot += sig[t] * sig[t];
  tot = rc_block_sum(tot, sh_sum);
  int r = 0;
  if (tid == 0 && tot > 0.0) {
    const double lim = b.tol * sqrt(tot);
    double tail2 = 0.0;  // sum of the discarded squares, from the smallest up
    r = kq;
    for (int c = kq - 1; c >= 1; --c) {
      const double s = sig[order[c]];
      tail2 += s * s;
      if (sqrt(tail2) <= lim) r = c;
      else break;
    }
    newrank[b.out] = r;
  } else if (tid == 0) {
    newrank[b.out] = 0;
  }
  if (tid == 0) *sh_rot = r;
  __syncthreads();
  r = *sh_rot;
  // 6. kept right singular vectors in Rv coordinates, z_c = P w_t / s_t
  // (t = order[c]), and left ones times s in Ru coordinates,
  // y_c = K z_c = Ru D (Rv^T z_c); then the triangular solves on the
  // selected rows, all kept columns together
  for (int e = tid; e < r * rv; e += RC_T) {
    const int j = e % rv, c = e / rv;
    const int t = order[c];
    ztmp[(int64_t)c * k + perm[j]] = W[(int64_t)t * k + j] / sig[t];
  }
  __syncthreads();
  double* Ab = K;  // k x r: K is free once its R went to W
  for (int e = tid; e < k * r; e += RC_T) {
    const int l = e % k, c = e / k;
    double x = 0.0;
    for (int t = 0; t < rv; ++t) x += Rv[(int64_t)t * k + l] * ztmp[(int64_t)c * k + t];
    Ab[(int64_t)c * k + l] = x * dd[l];
  }
  __syncthreads();
  for (int e = tid; e < ru * r; e += RC_T) {
    const int s = e % ru, c = e / ru;
    double x = 0.0;
    for (int l = 0; l < k; ++l) x += Ru_keep[(int64_t)s * k + l] * Ab[(int64_t)c * k + l];
    ytmp[(int64_t)c * k + s] = x;
  }
  __syncthreads();
  rc_trsm(Ru_keep, k, selu, ru, ytmp, r);
  rc_trsm(Rv, k, selv, rv, ztmp, r);
  // 7. Tu (k x r) and Tv (k x r)
  for (int e = tid; e < r * k; e += RC_T) {
    Tu[e % k + (int64_t)(e / k) * k] = 0.0;
    Tv[e % k + (int64_t)(e / k) * k] = 0.0;
  }
  __syncthreads();
  for (int e = tid; e < r * ru; e += RC_T) {
    const int s = e % ru, c = e / ru;
    Tu[(int64_t)c * k + selu[s]] = ytmp[(int64_t)c * k + s] * ia[selu[s]];
  }
  for (int e = tid; e < r * rv; e += RC_T) {
    const int s = e % rv, c = e / rv;
    Tv[(int64_t)c * k + selv[s]] = ztmp[(int64_t)c * k + s] * ib[selv[s]];
  }
}

}  // namespace

// Ranks and transforms of one chunk of blocks, work arrays in the global
// workspace (any rank up to RC_KMAX).  Workspace per block (doubles, ld k):
// Gu (then y) | Ru | Gv (then z) | Rv | K | W | Tu | Tv.
__global__ __launch_bounds__(RC_T) void k_recompress(const RcDev* __restrict__ blocks, const double* __restrict__ scratch,
                                                     double* __restrict__ work, int* __restrict__ newrank) {
  __shared__ double stage[RC_ROWS * RC_KMAX];
  __shared__ double ia[RC_KMAX], ib[RC_KMAX], dd[RC_KMAX], sig[RC_KMAX];
  __shared__ int selu[RC_KMAX], selv[RC_KMAX], taken[RC_KMAX], order[RC_KMAX];
  __shared__ RcMax sh_max[RC_W];
  __shared__ double sh_sum[RC_W];
  __shared__ int sh_rot;
  const RcDev b = blocks[blockIdx.x];
  const int64_t kk = (int64_t)b.k * b.k;
  double* W = work + b.w_off;
  rc_core(b, scratch, newrank, stage, RC_KMAX, W, W + kk, W + 2 * kk, W + 3 * kk, W + 4 * kk, W + 5 * kk, W + kk, W,
          W + 2 * kk, W + 6 * kk, W + 7 * kk, ia, ib, dd, sig, selu, selv, taken, order, sh_max, sh_sum, &sh_rot);
}

// The same for blocks of rank up to KM with the k x k arrays in LDS (three
// KM x KM areas: A holds Gu, then Gv, then K; B holds Ru, then W; C holds
// Rv); Ru is copied to the workspace before W overwrites it.  The steps and
// their order are those of k_recompress, so both give the same results.
template <int KM>
__global__ __launch_bounds__(RC_T) void k_recompress_lds(const RcDev* __restrict__ blocks,
                                                         const double* __restrict__ scratch, double* __restrict__ work,
                                                         int* __restrict__ newrank) {
  __shared__ double stage[RC_ROWS * KM];
  __shared__ double A[KM * KM], B[KM * KM], Cm[KM * KM];
  __shared__ double ia[KM], ib[KM], dd[KM], sig[KM];
  __shared__ int selu[KM], selv[KM], taken[KM], order[KM];
  __shared__ RcMax sh_max[RC_W];
  __shared__ double sh_sum[RC_W];
  __shared__ int sh_rot;
  const RcDev b = blocks[blockIdx.x];
  const int64_t kk = (int64_t)b.k * b.k;
  double* W = work + b.w_off;
  rc_core(b, scratch, newrank, stage, KM, A, B, A, Cm, A, B, W + kk, W, W + 2 * kk, W + 6 * kk, W + 7 * kk, ia, ib,
          dd, sig, selu, selv, taken, order, sh_max, sh_sum, &sh_rot);
}

// U' = U Tu and V' = V Tv into the staging buffer (m x r and n x r,
// column-major at du and dv), 16 output columns at a time with the
// transform columns in LDS.
template <class ST>
__global__ __launch_bounds__(RC_T) void k_recompress_apply(const RcDev* __restrict__ blocks,
                                                           const double* __restrict__ scratch,
                                                           const double* __restrict__ work,
                                                           const int* __restrict__ newrank, ST* __restrict__ stage) {
  __shared__ double T[RC_KMAX * 16];
  const RcDev b = blocks[blockIdx.x];
  const int k = b.k;
  const int r = newrank[b.out];
  const double* Wk = work + b.w_off;
  for (int side = 0; side < 2; ++side) {
    const int len = side ? b.n : b.m;
    const double* P = scratch + (side ? b.v_off : b.u_off);
    const double* Tm = Wk + (int64_t)(side ? 7 : 6) * k * k;
    ST* out = stage + (side ? b.dv : b.du);
    for (int c0 = 0; c0 < r; c0 += 16) {
      const int nc = min(16, r - c0);
      __syncthreads();
      for (int e = threadIdx.x; e < k * 16; e += RC_T) {
        const int l = e % k, c = e / k;
        T[l * 16 + c] = c < nc ? Tm[(int64_t)(c0 + c) * k + l] : 0.0;
      }
      __syncthreads();
      for (int i = threadIdx.x; i < len; i += RC_T) {
        double acc[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) acc[c] = 0.0;
        for (int l = 0; l < k; ++l) {
          const double x = P[(int64_t)l * len + i];
#pragma unroll
          for (int c = 0; c < 16; ++c) acc[c] += x * T[l * 16 + c];
        }
        for (int c = 0; c < nc; ++c) out[(int64_t)(c0 + c) * len + i] = (ST)acc[c];
      }
    }
  }
}

namespace {

// One stream per device (default priority) for the bucket of the widest
// blocks, which then runs beside the others: its blocks are few and long,
// so alone they would leave most compute units idle.  Created on first use
// and kept until the process ends; callers on several threads share it (a
// call's work on it is ordered by that call's own events).
hipStream_t side_stream(int device) {
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  std::lock_guard<std::mutex> lk(mu);
  hipStream_t& st = streams[device];
  if (!st) HM_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  return st;
}

struct CallEvents {
  hipEvent_t fork = nullptr, join = nullptr;
  CallEvents() {
    HM_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    HM_HIP(hipEventCreateWithFlags(&join, hipEventDisableTiming));
  }
  ~CallEvents() {
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
  }
  CallEvents(const CallEvents&) = delete;
  CallEvents& operator=(const CallEvents&) = delete;
};

}  // namespace

void recompress_blocks(std::vector<RcDev>& blocks, const double* scratch, void* stage, bool stage_f64,
                       int* d_newrank, hipStream_t s) {
  if (blocks.empty()) return;
  // blocks by rank: the LDS variants for ranks up to 16, 32 and 64, the
  // global-workspace kernel above
  std::vector<RcDev> bucket[4];
  for (const RcDev& b : blocks) bucket[b.k <= 16 ? 0 : b.k <= 32 ? 1 : b.k <= 64 ? 2 : 3].push_back(b);
  // the widest blocks on the side stream with a workspace of their own when
  // there are others to run beside them (every block reads only its own
  // crosses and writes only its own factors and rank)
  const bool split = !bucket[3].empty() && (!bucket[0].empty() || !bucket[1].empty() || !bucket[2].empty());
  // chunks bounded by a workspace budget (a block needs 8 k^2 doubles): one
  // launch should hold enough blocks for several workgroups per compute
  // unit, since each block's steps are latency-bound; at most 2 GB in all
  int64_t need[2] = {0, 0};  // [0]: the buckets on s, [1]: the side bucket
  for (int v = 0; v < 4; ++v)
    for (const RcDev& b : bucket[v]) need[split && v == 3 ? 1 : 0] += recompress_work_doubles(b.k) * 8;
  const int64_t cap = split ? (int64_t)1 << 30 : (int64_t)2 << 30;
  int64_t budget[2];
  DevBuf work[2];
  for (int w = 0; w < (split ? 2 : 1); ++w) {
    // the widest rank this workspace serves
    const int kmax = (w == 1 || (!split && !bucket[3].empty())) ? RC_KMAX : 64;
    budget[w] = std::max<int64_t>(recompress_work_doubles(kmax) * 8, std::min<int64_t>(need[w], cap));
    work[w].alloc((size_t)budget[w]);
  }
  std::unique_ptr<CallEvents> ev;
  hipStream_t side = nullptr;
  std::vector<DevBuf> descs;
  // the side bucket first: its launch is the longest
  const int order[4] = {3, 0, 1, 2};
  for (int oi = 0; oi < 4; ++oi) {
    const int v = order[oi];
    std::vector<RcDev>& bl = bucket[v];
    if (bl.empty()) continue;
    const int w = split && v == 3 ? 1 : 0;
    std::vector<size_t> starts;
    int64_t used = budget[w];
    for (size_t q = 0; q < bl.size(); ++q) {
      const int64_t nd = recompress_work_doubles(bl[q].k) * 8;
      if (used + nd > budget[w]) {
        starts.push_back(q);
        used = 0;
      }
      bl[q].w_off = used / 8;
      used += nd;
    }
    starts.push_back(bl.size());
    descs.emplace_back();
    upload(descs.back(), bl, s);
    hipStream_t st = s;
    if (w == 1) {
      int dev = 0;
      HM_HIP(hipGetDevice(&dev));
      side = side_stream(dev);
      ev = std::make_unique<CallEvents>();
      HM_HIP(hipEventRecord(ev->fork, s));  // after the crosses and the descriptors
      HM_HIP(hipStreamWaitEvent(side, ev->fork, 0));
      st = side;
    }
    double* wk = work[w].get<double>();
    for (size_t c = 0; c + 1 < starts.size(); ++c) {
      const unsigned cnt = (unsigned)(starts[c + 1] - starts[c]);
      const RcDev* bp = descs.back().get<RcDev>() + starts[c];
      if (v == 0)
        hipLaunchKernelGGL(k_recompress_lds<16>, dim3(cnt), dim3(RC_T), 0, st, bp, scratch, wk, d_newrank);
      else if (v == 1)
        hipLaunchKernelGGL(k_recompress_lds<32>, dim3(cnt), dim3(RC_T), 0, st, bp, scratch, wk, d_newrank);
      else if (v == 2)
        hipLaunchKernelGGL(k_recompress_lds<64>, dim3(cnt), dim3(RC_T), 0, st, bp, scratch, wk, d_newrank);
      else
        hipLaunchKernelGGL(k_recompress, dim3(cnt), dim3(RC_T), 0, st, bp, scratch, wk, d_newrank);
      if (stage_f64)
        hipLaunchKernelGGL(k_recompress_apply<double>, dim3(cnt), dim3(RC_T), 0, st, bp, scratch, wk,
                           (const int*)d_newrank, (double*)stage);
      else
        hipLaunchKernelGGL(k_recompress_apply<float>, dim3(cnt), dim3(RC_T), 0, st, bp, scratch, wk,
                           (const int*)d_newrank, (float*)stage);
      HM_HIP(hipGetLastError());
    }
    if (w == 1) HM_HIP(hipEventRecord(ev->join, side));
  }
  if (ev) HM_HIP(hipStreamWaitEvent(s, ev->join, 0));
  // the workspaces and the descriptors are released when the work is done
  HM_HIP(hipStreamSynchronize(s));
}

}  // namespace hm
