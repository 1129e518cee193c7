// Hierarchical block LU of the reflection matrix on gfx950 (Sec. 5.1) and
// its forward / backward substitution (Sec. 5.2).
//
// C = I - diag(1 - eps) F is kept in the block structure of F (Algorithm 2):
// every node of the block tree is subdivided 2 x 2, dense, or low rank
// (U V^T), FP64.  The factorisation follows the paper's four steps on every
// subdivided diagonal block:
//   1. L11 U11 = C11 (recursively; a dense LU without row exchanges in the
//      leaves),
//   2. U12 = L11^-1 C12 (forward substitution over the block structure),
//   3. L21 = C21 U11^-1 (backward substitution),
//   4. L22 U22 = C22 - L21 U12 (the Schur complement, then recursively),
// with every addition into a low-rank block followed by a truncation at the
// relative accuracy eps_rel from the singular values (the recompression
// kernels: Gram matrices, pivoted Cholesky, one-sided Jacobi).  A product
// that lands in a low-rank block is formed in low-rank form first: through
// the low-rank factor when one operand is low rank, with an identity factor
// on the side of a leaf cluster when one operand is dense, and from the
// agglomerated 2 x 2 pieces (truncated) when both are subdivided.
//
// The recursion runs on the host; every numerical step (leaf LU, triangular
// solves, products, truncations) is a kernel on the context's stream.  The
// solve x = U^-1 (L^-1 b) walks the same blocks with the right-hand sides as
// dense column blocks.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>
#include <mutex>
#include <vector>

#include "dev_common.hpp"
#include "hm_internal.hpp"
#include "recompress.hpp"

namespace hm {

namespace {

// ------------------------------------------------------------------ kernels
constexpr int GT = 16;  // tile edge of the product kernel

// C = beta C + alpha op(A) op(B); C m x n (ldc), op(A) m x kk, op(B) kk x n,
// all column-major; op = transpose when the flag is set.
__global__ __launch_bounds__(GT* GT) void k_dgemm(int64_t m, int64_t n, int64_t kk, double alpha,
                                                  const double* __restrict__ A, int64_t lda, int ta,
                                                  const double* __restrict__ B, int64_t ldb, int tb, double beta,
                                                  double* __restrict__ C, int64_t ldc) {
  __shared__ double As[GT][GT + 1], Bs[GT][GT + 1];
  const int tx = threadIdx.x % GT, ty = threadIdx.x / GT;
  const int64_t row = (int64_t)blockIdx.x * GT + tx, col = (int64_t)blockIdx.y * GT + ty;
  double acc = 0.0;
  for (int64_t k0 = 0; k0 < kk; k0 += GT) {
    // As[tx][ty] = op(A)(blockrow + tx, k0 + ty); Bs[tx][ty] = op(B)(k0 + tx, blockcol + ty)
    {
      const int64_t r = (int64_t)blockIdx.x * GT + tx, k = k0 + ty;
      double v = 0.0;
      if (r < m && k < kk) v = ta ? A[r * lda + k] : A[k * lda + r];
      As[tx][ty] = v;
    }
    {
      const int64_t k = k0 + tx, c = (int64_t)blockIdx.y * GT + ty;
      double v = 0.0;
      if (k < kk && c < n) v = tb ? B[k * ldb + c] : B[c * ldb + k];
      Bs[tx][ty] = v;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < GT; ++q) acc += As[tx][q] * Bs[q][ty];
    __syncthreads();
  }
  if (row < m && col < n) {
    double* c = C + col * ldc + row;
    *c = beta == 0.0 ? alpha * acc : beta * *c + alpha * acc;
  }
}

// dst = alpha src for an m x n block (column-major, own leading dimensions);
// trans: dst(i, j) = alpha src(j, i)
__global__ void k_dcopy2d(int64_t m, int64_t n, double alpha, const double* __restrict__ src, int64_t lds, int trans,
                          double* __restrict__ dst, int64_t ldd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * n) return;
  const int64_t i = e % m, j = e / m;
  dst[j * ldd + i] = alpha * (trans ? src[i * lds + j] : src[j * lds + i]);
}

// dst += alpha src (m x n)
__global__ void k_daxpy2d(int64_t m, int64_t n, double alpha, const double* __restrict__ src, int64_t lds,
                          double* __restrict__ dst, int64_t ldd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * n) return;
  const int64_t i = e % m, j = e / m;
  dst[j * ldd + i] += alpha * src[j * lds + i];
}

// dst = diag * I (m x n)
__global__ void k_dset2d(int64_t m, int64_t n, double diag, double* __restrict__ dst, int64_t ldd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * n) return;
  const int64_t i = e % m, j = e / m;
  dst[j * ldd + i] = i == j ? diag : 0.0;
}

// In-place LU without row exchanges of an m x m block (one workgroup): for
// each k, the column below the pivot is divided by it and the trailing block
// takes the rank-1 update, as A[k+1:, k] /= A[k, k];
// A[k+1:, k+1:] -= outer(A[k+1:, k], A[k, k+1:]).  Blocks up to 64 x 64 are
// factorised in LDS.
#pragma clang fp contract(off)
__global__ __launch_bounds__(256) void k_dlu(double* __restrict__ A, int m, int64_t lda) {
  __shared__ double S[64 * 64];
  const bool lds = m <= 64;
  double* W = lds ? S : A;
  const int64_t ld = lds ? m : lda;
  if (lds)
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) S[e] = A[(int64_t)(e / m) * lda + e % m];
  __syncthreads();
  for (int k = 0; k < m - 1; ++k) {
    const double piv = W[k * ld + k];
    for (int i = k + 1 + threadIdx.x; i < m; i += blockDim.x) W[k * ld + i] = W[k * ld + i] / piv;
    __syncthreads();
    const int r = m - k - 1;
    for (int e = threadIdx.x; e < r * r; e += blockDim.x) {
      const int i = k + 1 + e % r, j = k + 1 + e / r;
      W[j * ld + i] = W[j * ld + i] - W[k * ld + i] * W[j * ld + k];
    }
    __syncthreads();
  }
  if (lds)
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) A[(int64_t)(e / m) * lda + e % m] = S[e];
}
#pragma clang fp contract(on)

// Triangular solves with a factorised dense block T (m x m): one thread per
// right-hand side.  mode 0: X <- L^-1 X (unit lower); 1: X <- U^-1 X;
// 2: X <- U^-T X (X m x c, column j at X + j ldx); 3: X <- X U^-1 (X r x m,
// row i at X + i with stride ldx).
__global__ void k_dtrsm(const double* __restrict__ T, int m, int64_t ldt, double* __restrict__ X, int64_t ldx,
                        int64_t c, int mode) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= c) return;
  if (mode == 3) {
    double* x = X + j;  // row j of an r x m block: entries at x[q ldx]
    for (int q = 0; q < m; ++q) {
      double v = x[q * ldx];
      for (int p = 0; p < q; ++p) v -= x[p * ldx] * T[(int64_t)q * ldt + p];
      x[q * ldx] = v / T[(int64_t)q * ldt + q];
    }
    return;
  }
  double* x = X + j * ldx;
  if (mode == 0) {
    for (int i = 1; i < m; ++i) {
      double v = x[i];
      for (int p = 0; p < i; ++p) v -= T[(int64_t)p * ldt + i] * x[p];
      x[i] = v;
    }
  } else if (mode == 1) {
    for (int i = m - 1; i >= 0; --i) {
      double v = x[i];
      for (int p = i + 1; p < m; ++p) v -= T[(int64_t)p * ldt + i] * x[p];
      x[i] = v / T[(int64_t)i * ldt + i];
    }
  } else {
    for (int i = 0; i < m; ++i) {
      double v = x[i];
      for (int p = 0; p < i; ++p) v -= T[(int64_t)i * ldt + p] * x[p];
      x[i] = v / T[(int64_t)i * ldt + i];
    }
  }
}

// The same solves for modes 0 and 1 with a leaf of at most 64 rows and few
// right-hand sides: one wave per right-hand side, the block and the column
// in LDS, lane i owning row i; the solve goes column by column of T (the
// row-by-row loop above leaves one thread walking the whole block).  Mode
// 0 subtracts the terms of each row in the same order as above.
constexpr int TRSM_LDS_M = 64;
__global__ __launch_bounds__(64) void k_dtrsm_lds(const double* __restrict__ T, int m, int64_t ldt,
                                                  double* __restrict__ X, int64_t ldx, int mode) {
  __shared__ double Ts[TRSM_LDS_M * (TRSM_LDS_M + 1)];
  __shared__ double xs[TRSM_LDS_M];
  const int i = threadIdx.x;
  double* x = X + (int64_t)blockIdx.x * ldx;
  for (int e = i; e < m * m; e += 64) {
    const int p = e / m, r = e - p * m;
    Ts[p * (TRSM_LDS_M + 1) + r] = T[(int64_t)p * ldt + r];
  }
  xs[i] = i < m ? x[i] : 0.0;
  __syncthreads();
  if (mode == 0) {
    for (int p = 0; p < m - 1; ++p) {
      if (i > p && i < m) xs[i] -= Ts[p * (TRSM_LDS_M + 1) + i] * xs[p];
      __syncthreads();
    }
  } else {
    for (int p = m - 1; p >= 0; --p) {
      if (i == p) xs[p] /= Ts[p * (TRSM_LDS_M + 1) + p];
      __syncthreads();
      if (i < p) xs[i] -= Ts[p * (TRSM_LDS_M + 1) + i] * xs[p];
      __syncthreads();
    }
  }
  if (i < m) x[i] = xs[i];
}

// One leaf of a flattened subtree for the substitutions: rows [ro, ro+m)
// and columns [co, co+n) relative to the subtree; dense D (ld m) or low rank
// U (m x k), V (n x k); toff: first row of its k x c intermediate V^T x in
// the (sum of ranks) x c row-major buffer of the subtree.
struct FlatLeaf {
  const double* D;
  const double* U;
  const double* V;
  int64_t toff;
  int32_t ro, co, m, n, k, kind;  // kind 1 dense, 2 low rank
};

// t = V^T x for every low-rank leaf (one workgroup per leaf, one wave per
// rank column, lanes over rows)
__global__ __launch_bounds__(256) void k_flat_t(const FlatLeaf* __restrict__ lv, const double* __restrict__ X,
                                                int64_t ldx, int c, double* __restrict__ t) {
  const FlatLeaf L = lv[blockIdx.x];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int l = w; l < L.k; l += 4)
    for (int q = 0; q < c; ++q) {
      double a = 0.0;
      for (int j = lane; j < L.n; j += 64) a += L.V[(int64_t)l * L.n + j] * X[(int64_t)q * ldx + L.co + j];
      a = wave_sum(a);
      if (lane == 0) t[(L.toff + l) * c + q] = a;
    }
}

// y += alpha (leaf x) for every leaf, added with atomics (leaves of a
// subtree cover disjoint column ranges of the same rows)
__global__ __launch_bounds__(256) void k_flat_apply(const FlatLeaf* __restrict__ lv, const double* __restrict__ X,
                                                    int64_t ldx, int c, const double* __restrict__ t, double alpha,
                                                    double* __restrict__ Y, int64_t ldy) {
  const FlatLeaf L = lv[blockIdx.x];
  for (int i = threadIdx.x; i < L.m; i += blockDim.x)
    for (int q = 0; q < c; ++q) {
      double a = 0.0;
      if (L.kind == 1) {
        for (int j = 0; j < L.n; ++j) a += L.D[(int64_t)j * L.m + i] * X[(int64_t)q * ldx + L.co + j];
      } else {
        for (int l = 0; l < L.k; ++l) a += L.U[(int64_t)l * L.m + i] * t[(L.toff + l) * c + q];
      }
      atomicAdd(Y + (int64_t)q * ldy + L.ro + i, alpha * a);
    }
}

template <class VT>
__global__ void k_hlu_gather(const int32_t* __restrict__ perm, const double* __restrict__ in, int64_t ldi,
                             double* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i < n) out[i + j * n] = in[perm[i] + j * ldi];
}

__global__ void k_hlu_scatter(const int32_t* __restrict__ perm, const double* __restrict__ in, double* __restrict__ out,
                              int64_t ldo, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i < n) out[perm[i] + j * ldo] = in[i + j * n];
}

__global__ void k_hlu_om(const int32_t* __restrict__ perm, const double* __restrict__ eps, double* __restrict__ om,
                         int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) om[i] = 1.0 - eps[perm[i]];
}

// ------------------------------------------------------------------ host matrices
struct MatV {  // non-owning column-major view
  double* p = nullptr;
  int64_t rows = 0, cols = 0, ld = 1;
  MatV sub(int64_t r0, int64_t nr, int64_t c0, int64_t nc) const { return MatV{p + c0 * ld + r0, nr, nc, ld}; }
  MatV rowsv(int64_t r0, int64_t nr) const { return sub(r0, nr, 0, cols); }
};

struct MatO {  // owning, ld = rows
  DevBuf buf;
  int64_t rows = 0, cols = 0;
  MatV v() const { return MatV{buf.get<double>(), rows, cols, std::max<int64_t>(1, rows)}; }
};

unsigned blocks_for(int64_t e) { return (unsigned)std::max<int64_t>(1, (e + 255) / 256); }

}  // namespace

// The factorised matrix (opaque at the ABI).
}  // namespace hm

struct hm_hlu {
  struct Node {
    int32_t r0, r1, c0, c1;
    int kind = 1;  // 0: subdivided, 1: dense, 2: low rank
    int ch[2][2] = {{-1, -1}, {-1, -1}};
    hm::MatO D, U, V;  // dense block; low-rank factors (U m x k, V n x k)
    int32_t m() const { return r1 - r0; }
    int32_t n() const { return c1 - c0; }
  };
  int device = 0;
  int64_t n = 0;
  double tol = 1e-6;
  std::vector<int32_t> perm;
  hm::DevBuf d_perm;
  std::vector<Node> nodes;
  int root = 0;
  double factor_seconds = 0.0;
  int64_t truncations = 0;
  // the off-diagonal subtrees the substitutions multiply, flattened after
  // the factorisation: node -> (device leaf list, leaves, low-rank leaves
  // first, their count, intermediate size per right-hand side)
  struct Flat {
    hm::DevBuf leaves;
    int n = 0, nlr = 0;
    int64_t tsize = 0;
  };
  std::vector<Flat> flat;  // indexed by node
  // The substitutions for a given number of right-hand sides, captured as
  // a graph at the first solve with that number (persistent work vector
  // and per-node intermediates, so that the graph's pointers stay valid);
  // solves on these factors are serialised by solve_mu.  At most
  // MAX_GRAPHS counts are kept, the most recently used first.
  struct SolveGraph {
    int nrhs = 0;
    hm::DevBuf W;
    std::vector<hm::DevBuf> t;  // indexed by node
    hipGraphExec_t exec = nullptr;
    ~SolveGraph() {
      if (exec) (void)hipGraphExecDestroy(exec);
    }
  };
  static constexpr size_t MAX_GRAPHS = 4;
  std::mutex solve_mu;
  std::vector<std::unique_ptr<SolveGraph>> graphs;
  hipStream_t cap = nullptr;  // private stream used only to capture
  ~hm_hlu() {
    graphs.clear();
    if (cap) (void)hipStreamDestroy(cap);
  }
};

namespace hm {

namespace {

using Node = hm_hlu::Node;

struct Hlu {
  hm_hlu& H;
  hipStream_t s;
  double tol;
  // low-rank blocks that took additions since their last truncation; they
  // are truncated together (one batched launch) before the next
  // factorisation or block substitution step, or at once when their rank
  // passes RC_KMAX
  std::vector<char> dirty;
  std::vector<int> dirty_list;

  Node& nd(int i) { return H.nodes[i]; }

  MatO alloc(int64_t r, int64_t c, bool zero = true) {
    MatO o;
    o.rows = r;
    o.cols = c;
    o.buf.alloc((size_t)std::max<int64_t>(1, r * c) * 8);
    if (zero && r * c > 0)
      hipLaunchKernelGGL(k_dset2d, dim3(blocks_for(r * c)), dim3(256), 0, s, r, c, 0.0, o.buf.get<double>(), r);
    return o;
  }
  MatO identity(int64_t r) {
    MatO o = alloc(r, r, false);
    if (r > 0) hipLaunchKernelGGL(k_dset2d, dim3(blocks_for(r * r)), dim3(256), 0, s, r, r, 1.0, o.buf.get<double>(), r);
    return o;
  }
  void copy(const MatV& src, const MatV& dst, double alpha = 1.0, bool trans = false) {
    const int64_t m = dst.rows, n = dst.cols;
    if (m * n == 0) return;
    hipLaunchKernelGGL(k_dcopy2d, dim3(blocks_for(m * n)), dim3(256), 0, s, m, n, alpha, (const double*)src.p, src.ld,
                       trans ? 1 : 0, dst.p, dst.ld);
  }
  void axpy(double alpha, const MatV& src, const MatV& dst) {
    const int64_t m = dst.rows, n = dst.cols;
    if (m * n == 0) return;
    hipLaunchKernelGGL(k_daxpy2d, dim3(blocks_for(m * n)), dim3(256), 0, s, m, n, alpha, (const double*)src.p, src.ld,
                       dst.p, dst.ld);
  }
  // C = beta C + alpha op(A) op(B)
  void gemm(bool ta, bool tb, double alpha, const MatV& A, const MatV& B, double beta, const MatV& C) {
    const int64_t m = C.rows, n = C.cols, kk = ta ? A.rows : A.cols;
    if (m == 0 || n == 0) return;
    if (kk == 0) {
      if (beta == 0.0) hipLaunchKernelGGL(k_dset2d, dim3(blocks_for(m * n)), dim3(256), 0, s, m, n, 0.0, C.p, C.ld);
      return;
    }
    dim3 grid((unsigned)((m + GT - 1) / GT), (unsigned)((n + GT - 1) / GT));
    hipLaunchKernelGGL(k_dgemm, grid, dim3(GT * GT), 0, s, m, n, kk, alpha, (const double*)A.p, A.ld, ta ? 1 : 0,
                       (const double*)B.p, B.ld, tb ? 1 : 0, beta, C.p, C.ld);
  }
  void trsm(const Node& T, const MatV& X, int mode) {
    const int64_t c = mode == 3 ? X.rows : X.cols;
    if (c == 0) return;
    if (mode <= 1 && T.m() <= TRSM_LDS_M && c <= 64)
      hipLaunchKernelGGL(k_dtrsm_lds, dim3((unsigned)c), dim3(64), 0, s, (const double*)T.D.buf.get<double>(),
                         (int)T.m(), (int64_t)T.m(), X.p, X.ld, mode);
    else
      hipLaunchKernelGGL(k_dtrsm, dim3(blocks_for(c)), dim3(256), 0, s, (const double*)T.D.buf.get<double>(), T.m(),
                         (int64_t)T.m(), X.p, X.ld, c, mode);
  }

  // ---- products with dense column blocks: Y += alpha op(b) X
  void mulvec(int bi, const MatV& X, const MatV& Y, double alpha, bool trans) {
    Node& b = nd(bi);
    if (b.kind == 1) {
      gemm(trans, false, alpha, b.D.v(), X, 1.0, Y);
    } else if (b.kind == 2) {
      const int64_t k = b.U.cols;
      if (k == 0 || X.cols == 0) return;
      MatO T = alloc(k, X.cols, false);
      if (!trans) {
        gemm(true, false, 1.0, b.V.v(), X, 0.0, T.v());
        gemm(false, false, alpha, b.U.v(), T.v(), 1.0, Y);
      } else {
        gemm(true, false, 1.0, b.U.v(), X, 0.0, T.v());
        gemm(false, false, alpha, b.V.v(), T.v(), 1.0, Y);
      }
    } else {
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          const Node& c = nd(b.ch[i][j]);
          const int64_t ro = c.r0 - b.r0, co = c.c0 - b.c0;
          if (!trans) mulvec(b.ch[i][j], X.rowsv(co, c.n()), Y.rowsv(ro, c.m()), alpha, false);
          else mulvec(b.ch[i][j], X.rowsv(ro, c.m()), Y.rowsv(co, c.n()), alpha, true);
        }
    }
  }

  // ---- flattened products for the substitutions (built once the factors are final)
  void flatten(int bi) {
    std::vector<FlatLeaf> lr, dn;
    const Node& root = nd(bi);
    int64_t tsz = 0;
    std::vector<int> st{bi};
    while (!st.empty()) {
      const int x = st.back();
      st.pop_back();
      const Node& b = nd(x);
      if (b.kind == 0) {
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j) st.push_back(b.ch[i][j]);
        continue;
      }
      FlatLeaf L{};
      L.ro = b.r0 - root.r0;
      L.co = b.c0 - root.c0;
      L.m = b.m();
      L.n = b.n();
      L.kind = b.kind;
      if (b.kind == 1) {
        L.D = b.D.buf.get<double>();
        dn.push_back(L);
      } else if (b.U.cols > 0) {
        L.U = b.U.buf.get<double>();
        L.V = b.V.buf.get<double>();
        L.k = (int32_t)b.U.cols;
        L.toff = tsz;
        tsz += L.k;
        lr.push_back(L);
      }
    }
    hm_hlu::Flat& F = H.flat[bi];
    F.nlr = (int)lr.size();
    F.n = (int)(lr.size() + dn.size());
    F.tsize = tsz;
    lr.insert(lr.end(), dn.begin(), dn.end());
    if (!lr.empty()) upload(F.leaves, lr, s);
  }
  void build_flat(int ai) {  // the L21 and U12 subtrees of every subdivided diagonal block
    const Node& A = nd(ai);
    if (A.kind != 0) return;
    flatten(A.ch[1][0]);
    flatten(A.ch[0][1]);
    build_flat(A.ch[0][0]);
    build_flat(A.ch[1][1]);
  }
  // Y += alpha b X through the flattened leaves of b
  // per-node intermediates of the substitutions (tbuf[bi] holds at least
  // tsize x c doubles), or NULL: allocated per call
  std::vector<DevBuf>* tbuf = nullptr;
  void mulvec_flat(int bi, const MatV& X, const MatV& Y, double alpha) {
    const hm_hlu::Flat& F = H.flat[bi];
    if (F.n == 0 || X.cols == 0) return;
    const int c = (int)X.cols;
    DevBuf own;
    double* t;
    if (tbuf) {
      t = (*tbuf)[bi].get<double>();
    } else {
      own.alloc((size_t)std::max<int64_t>(1, F.tsize * c) * 8);
      t = own.get<double>();
    }
    const FlatLeaf* lv = F.leaves.get<FlatLeaf>();
    if (F.nlr > 0)
      hipLaunchKernelGGL(k_flat_t, dim3((unsigned)F.nlr), dim3(256), 0, s, lv, (const double*)X.p, X.ld, c, t);
    hipLaunchKernelGGL(k_flat_apply, dim3((unsigned)F.n), dim3(256), 0, s, lv, (const double*)X.p, X.ld, c,
                       (const double*)t, alpha, Y.p, Y.ld);
  }
  void solve_lower_flat(int li, const MatV& X) {
    Node& L = nd(li);
    if (L.kind == 1) return trsm(L, X, 0);
    const int64_t m0 = nd(L.ch[0][0]).m();
    const MatV X0 = X.rowsv(0, m0), X1 = X.rowsv(m0, X.rows - m0);
    solve_lower_flat(L.ch[0][0], X0);
    mulvec_flat(L.ch[1][0], X0, X1, -1.0);
    solve_lower_flat(L.ch[1][1], X1);
  }
  void solve_upper_flat(int ui, const MatV& X) {
    Node& U = nd(ui);
    if (U.kind == 1) return trsm(U, X, 1);
    const int64_t m0 = nd(U.ch[0][0]).m();
    const MatV X0 = X.rowsv(0, m0), X1 = X.rowsv(m0, X.rows - m0);
    solve_upper_flat(U.ch[1][1], X1);
    mulvec_flat(U.ch[0][1], X1, X0, -1.0);
    solve_upper_flat(U.ch[0][0], X0);
  }

  // ---- substitutions with dense right-hand sides (in place)
  void solve_lower(int li, const MatV& X) {  // X <- L^-1 X
    Node& L = nd(li);
    if (L.kind == 1) return trsm(L, X, 0);
    const int64_t m0 = nd(L.ch[0][0]).m();
    const MatV X0 = X.rowsv(0, m0), X1 = X.rowsv(m0, X.rows - m0);
    solve_lower(L.ch[0][0], X0);
    mulvec(L.ch[1][0], X0, X1, -1.0, false);
    solve_lower(L.ch[1][1], X1);
  }
  void solve_upper(int ui, const MatV& X) {  // X <- U^-1 X
    Node& U = nd(ui);
    if (U.kind == 1) return trsm(U, X, 1);
    const int64_t m0 = nd(U.ch[0][0]).m();
    const MatV X0 = X.rowsv(0, m0), X1 = X.rowsv(m0, X.rows - m0);
    solve_upper(U.ch[1][1], X1);
    mulvec(U.ch[0][1], X1, X0, -1.0, false);
    solve_upper(U.ch[0][0], X0);
  }
  void solve_upper_t(int ui, const MatV& X) {  // X <- U^-T X
    Node& U = nd(ui);
    if (U.kind == 1) return trsm(U, X, 2);
    const int64_t m0 = nd(U.ch[0][0]).m();
    const MatV X0 = X.rowsv(0, m0), X1 = X.rowsv(m0, X.rows - m0);
    solve_upper_t(U.ch[0][0], X0);
    mulvec(U.ch[0][1], X0, X1, -1.0, true);
    solve_upper_t(U.ch[1][1], X1);
  }

  // ---- truncation of U V^T (m x k, n x k) at tol relative to its own norm
  void truncate(const MatV& U, const MatV& V, MatO& Uo, MatO& Vo) {
    const int64_t m = U.rows, n = V.rows;
    int64_t k = U.cols;
    if (k > RC_KMAX) {
      // the first RC_KMAX columns first, then the rest added to the result
      MatO U1, V1;
      truncate(U.sub(0, m, 0, RC_KMAX), V.sub(0, n, 0, RC_KMAX), U1, V1);
      const int64_t k1 = U1.cols, k2 = k - RC_KMAX;
      MatO Uc = alloc(m, k1 + k2, false), Vc = alloc(n, k1 + k2, false);
      copy(U1.v(), Uc.v().sub(0, m, 0, k1));
      copy(V1.v(), Vc.v().sub(0, n, 0, k1));
      copy(U.sub(0, m, RC_KMAX, k2), Uc.v().sub(0, m, k1, k2));
      copy(V.sub(0, n, RC_KMAX, k2), Vc.v().sub(0, n, k1, k2));
      return truncate(Uc.v(), Vc.v(), Uo, Vo);
    }
    if (k <= 1) {
      Uo = alloc(m, k, false);
      Vo = alloc(n, k, false);
      copy(U, Uo.v());
      copy(V, Vo.v());
      return;
    }
    ++H.truncations;
    MatO scr = alloc(m * k + n * k, 1, false);
    copy(U, MatV{scr.buf.get<double>(), m, k, m});
    copy(V, MatV{scr.buf.get<double>() + m * k, n, k, n});
    DevBuf stage((size_t)(m + n) * k * 8), d_nr(4);
    std::vector<RcDev> rc{RcDev{0, m * k, 0, 0, m * k, (int32_t)m, (int32_t)n, (int32_t)k, 0, tol, k > 64 ? 1 : 0}};
    recompress_blocks(rc, scr.buf.get<double>(), stage.get(), true, d_nr.get<int>(), s);
    int r = 0;
    HM_HIP(hipMemcpyAsync(&r, d_nr.get(), 4, hipMemcpyDeviceToHost, s));
    HM_HIP(hipStreamSynchronize(s));
    Uo = alloc(m, r, false);
    Vo = alloc(n, r, false);
    copy(MatV{stage.get<double>(), m, r, m}, Uo.v());
    copy(MatV{stage.get<double>() + m * k, n, r, n}, Vo.v());
    HM_HIP(hipStreamSynchronize(s));  // stage and scratch are released on return
  }

  // truncates every dirty block in one batched launch
  void flush() {
    if (dirty_list.empty()) return;
    std::vector<int> ids;
    for (int id : dirty_list) {
      dirty[id] = 0;
      if (nd(id).kind == 2 && nd(id).U.cols >= 2) ids.push_back(id);
    }
    dirty_list.clear();
    if (ids.empty()) return;
    int64_t so = 0;
    std::vector<int64_t> off(ids.size());
    for (size_t q = 0; q < ids.size(); ++q) {
      const Node& b = nd(ids[q]);
      off[q] = so;
      so += (int64_t)(b.m() + b.n()) * b.U.cols;
    }
    DevBuf scr((size_t)so * 8), stage((size_t)so * 8), d_nr(ids.size() * 4);
    std::vector<RcDev> rc;
    for (size_t q = 0; q < ids.size(); ++q) {
      const Node& b = nd(ids[q]);
      const int64_t m = b.m(), n = b.n(), k = b.U.cols;
      HM_HIP(hipMemcpyAsync(scr.get<double>() + off[q], b.U.buf.get(), (size_t)m * k * 8, hipMemcpyDeviceToDevice, s));
      HM_HIP(hipMemcpyAsync(scr.get<double>() + off[q] + m * k, b.V.buf.get(), (size_t)n * k * 8,
                            hipMemcpyDeviceToDevice, s));
      rc.push_back(RcDev{off[q], off[q] + m * k, 0, off[q], off[q] + m * k, (int32_t)m, (int32_t)n, (int32_t)k,
                         (int32_t)q, tol, k > 64 ? 1 : 0});
    }
    H.truncations += (int64_t)ids.size();
    recompress_blocks(rc, scr.get<double>(), stage.get(), true, d_nr.get<int>(), s);
    std::vector<int> nr(ids.size());
    HM_HIP(hipMemcpyAsync(nr.data(), d_nr.get(), nr.size() * 4, hipMemcpyDeviceToHost, s));
    HM_HIP(hipStreamSynchronize(s));
    for (size_t q = 0; q < ids.size(); ++q) {
      Node& b = nd(ids[q]);
      const int64_t m = b.m(), n = b.n(), k = b.U.cols, r = nr[q];
      b.U = alloc(m, r, false);
      b.V = alloc(n, r, false);
      copy(MatV{stage.get<double>() + off[q], m, r, m}, b.U.v());
      copy(MatV{stage.get<double>() + off[q] + m * k, n, r, n}, b.V.v());
    }
    HM_HIP(hipStreamSynchronize(s));  // stage and scratch are released on return
  }
  void mark_dirty(int id) {
    if (nd(id).U.cols > RC_KMAX) {
      // too wide for one recompression: truncated now
      Node& b = nd(id);
      MatO Uo, Vo;
      truncate(b.U.v(), b.V.v(), Uo, Vo);
      b.U = std::move(Uo);
      b.V = std::move(Vo);
      return;
    }
    if (!dirty[id]) {
      dirty[id] = 1;
      dirty_list.push_back(id);
    }
  }

  // ---- products and additions of blocks
  struct Prod {
    bool dense = false;
    MatO D, U, V;
  };
  struct ProdV {
    bool dense = false;
    MatV D, U, V;
  };
  static ProdV view(const Prod& p) { return ProdV{p.dense, p.D.v(), p.U.v(), p.V.v()}; }

  void to_dense(int bi, const MatV& out) {
    Node& b = nd(bi);
    if (b.kind == 1) return copy(b.D.v(), out);
    if (b.kind == 2) return gemm(false, true, 1.0, b.U.v(), b.V.v(), 0.0, out);
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        const Node& c = nd(b.ch[i][j]);
        to_dense(b.ch[i][j], out.sub(c.r0 - b.r0, c.m(), c.c0 - b.c0, c.n()));
      }
  }

  // a dense m x n piece as low-rank factors with an identity on its smaller side
  void lr_of_dense(const MatV& D, Prod& p) {
    const int64_t m = D.rows, n = D.cols;
    p.dense = false;
    if (n <= m) {
      p.U = alloc(m, n, false);
      copy(D, p.U.v());
      p.V = identity(n);
    } else {
      p.U = identity(m);
      p.V = alloc(n, m, false);
      copy(D, p.V.v(), 1.0, true);
    }
  }

  Prod product(double alpha, int ai, int bi, bool want_dense) {
    Node& A = nd(ai);
    Node& B = nd(bi);
    Prod p;
    if (B.kind == 2) {
      p.U = alloc(A.m(), B.U.cols);
      mulvec(ai, B.U.v(), p.U.v(), alpha, false);
      p.V = alloc(B.n(), B.V.cols, false);
      copy(B.V.v(), p.V.v());
      return p;
    }
    if (A.kind == 2) {
      p.U = alloc(A.m(), A.U.cols, false);
      copy(A.U.v(), p.U.v(), alpha);
      p.V = alloc(B.n(), A.V.cols);
      mulvec(bi, A.V.v(), p.V.v(), 1.0, true);
      return p;
    }
    if (A.kind == 1 && B.kind == 1) {
      p.dense = true;
      p.D = alloc(A.m(), B.n(), false);
      gemm(false, false, alpha, A.D.v(), B.D.v(), 0.0, p.D.v());
      return p;
    }
    if (A.kind == 1) {  // A dense (its rows a leaf cluster), B subdivided: I (alpha B^T A^T)^T
      MatO At = alloc(A.n(), A.m(), false);
      copy(A.D.v(), At.v(), 1.0, true);
      p.U = identity(A.m());
      p.V = alloc(B.n(), A.m());
      mulvec(bi, At.v(), p.V.v(), alpha, true);
      return p;
    }
    if (B.kind == 1) {  // B dense (its columns a leaf cluster), A subdivided: (alpha A B) I
      p.U = alloc(A.m(), B.n());
      mulvec(ai, B.D.v(), p.U.v(), alpha, false);
      p.V = identity(B.n());
      return p;
    }
    // both subdivided
    if (want_dense) {
      MatO Bd = alloc(B.m(), B.n(), false);
      to_dense(bi, Bd.v());
      p.dense = true;
      p.D = alloc(A.m(), B.n());
      mulvec(ai, Bd.v(), p.D.v(), alpha, false);
      return p;
    }
    // the four pieces of the result, each a sum of two products, padded into
    // full-height / full-width factors and truncated together
    std::vector<Prod> parts;
    std::vector<std::pair<int, int>> where;
    int64_t ktot = 0;
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        for (int k = 0; k < 2; ++k) {
          Prod q = product(alpha, A.ch[i][k], B.ch[k][j], false);
          if (q.dense) {
            Prod r;
            lr_of_dense(q.D.v(), r);
            q = std::move(r);
          }
          ktot += q.U.cols;
          parts.push_back(std::move(q));
          where.emplace_back(i, j);
        }
    const int64_t m = A.m(), n = B.n();
    MatO Ub = alloc(m, ktot), Vb = alloc(n, ktot);
    int64_t col = 0;
    for (size_t q = 0; q < parts.size(); ++q) {
      const int i = where[q].first, j = where[q].second;
      const Node& ai0 = nd(A.ch[i][0]);
      const Node& bj0 = nd(B.ch[0][j]);
      const int64_t ro = ai0.r0 - A.r0, co = bj0.c0 - B.c0;
      const int64_t kq = parts[q].U.cols;
      copy(parts[q].U.v(), Ub.v().sub(ro, ai0.m(), col, kq));
      copy(parts[q].V.v(), Vb.v().sub(co, bj0.n(), col, kq));
      col += kq;
    }
    if (ktot > RC_KMAX) {
      truncate(Ub.v(), Vb.v(), p.U, p.V);
    } else {
      // the block it is added to is truncated with the others later
      p.U = std::move(Ub);
      p.V = std::move(Vb);
    }
    return p;
  }

  void add(int ci, const ProdV& P) {
    Node& C = nd(ci);
    if (C.kind == 1) {
      if (P.dense) axpy(1.0, P.D, C.D.v());
      else gemm(false, true, 1.0, P.U, P.V, 1.0, C.D.v());
      return;
    }
    if (C.kind == 2) {
      MatV Pu = P.U, Pv = P.V;
      Prod tmp;
      if (P.dense) {
        lr_of_dense(P.D, tmp);
        Pu = tmp.U.v();
        Pv = tmp.V.v();
      }
      const int64_t m = C.m(), n = C.n(), k1 = C.U.cols, k2 = Pu.cols;
      MatO Uc = alloc(m, k1 + k2, false), Vc = alloc(n, k1 + k2, false);
      copy(C.U.v(), Uc.v().sub(0, m, 0, k1));
      copy(C.V.v(), Vc.v().sub(0, n, 0, k1));
      copy(Pu, Uc.v().sub(0, m, k1, k2));
      copy(Pv, Vc.v().sub(0, n, k1, k2));
      C.U = std::move(Uc);
      C.V = std::move(Vc);
      mark_dirty(ci);
      return;
    }
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        const Node& c = nd(C.ch[i][j]);
        const int64_t ro = c.r0 - C.r0, co = c.c0 - C.c0;
        ProdV q;
        q.dense = P.dense;
        if (P.dense) q.D = P.D.sub(ro, c.m(), co, c.n());
        else {
          q.U = P.U.rowsv(ro, c.m());
          q.V = P.V.rowsv(co, c.n());
        }
        add(C.ch[i][j], q);
      }
  }

  void gemm_block(int ci, double alpha, int ai, int bi) {  // C += alpha A B
    Node& C = nd(ci);
    Node& A = nd(ai);
    Node& B = nd(bi);
    if (C.kind == 0 && A.kind == 0 && B.kind == 0) {
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
          for (int k = 0; k < 2; ++k) gemm_block(nd(ci).ch[i][j], alpha, nd(ai).ch[i][k], nd(bi).ch[k][j]);
      return;
    }
    Prod p = product(alpha, ai, bi, C.kind == 1);
    add(ci, view(p));
  }

  // ---- block substitutions (steps 2 and 3)
  void solve_lower_block(int li, int bi) {  // B <- L^-1 B
    flush();
    Node& B = nd(bi);
    if (B.kind == 2) return solve_lower(li, B.U.v());
    if (B.kind == 1) return solve_lower(li, B.D.v());
    const Node& L = nd(li);
    for (int j = 0; j < 2; ++j) {
      solve_lower_block(L.ch[0][0], nd(bi).ch[0][j]);
      gemm_block(nd(bi).ch[1][j], -1.0, L.ch[1][0], nd(bi).ch[0][j]);
      solve_lower_block(L.ch[1][1], nd(bi).ch[1][j]);
    }
  }
  void solve_upper_block(int ui, int bi) {  // B <- B U^-1
    flush();
    Node& B = nd(bi);
    if (B.kind == 2) return solve_upper_t(ui, B.V.v());
    if (B.kind == 1) {
      const Node& U = nd(ui);
      if (U.kind == 1) return trsm(U, B.D.v(), 3);
      MatO Dt = alloc(B.n(), B.m(), false);
      copy(B.D.v(), Dt.v(), 1.0, true);
      solve_upper_t(ui, Dt.v());
      copy(Dt.v(), B.D.v(), 1.0, true);
      return;
    }
    const Node& U = nd(ui);
    for (int i = 0; i < 2; ++i) {
      solve_upper_block(U.ch[0][0], nd(bi).ch[i][0]);
      gemm_block(nd(bi).ch[i][1], -1.0, nd(bi).ch[i][0], U.ch[0][1]);
      solve_upper_block(U.ch[1][1], nd(bi).ch[i][1]);
    }
  }

  void factorize(int ai) {
    flush();
    Node& A = nd(ai);
    if (A.kind == 1) {
      hipLaunchKernelGGL(k_dlu, dim3(1), dim3(256), 0, s, A.D.buf.get<double>(), A.m(), (int64_t)A.m());
      return;
    }
    const int a00 = A.ch[0][0], a01 = A.ch[0][1], a10 = A.ch[1][0], a11 = A.ch[1][1];
    factorize(a00);                    // 1
    solve_lower_block(a00, a01);       // 2
    solve_upper_block(a00, a10);       // 3
    gemm_block(a11, -1.0, a10, a01);   // 4: Schur complement
    factorize(a11);                    // 4: its factorisation
  }
};

}  // namespace

hm_hlu* hlu_factor(hm_ctx& ctx, const hm_tree& t, const double* eps, const hm_assembly_params& p) {
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = ctx.stream;
  auto H = std::make_unique<hm_hlu>();
  H->device = ctx.device;
  H->n = t.n;
  H->tol = p.aca_tol;
  H->perm = t.perm;
  upload(H->d_perm, H->perm, s);
  DevBuf om(t.n * 8);
  hipLaunchKernelGGL(k_hlu_om, dim3(blocks_for(t.n)), dim3(256), 0, s, H->d_perm.get<int32_t>(), eps,
                     om.get<double>(), t.n);
  HM_HIP(hipGetLastError());
  // block tree of Algorithm 2 with its inner nodes
  std::vector<BlockRef> leaves;
  std::vector<uint8_t> dense;
  std::vector<int> leaf_node;
  struct Rec {
    hm_hlu& H;
    const hm_tree& t;
    std::vector<BlockRef>& leaves;
    std::vector<uint8_t>& dense;
    std::vector<int>& leaf_node;
    int go(int si, int ti) {
      const ClusterNode& a = t.nodes[si];
      const ClusterNode& b = t.nodes[ti];
      const int me = (int)H.nodes.size();
      H.nodes.emplace_back();
      H.nodes[me].r0 = a.begin;
      H.nodes[me].r1 = a.end;
      H.nodes[me].c0 = b.begin;
      H.nodes[me].c1 = b.end;
      const bool adm = tree_admissible(a, b, t.params.eta);
      if (adm || a.child[0] < 0 || b.child[0] < 0) {
        H.nodes[me].kind = adm ? 2 : 1;
        leaves.push_back(BlockRef{a.begin, a.end, b.begin, b.end});
        dense.push_back(adm ? 0 : 1);
        leaf_node.push_back(me);
        return me;
      }
      H.nodes[me].kind = 0;
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          const int c = go(a.child[i], b.child[j]);
          H.nodes[me].ch[i][j] = c;
        }
      return me;
    }
  } rec{*H, t, leaves, dense, leaf_node};
  H->root = rec.go(0, 0);
  std::vector<BlockFactor> fac;
  reflection_blocks(ctx, t, om.get<double>(), leaves, dense, p, fac);
  for (size_t q = 0; q < leaves.size(); ++q) {
    Node& nd = H->nodes[leaf_node[q]];
    const int64_t m = nd.m(), n = nd.n();
    if (fac[q].lowrank && !dense[q]) {
      nd.kind = 2;
      nd.U.buf = std::move(fac[q].U);
      nd.U.rows = m;
      nd.U.cols = fac[q].k;
      nd.V.buf = std::move(fac[q].V);
      nd.V.rows = n;
      nd.V.cols = fac[q].k;
    } else {
      nd.kind = 1;
      nd.D.buf = std::move(fac[q].D);
      nd.D.rows = m;
      nd.D.cols = n;
    }
  }
  Hlu f{*H, s, p.aca_tol};
  f.dirty.assign(H->nodes.size(), 0);
  f.factorize(H->root);
  f.flush();
  H->flat.resize(H->nodes.size());
  f.build_flat(H->root);
  HM_HIP(hipGetLastError());
  HM_HIP(hipStreamSynchronize(s));
  H->factor_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return H.release();
}

void hlu_solve(hm_ctx& ctx, const hm_hlu& Hc, int nrhs, const double* B, int64_t ldb, double* X, int64_t ldx) {
  hipStream_t s = ctx.stream;
  // the factors are not changed; the graph cache and its buffers are
  hm_hlu& H = const_cast<hm_hlu&>(Hc);
  std::lock_guard<std::mutex> lk(H.solve_mu);
  const int64_t n = H.n;
  hm_hlu::SolveGraph* g = nullptr;
  for (size_t q = 0; q < H.graphs.size() && !g; ++q)
    if (H.graphs[q]->nrhs == nrhs) {
      // to the front: the most recently used count
      std::rotate(H.graphs.begin(), H.graphs.begin() + q, H.graphs.begin() + q + 1);
      g = H.graphs.front().get();
    }
  bool fresh = false;
  if (!g) {
    // built whole before it joins the list (an allocation that fails
    // leaves the list as it was); the least recently used count gives way
    // (every solve that used its buffers ended with a synchronisation
    // under solve_mu)
    auto ng = std::make_unique<hm_hlu::SolveGraph>();
    ng->nrhs = nrhs;
    ng->W.alloc((size_t)n * nrhs * 8);
    ng->t.resize(H.flat.size());
    for (size_t b = 0; b < H.flat.size(); ++b)
      if (H.flat[b].n > 0) ng->t[b].alloc((size_t)std::max<int64_t>(1, H.flat[b].tsize * nrhs) * 8);
    if (H.graphs.size() >= hm_hlu::MAX_GRAPHS) H.graphs.pop_back();
    H.graphs.insert(H.graphs.begin(), std::move(ng));
    g = H.graphs.front().get();
    fresh = true;
  }
  MatV Wv{g->W.get<double>(), n, nrhs, n};
  auto substitutions = [&](hipStream_t st) {
    Hlu f{H, st, H.tol};
    f.tbuf = &g->t;
    f.solve_lower_flat(H.root, Wv);
    f.solve_upper_flat(H.root, Wv);
  };
  if (fresh) {
    // capture once on the private stream (ordered after everything that
    // built the buffers); a failed capture leaves direct launches
    HM_HIP(hipStreamSynchronize(s));
    if (!H.cap && hipStreamCreateWithFlags(&H.cap, hipStreamNonBlocking) != hipSuccess) H.cap = nullptr;
    if (H.cap && hipStreamBeginCapture(H.cap, hipStreamCaptureModeThreadLocal) == hipSuccess) {
      bool ok = true;
      try {
        substitutions(H.cap);
      } catch (const Error&) {
        ok = false;
      }
      hipGraph_t gr = nullptr;
      if (hipStreamEndCapture(H.cap, &gr) != hipSuccess || !gr) ok = false;
      if (ok && hipGraphInstantiate(&g->exec, gr, nullptr, nullptr, 0) != hipSuccess) g->exec = nullptr;
      if (gr) (void)hipGraphDestroy(gr);
      (void)hipGetLastError();
    }
  }
  dim3 grid(blocks_for(n), (unsigned)nrhs);
  hipLaunchKernelGGL(k_hlu_gather<double>, grid, dim3(256), 0, s, H.d_perm.get<int32_t>(), B, ldb, g->W.get<double>(), n);
  if (g->exec)
    HM_HIP(hipGraphLaunch(g->exec, s));
  else
    substitutions(s);
  hipLaunchKernelGGL(k_hlu_scatter, grid, dim3(256), 0, s, H.d_perm.get<int32_t>(), (const double*)g->W.get<double>(),
                     X, ldx, n);
  HM_HIP(hipGetLastError());
  HM_HIP(hipStreamSynchronize(s));
}

int64_t hlu_rows(const hm_hlu& H) { return H.n; }
int hlu_device(const hm_hlu& H) { return H.device; }
void hlu_destroy(hm_hlu* H) {
  (void)hipSetDevice(H->device);
  (void)hipDeviceSynchronize();
  delete H;
}

void hlu_stats(const hm_hlu& H, int64_t* bytes, int64_t* entries, int32_t* max_rank, double* seconds) {
  int64_t b = 0, e = 0;
  int32_t mr = 0;
  for (const Node& nd : H.nodes) {
    if (nd.kind == 1) e += (int64_t)nd.D.rows * nd.D.cols;
    if (nd.kind == 2) {
      e += (int64_t)(nd.U.rows + nd.V.rows) * nd.U.cols;
      mr = std::max<int32_t>(mr, (int32_t)nd.U.cols);
    }
    b += (int64_t)(nd.D.buf.bytes() + nd.U.buf.bytes() + nd.V.buf.bytes());
  }
  if (bytes) *bytes = b;
  if (entries) *entries = e;
  if (max_rank) *max_rank = mr;
  if (seconds) *seconds = H.factor_seconds;
}

}  // namespace hm
