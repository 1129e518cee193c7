"""Hierarchical block LU of the reflection matrix (oracle; test
infrastructure only).

Sec. 5 keeps the reflection matrix ``C = I - Lambda F`` of eq. (11) in the
block structure of F (Algorithm 2): the diagonal scaling only multiplies the
rows of every block and the identity goes into the dense diagonal blocks.
Sec. 5.1 factorises ``C ~ L U`` recursively over the 2 x 2 subdivision of a
block:

1. ``L11 U11 = C11`` (recursively; a dense LU in the leaf blocks),
2. ``U12 = L11^-1 C12`` by forward substitution,
3. ``L21 = C21 U11^-1`` by backward substitution,
4. ``L22 U22 = C22 - L21 U12`` (recursively),

the substitutions themselves being recursive block products and additions.
Every addition into a low-rank block raises its rank and is followed by a
truncation at the relative accuracy ``eps_rel`` from the singular value
decay (``aca.recompress``).  Sec. 5.2 then applies ``C^-1 x = U^-1 (L^-1 x)``
by a forward and a backward substitution over the same blocks.

Readings fixed here (the paper leaves them to the H-matrix literature):

* no pivoting: the dense leaf LU runs without row exchanges (C has a unit
  diagonal and off-diagonal row sums (1 - eps_i) s_i, close to or below 1);
* the low-rank blocks of C are the ACA crosses of F's admissible blocks with
  their U rows scaled by ``-(1 - eps_i)``, recompressed at ``eps_rel``; an
  admissible block that ACA stores dense stays dense;
* a product whose factors are a dense block of a leaf cluster and a
  hierarchical block is formed as a dense or low-rank block of the size of
  that leaf cluster; a product that lands in a low-rank block is brought to
  low-rank form first (products of two subdivided blocks by their 2 x 2
  pieces, agglomerated), then added and truncated;
* the truncation tolerance of every addition is ``eps_rel`` relative to the
  Frobenius norm of the block being formed.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import aca, clustering
from .viewfactor import view_factor_block


class HBlock:
    """One block (rows [r0, r1), columns [c0, c1) of the permuted order):
    ``kind`` "sub" (2 x 2 children ``ch``), "dense" (``D``) or "lr"
    (``U`` m x k, ``V`` n x k, the block is ``U V^T``)."""

    __slots__ = ("r0", "r1", "c0", "c1", "kind", "ch", "D", "U", "V")

    def __init__(self, r0, r1, c0, c1, kind):
        self.r0, self.r1, self.c0, self.c1, self.kind = r0, r1, c0, c1, kind
        self.ch = None
        self.D = self.U = self.V = None

    @property
    def m(self):
        return self.r1 - self.r0

    @property
    def n(self):
        return self.c1 - self.c0


def build_reflection(c, nrm, area, eps, n_min, eta, tol, k_max=256, pivot="partial"):
    """C = I - diag(1 - eps) F in the block structure of Algorithm 2 (in the
    cluster-permuted order).  Returns (root block, perm)."""
    root, perm = clustering.build_index_tree(c, n_min)
    cp, np_, ap = c[perm], nrm[perm], area[perm]
    om = 1.0 - np.asarray(eps, dtype=np.float64)[perm]

    def rec(s, t):
        rows = np.arange(s.begin, s.end)
        cols = np.arange(t.begin, t.end)
        if clustering.admissible(s, t, eta):
            m, n = rows.size, cols.size
            cap = aca.rank_cap(m, n, k_max)
            if pivot == "full":
                res = aca.aca_full(view_factor_block(cp, np_, ap, rows, cols), tol, cap)
            else:
                res = aca.aca_partial(lambda i: view_factor_block(cp, np_, ap, [s.begin + i], cols)[0],
                                      lambda j: view_factor_block(cp, np_, ap, rows, [t.begin + j])[:, 0],
                                      m, n, tol, cap)
            k = res.U.shape[1]
            if res.converged and k * (m + n) < m * n:
                b = HBlock(s.begin, s.end, t.begin, t.end, "lr")
                if k == 0:
                    b.U, b.V = np.zeros((m, 0)), np.zeros((n, 0))
                else:
                    b.U, b.V = aca.recompress(-om[rows][:, None] * res.U, res.V, tol)
                return b
        if clustering.admissible(s, t, eta) or s.is_leaf or t.is_leaf:
            b = HBlock(s.begin, s.end, t.begin, t.end, "dense")
            b.D = -om[rows][:, None] * view_factor_block(cp, np_, ap, rows, cols)
            if s is t:
                b.D = b.D + np.eye(rows.size)
            return b
        b = HBlock(s.begin, s.end, t.begin, t.end, "sub")
        b.ch = [[rec(s.children[i], t.children[j]) for j in range(2)] for i in range(2)]
        return b

    return rec(root, root), perm


def to_dense(b):
    if b.kind == "dense":
        return b.D.copy()
    if b.kind == "lr":
        return b.U @ b.V.T
    return np.block([[to_dense(b.ch[i][j]) for j in range(2)] for i in range(2)])


def _split_rows(b, X):
    m0 = b.ch[0][0].m
    return X[:m0], X[m0:]


def _split_cols(b, X):
    n0 = b.ch[0][0].n
    return X[:n0], X[n0:]


def mulvec(b, X):
    """b @ X for a dense X with b.n rows."""
    if b.kind == "dense":
        return b.D @ X
    if b.kind == "lr":
        return b.U @ (b.V.T @ X)
    X0, X1 = _split_cols(b, X)
    top = mulvec(b.ch[0][0], X0) + mulvec(b.ch[0][1], X1)
    bot = mulvec(b.ch[1][0], X0) + mulvec(b.ch[1][1], X1)
    return np.vstack([top, bot])


def mulvec_t(b, X):
    """b^T @ X for a dense X with b.m rows."""
    if b.kind == "dense":
        return b.D.T @ X
    if b.kind == "lr":
        return b.V @ (b.U.T @ X)
    X0, X1 = _split_rows(b, X)
    left = mulvec_t(b.ch[0][0], X0) + mulvec_t(b.ch[1][0], X1)
    right = mulvec_t(b.ch[0][1], X0) + mulvec_t(b.ch[1][1], X1)
    return np.vstack([left, right])


# ------------------------------------------------------------- substitutions with dense right-hand sides
def solve_lower(L, X):
    """L^-1 X, L the unit lower triangle of a factorised diagonal block."""
    if L.kind == "dense":
        return sla.solve_triangular(L.D, X, lower=True, unit_diagonal=True)
    X0, X1 = _split_rows(L, X)
    Y0 = solve_lower(L.ch[0][0], X0)
    Y1 = solve_lower(L.ch[1][1], X1 - mulvec(L.ch[1][0], Y0))
    return np.vstack([Y0, Y1])


def solve_upper(U, X):
    """U^-1 X, U the upper triangle (with its diagonal) of a factorised block."""
    if U.kind == "dense":
        return sla.solve_triangular(U.D, X, lower=False)
    X0, X1 = _split_rows(U, X)
    Y1 = solve_upper(U.ch[1][1], X1)
    Y0 = solve_upper(U.ch[0][0], X0 - mulvec(U.ch[0][1], Y1))
    return np.vstack([Y0, Y1])


def solve_upper_t(U, X):
    """U^-T X (forward substitution with the transposed upper triangle)."""
    if U.kind == "dense":
        return sla.solve_triangular(U.D, X, lower=False, trans="T")
    X0, X1 = _split_rows(U, X)
    Y0 = solve_upper_t(U.ch[0][0], X0)
    Y1 = solve_upper_t(U.ch[1][1], X1 - mulvec_t(U.ch[0][1], Y0))
    return np.vstack([Y0, Y1])


# ------------------------------------------------------------- block arithmetic with truncation
def _lr_from_dense(D, tol):
    """Truncated SVD of a dense piece (the same rule as recompress)."""
    if D.size == 0 or not np.any(D):
        return np.zeros((D.shape[0], 0)), np.zeros((D.shape[1], 0))
    W, S, Zt = np.linalg.svd(D, full_matrices=False)
    return aca.recompress(W * S, Zt.T, tol)


def _truncate(U, V, tol):
    if U.shape[1] == 0 or not (np.any(U) and np.any(V)):
        return np.zeros((U.shape[0], 0)), np.zeros((V.shape[0], 0))
    return aca.recompress(U, V, tol)


def product(alpha, A, B, tol, want):
    """alpha A B as ("lr", U, V) or ("dense", D) (``want`` = "lr" or "dense"
    for the kind of block it will be added to when both factors are
    subdivided)."""
    if B.kind == "lr":
        return ("lr", alpha * mulvec(A, B.U), B.V)
    if A.kind == "lr":
        return ("lr", alpha * A.U, mulvec_t(B, A.V))
    if A.kind == "dense" and B.kind == "dense":
        return ("dense", alpha * (A.D @ B.D))
    if A.kind == "dense":
        return ("dense", alpha * mulvec_t(B, A.D.T).T)
    if B.kind == "dense":
        return ("dense", alpha * mulvec(A, B.D))
    # both subdivided
    if want == "dense":
        return ("dense", alpha * mulvec(A, to_dense(B)))
    m0, n0 = A.ch[0][0].m, B.ch[0][0].n
    m, n = A.m, B.n
    Us, Vs = [], []
    for i in range(2):
        for j in range(2):
            Ui = np.zeros((m, 0))
            Vj = np.zeros((n, 0))
            for k in range(2):
                p = product(alpha, A.ch[i][k], B.ch[k][j], tol, "lr")
                pu, pv = (p[1], p[2]) if p[0] == "lr" else _lr_from_dense(p[1], tol)
                fu = np.zeros((m, pu.shape[1]))
                fv = np.zeros((n, pv.shape[1]))
                fu[(0 if i == 0 else m0):(m0 if i == 0 else m)] = pu
                fv[(0 if j == 0 else n0):(n0 if j == 0 else n)] = pv
                Ui = np.hstack([Ui, fu])
                Vj = np.hstack([Vj, fv])
            Us.append(Ui)
            Vs.append(Vj)
    return ("lr",) + _truncate(np.hstack(Us), np.hstack(Vs), tol)


def add(C, P, tol):
    """C += P (P from ``product``), truncating low-rank results."""
    if C.kind == "dense":
        C.D = C.D + (P[1] if P[0] == "dense" else P[1] @ P[2].T)
        return
    if C.kind == "lr":
        pu, pv = (P[1], P[2]) if P[0] == "lr" else _lr_from_dense(P[1], tol)
        C.U, C.V = _truncate(np.hstack([C.U, pu]), np.hstack([C.V, pv]), tol)
        return
    m0, n0 = C.ch[0][0].m, C.ch[0][0].n
    for i in range(2):
        rs = slice(0, m0) if i == 0 else slice(m0, C.m)
        for j in range(2):
            cs = slice(0, n0) if j == 0 else slice(n0, C.n)
            if P[0] == "dense":
                add(C.ch[i][j], ("dense", P[1][rs, cs]), tol)
            else:
                add(C.ch[i][j], ("lr", P[1][rs], P[2][cs]), tol)


def gemm(C, alpha, A, B, tol):
    """C += alpha A B over the block structure."""
    if C.kind == "sub" and A.kind == "sub" and B.kind == "sub":
        for i in range(2):
            for j in range(2):
                for k in range(2):
                    gemm(C.ch[i][j], alpha, A.ch[i][k], B.ch[k][j], tol)
        return
    add(C, product(alpha, A, B, tol, "dense" if C.kind == "dense" else "lr"), tol)


def solve_lower_block(L, B, tol):
    """B <- L^-1 B for a block B whose rows are L's cluster (step 2)."""
    if B.kind == "lr":
        B.U = solve_lower(L, B.U)
    elif B.kind == "dense":
        B.D = solve_lower(L, B.D)
    else:
        for j in range(2):
            solve_lower_block(L.ch[0][0], B.ch[0][j], tol)
            gemm(B.ch[1][j], -1.0, L.ch[1][0], B.ch[0][j], tol)
            solve_lower_block(L.ch[1][1], B.ch[1][j], tol)


def solve_upper_block(U, B, tol):
    """B <- B U^-1 for a block B whose columns are U's cluster (step 3)."""
    if B.kind == "lr":
        B.V = solve_upper_t(U, B.V)
    elif B.kind == "dense":
        B.D = solve_upper_t(U, B.D.T).T
    else:
        for i in range(2):
            solve_upper_block(U.ch[0][0], B.ch[i][0], tol)
            gemm(B.ch[i][1], -1.0, B.ch[i][0], U.ch[0][1], tol)
            solve_upper_block(U.ch[1][1], B.ch[i][1], tol)


def _dense_lu_nopivot(D):
    A = D.copy()
    m = A.shape[0]
    for k in range(m - 1):
        A[k + 1:, k] /= A[k, k]
        A[k + 1:, k + 1:] -= np.outer(A[k + 1:, k], A[k, k + 1:])
    return A


def factorize(A, tol):
    """The four steps of Sec. 5.1, in place: afterwards every diagonal block
    holds L (unit lower, below the diagonal) and U (upper), the blocks below
    the diagonal hold L and those above hold U."""
    if A.kind == "dense":
        A.D = _dense_lu_nopivot(A.D)
        return
    factorize(A.ch[0][0], tol)                                  # 1
    solve_lower_block(A.ch[0][0], A.ch[0][1], tol)              # 2
    solve_upper_block(A.ch[0][0], A.ch[1][0], tol)              # 3
    gemm(A.ch[1][1], -1.0, A.ch[1][0], A.ch[0][1], tol)         # 4 (Schur complement)
    factorize(A.ch[1][1], tol)                                  # 4 (its factorisation)


def solve(LU, b):
    """C^-1 b ~ U^-1 (L^-1 b) (Sec. 5.2), b in the permuted order (n or n x r)."""
    one = np.ndim(b) == 1
    B = np.asarray(b, dtype=np.float64).reshape(LU.m, -1)
    X = solve_upper(LU, solve_lower(LU, B))
    return X[:, 0] if one else X


def lower_upper_dense(LU):
    """(L, U) of a factorised block tree, expanded to dense matrices."""
    D = to_dense(LU)
    return np.tril(D, -1) + np.eye(D.shape[0]), np.triu(D)


def stored_entries(b):
    if b.kind == "dense":
        return b.D.size
    if b.kind == "lr":
        return b.U.size + b.V.size
    return sum(stored_entries(b.ch[i][j]) for i in range(2) for j in range(2))


def max_rank(b):
    if b.kind == "lr":
        return b.U.shape[1]
    if b.kind == "dense":
        return 0
    return max(max_rank(b.ch[i][j]) for i in range(2) for j in range(2))
