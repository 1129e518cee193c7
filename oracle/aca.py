"""Adaptive cross approximation and the block-wise product (oracle; test
infrastructure only).

Sec. 4.3: an admissible block X is approximated through a set of pivot rows R
and pivot columns C as ``X ~ X(:,C) X(R,C)^-1 X(R,:)`` (eq. (30)), built one
cross at a time in O(mnk) work and post-processed into ``U V^T``; each block
must satisfy ``|X - U V^T| / |X| <= eps_rel`` (eq. (31)).  Sec. 5.2: the
product ``x -> F x`` runs over the block structure and adds no approximation
beyond the stored blocks.

The paper leaves the pivoting to the literature (it used full pivoting).
This oracle follows the deterministic partial-pivoting reading:

1. start at the first local row; the residual row
   ``r = X(i,:) - sum_l u_l(i) v_l`` is evaluated, ``j = argmax |r|`` (first
   index on ties);
2. a zero residual row marks ``i`` as used and moves to the smallest unused
   row (stop when none is left);
3. otherwise ``v = r / r(j)``, ``u = X(:,j) - sum_l v_l(j) u_l``, the squared
   Frobenius norm of the approximation is updated exactly,
   ``S2 += |u|^2 |v|^2 + 2 sum_l (u_l.u)(v_l.v)``, and the cross is appended;
4. stop when ``|u| |v| <= eps_rel sqrt(S2)`` or the rank cap is reached;
   otherwise the next row is ``argmax |u(i)|`` over unused rows (first on ties).

Full pivoting (the paper's choice): ``aca_full`` takes each pivot as the
largest entry of the whole residual and stops on the exact residual norm of
eq. (31); it needs the evaluated block but cannot miss parts of it, which
partial pivoting does on blocks whose back-facing pairs leave whole groups of
rows or columns zero (the 13-sphere spiral of Sec. 6).

Recompression (optional): the crosses of a block stored low-rank are
truncated to the smallest rank that keeps the discarded singular values of
``U V^T`` within the tolerance (``recompress``).

Storage rule: the block is kept dense when the cap
``min(k_max, ceil(mn/(m+n)))`` is reached without meeting the stop test, or
when ``k (m + n) >= m n`` (low-rank storage would not be smaller).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import clustering
from .viewfactor import view_factor_block


@dataclass
class ACAResult:
    U: np.ndarray      # m x k
    V: np.ndarray      # n x k
    rows: list         # pivot rows R (local indices) in order
    cols: list         # pivot columns C (local indices) in order
    converged: bool


def aca_partial(row_fn, col_fn, m: int, n: int, tol: float, k_cap: int) -> ACAResult:
    """Partial-pivoting ACA of an implicit m x n block.

    ``row_fn(i)`` returns row i (length n), ``col_fn(j)`` column j (length m).
    """
    us, vs, R, C = [], [], [], []
    used = np.zeros(m, dtype=bool)
    i = 0
    s2 = 0.0
    converged = False
    while True:
        r = np.array(row_fn(i), dtype=np.float64)
        for u_l, v_l in zip(us, vs):
            r = r - u_l[i] * v_l
        j = int(np.argmax(np.abs(r)))
        if r[j] == 0.0:
            used[i] = True
            free = np.nonzero(~used)[0]
            if free.size == 0:
                converged = True
                break
            i = int(free[0])
            continue
        v = r / r[j]
        u = np.array(col_fn(j), dtype=np.float64)
        for u_l, v_l in zip(us, vs):
            u = u - v_l[j] * u_l
        nu2 = float(u @ u)
        nv2 = float(v @ v)
        cross = 0.0
        for u_l, v_l in zip(us, vs):
            cross += float(u_l @ u) * float(v_l @ v)
        s2 += nu2 * nv2 + 2.0 * cross
        us.append(u)
        vs.append(v)
        R.append(i)
        C.append(j)
        used[i] = True
        if math.sqrt(nu2 * nv2) <= tol * math.sqrt(max(s2, 0.0)):
            converged = True
            break
        if len(us) >= k_cap:
            break
        cand = np.where(used, -1.0, np.abs(u))
        if not (cand.max() >= 0.0):
            converged = True
            break
        i = int(np.argmax(cand))
    k = len(us)
    U = np.stack(us, axis=1) if k else np.zeros((m, 0))
    V = np.stack(vs, axis=1) if k else np.zeros((n, 0))
    return ACAResult(U, V, R, C, converged)


def aca_full(X, tol: float, k_cap: int) -> ACAResult:
    """Fully pivoted ACA of an explicit m x n block (the paper's choice,
    Sec. 1; Sec. 4.3): each cross takes the entry of largest magnitude of the
    whole residual R (first in row-major order on ties) as pivot,
    ``u = R(:, j)``, ``v = R(i, :) / R(i, j)``, and ``R <- R - u v^T``
    (eq. (30) built one cross at a time).  The residual is known exactly, so
    the stop test is eq. (31) itself: ``|R|_F <= tol |X|_F``, or a zero
    residual, or the rank cap."""
    R = np.array(X, dtype=np.float64, copy=True)
    m, n = R.shape
    nx = float(np.linalg.norm(X))
    us, vs, rows, cols = [], [], [], []
    converged = False
    while True:
        flat = int(np.argmax(np.abs(R)))
        i, j = divmod(flat, n)
        piv = R[i, j]
        if piv == 0.0:
            converged = True
            break
        u = R[:, j].copy()
        v = R[i, :] / piv
        R = R - np.outer(u, v)
        us.append(u)
        vs.append(v)
        rows.append(i)
        cols.append(j)
        if float(np.linalg.norm(R)) <= tol * nx:
            converged = True
            break
        if len(us) >= k_cap:
            break
    k = len(us)
    U = np.stack(us, axis=1) if k else np.zeros((m, 0))
    V = np.stack(vs, axis=1) if k else np.zeros((n, 0))
    return ACAResult(U, V, rows, cols, converged)


def rank_cap(m: int, n: int, k_max: int) -> int:
    """Smallest k at which ``k (m + n) >= m n``, limited by ``k_max``."""
    return max(1, min(k_max, -(-(m * n) // (m + n))))


def recompress(U, V, tol: float):
    """Post-processing of a cross approximation into truncated-SVD form
    (Sec. 4.3: the crosses are brought to standard form ``U V^T``; Sec. 5.1:
    ranks are set from the singular value decay at a fixed relative
    accuracy).  Householder QR of both factors (LAPACK), SVD of the small
    core ``R_u R_v^T = W S Z^T``, and the smallest rank ``r >= 1`` whose
    discarded singular values satisfy ``sqrt(sum_{i>r} s_i^2) <= tol *
    sqrt(sum_i s_i^2)`` (the Frobenius form of eq. (31)).  Returns
    ``U' = Q_u W_r S_r`` (m x r) and ``V' = Q_v Z_r`` (n x r, orthonormal
    columns)."""
    Qu, Ru = np.linalg.qr(U)
    Qv, Rv = np.linalg.qr(V)
    W, S, Zt = np.linalg.svd(Ru @ Rv.T)
    tail = np.sqrt(np.cumsum((S**2)[::-1]))[::-1]  # tail[r] = sqrt(sum_{i >= r} s_i^2)
    limit = tol * math.sqrt(float(np.sum(S**2)))
    r = S.size
    for q in range(1, S.size):
        if tail[q] <= limit:
            r = q
            break
    return Qu @ (W[:, :r] * S[:r]), Qv @ Zt[:r].T


@dataclass
class HMatrix:
    n: int
    perm: np.ndarray            # permuted position -> original facet index
    dense: list                 # (r0, r1, c0, c1, block)
    lowrank: list               # (r0, r1, c0, c1, U, V)
    fallback: int               # admissible blocks stored dense

    def matvec(self, x):
        """``y = F_H x`` in the ORIGINAL facet order (x may be n or n x r)."""
        x = np.asarray(x, dtype=np.float64)
        xp = x[self.perm]
        yp = np.zeros_like(xp)
        for r0, r1, c0, c1, B in self.dense:
            yp[r0:r1] += B @ xp[c0:c1]
        for r0, r1, c0, c1, U, V in self.lowrank:
            yp[r0:r1] += U @ (V.T @ xp[c0:c1])
        y = np.empty_like(yp)
        y[self.perm] = yp
        return y

    def to_dense(self):
        """Expand to the dense ``n x n`` matrix in the original order."""
        Fp = np.zeros((self.n, self.n))
        for r0, r1, c0, c1, B in self.dense:
            Fp[r0:r1, c0:c1] = B
        for r0, r1, c0, c1, U, V in self.lowrank:
            Fp[r0:r1, c0:c1] = U @ V.T
        F = np.empty_like(Fp)
        F[np.ix_(self.perm, self.perm)] = Fp
        return F

    def stored_entries(self):
        d = sum(b[4].size for b in self.dense)
        lr = sum(b[4].size + b[5].size for b in self.lowrank)
        return d, lr


def build_hmatrix(c, nrm, area, n_min: int, eta: float, tol: float, k_max: int = 256,
                  recompress_tol: float | None = None, pivot: str = "partial") -> HMatrix:
    """Cluster tree (Alg. 1), block tree (Alg. 2), dense near field, ACA
    (eqs. (30)-(31)) on every admissible block, with the storage rule; with
    ``recompress_tol``, every block stored low-rank is then truncated by
    ``recompress`` (the storage rule is decided on the ACA rank).
    ``pivot``: "partial" (``aca_partial``, entries evaluated by rows and
    columns) or "full" (``aca_full`` on the evaluated block)."""
    root, perm = clustering.build_index_tree(c, n_min)
    dense_blocks, lr_blocks = clustering.build_block_tree(root, eta)
    cp, np_, ap = c[perm], nrm[perm], area[perm]
    dense, lowrank = [], []
    fallback = 0
    for r0, r1, c0, c1 in dense_blocks:
        dense.append((r0, r1, c0, c1, view_factor_block(cp, np_, ap, np.arange(r0, r1), np.arange(c0, c1))))
    for r0, r1, c0, c1 in lr_blocks:
        m, nn = r1 - r0, c1 - c0
        cols = np.arange(c0, c1)
        rows = np.arange(r0, r1)
        if pivot == "full":
            res = aca_full(view_factor_block(cp, np_, ap, rows, cols), tol, rank_cap(m, nn, k_max))
        else:
            res = aca_partial(
                lambda i: view_factor_block(cp, np_, ap, [r0 + i], cols)[0],
                lambda j: view_factor_block(cp, np_, ap, rows, [c0 + j])[:, 0],
                m, nn, tol, rank_cap(m, nn, k_max),
            )
        k = res.U.shape[1]
        if (not res.converged) or k * (m + nn) >= m * nn:
            dense.append((r0, r1, c0, c1, view_factor_block(cp, np_, ap, rows, cols)))
            fallback += 1
        elif recompress_tol is not None:
            U2, V2 = recompress(res.U, res.V, recompress_tol)
            lowrank.append((r0, r1, c0, c1, U2, V2))
        else:
            lowrank.append((r0, r1, c0, c1, res.U, res.V))
    return HMatrix(c.shape[0], perm, dense, lowrank, fallback)
