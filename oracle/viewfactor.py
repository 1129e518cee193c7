"""Centroid-rule view factors (oracle; test infrastructure only).

Eq. (10) defines the facet-to-facet view factor as the double area integral
of cos(phi_i) cos(phi_j) / (pi R^2), with the angles measured between each
facet normal and the segment joining the centroids, and a zero diagonal.

Readings fixed here (the paper integrates with adaptive Gauss quadrature;
this path uses the one-point centroid rule for every pair):

* per-area normalisation: ``F_ij = cos_i cos_j A_j / (pi r^2)``.  Eq. (10) as
  printed integrates over both facets, i.e. it equals ``A_i F_ij`` in this
  convention; the reflection matrix (11) then divides by ``A_i`` again, so
  ``I - diag(1 - eps) F`` below is the paper's ``C``.
* back-facing pairs (a cosine <= 0) contribute 0 (no occlusion test: the paper
  leaves occlusion out, Sec. 4 (i)).
* coincident centroids contribute 0; ``F_ii = 0``.

The operation order of one entry is fixed (no fused multiply-add):
``d = c_j - c_i``; ``r2 = (dx*dx + dy*dy) + dz*dz``;
``ci = (nix*dx + niy*dy) + niz*dz``; ``cj = -((njx*dx + njy*dy) + njz*dz)``;
``F = (max(ci,0) * max(cj,0) * A_j) / ((pi * r2) * r2)``.
"""
from __future__ import annotations

import math

import numpy as np


def view_factor_block(c, nrm, area, rows, cols):
    """Dense block ``F[rows][:, cols]`` by the centroid rule, FP64."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    ci = c[rows]
    cj = c[cols]
    dx = cj[None, :, 0] - ci[:, None, 0]
    dy = cj[None, :, 1] - ci[:, None, 1]
    dz = cj[None, :, 2] - ci[:, None, 2]
    r2 = (dx * dx + dy * dy) + dz * dz
    ni = nrm[rows]
    nj = nrm[cols]
    cos_i = (ni[:, None, 0] * dx + ni[:, None, 1] * dy) + ni[:, None, 2] * dz
    cos_j = -((nj[None, :, 0] * dx + nj[None, :, 1] * dy) + nj[None, :, 2] * dz)
    num = np.maximum(cos_i, 0.0) * np.maximum(cos_j, 0.0) * area[cols][None, :]
    den = (math.pi * r2) * r2
    with np.errstate(divide="ignore", invalid="ignore"):
        f = num / den
    f[~(r2 > 0.0)] = 0.0
    # the diagonal is zero by definition (eq. (10) is only defined for i != j)
    f[rows[:, None] == cols[None, :]] = 0.0
    return f


def view_factor_matrix(c, nrm, area, chunk: int = 1024):
    """Full dense ``n x n`` view-factor matrix (per-area convention)."""
    n = c.shape[0]
    F = np.empty((n, n))
    allc = np.arange(n)
    for r0 in range(0, n, chunk):
        rows = np.arange(r0, min(n, r0 + chunk))
        F[rows] = view_factor_block(c, nrm, area, rows, allc)
    return F


def view_factor_rows(c, nrm, area, rows):
    """Selected full rows of F (used to check single outputs at large n)."""
    return view_factor_block(c, nrm, area, rows, np.arange(c.shape[0]))


def matvec_rows(c, nrm, area, rows, x, chunk: int = 256):
    """``(F x)[rows]`` evaluated row-panel by row-panel without storing F."""
    rows = np.asarray(rows, dtype=np.int64)
    x = np.asarray(x, dtype=np.float64)
    out = np.empty((rows.size,) + x.shape[1:])
    for k in range(0, rows.size, chunk):
        rr = rows[k:k + chunk]
        out[k:k + rr.size] = view_factor_rows(c, nrm, area, rr) @ x
    return out


def row_sums(F):
    """Scaled row sums ``s_i`` of eq. (32).  In the per-area convention the
    ``1/A_i`` of the paper is already inside ``F``."""
    return F.sum(axis=1)


def closed_cavity_scaling(F):
    """Closed-cavity treatment, eqs. (32)-(34): clamp the row sum to [0, 1]
    (eq. (33)) and divide every row whose clamped sum is non-zero by it
    (eq. (34)).  Rows with ``s_i > 1`` are clamped to 1 and so left as they
    are (literal reading of eq. (33))."""
    s = row_sums(F)
    cl = np.clip(s, 0.0, 1.0)
    out = F.copy()
    nz = cl != 0.0
    out[nz] /= cl[nz][:, None]
    return out
