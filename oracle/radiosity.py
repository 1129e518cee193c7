"""Radiosity solve and facet flux (oracle; test infrastructure only).

* emission, eq. (4): ``q = eps sigma T^4``; the radiation power of a facet is
  ``eta = T^4`` (eq. (8) on nodes, the same quantity per facet here);
* reflection matrix, eq. (11): ``C = I - Lambda F_paper`` with
  ``Lambda_ii = (1 - eps_i) / A_i``.  With the per-area view factors of
  ``viewfactor`` (``F_paper = diag(A) F``) this is ``C = I - diag(1 - eps) F``;
* radiosity: ``J = C^-1 (sigma eps eta)``, the balance
  ``J_i = eps_i sigma eta_i + (1 - eps_i) sum_j F_ij J_j``;
* facet flux, eq. (12):
  ``q_i = (sigma eps_i / A_i) sum_j eps_j sum_k F_paper_ik C^-1_kj (eta_j - eta_i)``;
* open cavities, eq. (35): the view fraction ``1 - c_i`` (clamped row sum
  c_i, eqs. (32)-(33)) exchanges with an ambient at ``T_amb``.

The dense system is solved by LU with partial pivoting (LAPACK getrf/getrs
through scipy), in FP64.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

SIGMA = 5.670374e-8


def reflection_matrix(F, eps):
    """``C = I - diag(1 - eps) F`` (eq. (11) in the per-area convention).
    Built as ``-(1 - eps) F`` plus 1 on the diagonal, the same values as
    ``I - (1 - eps) F`` without an n x n identity."""
    n = F.shape[0]
    C = (eps - 1.0)[:, None] * F
    C[np.diag_indices(n)] += 1.0
    return C


def emission(eps, T, sigma=SIGMA):
    """Right-hand side ``sigma eps T^4`` (eq. (4)); T may be n or n x r."""
    T = np.asarray(T, dtype=np.float64)
    e = eps if T.ndim == 1 else eps[:, None]
    return sigma * e * T**4


def clamped_row_sums(F):
    """``c_i = clamp(s_i, 0, 1)`` with the row sum ``s_i = sum_j F_ij``
    (eqs. (32)-(33); the ``1/A_i`` of eq. (32) is inside the per-area F)."""
    return np.clip(F.sum(axis=1), 0.0, 1.0)


def ambient_flux(c, T, T_amb, sigma=SIGMA):
    """Open-cavity exchange with the ambient, eq. (35): the fraction
    ``1 - c_i`` of facet i's view that leaves the cavity carries
    ``sigma (1 - c_i) (T_i^4 - T_amb^4)`` away from the facet (the printed
    term omits sigma; it is restored for units).  Returned as the flux INTO
    the facet (the sign convention of eq. (12)): ``-sigma (1 - c)(T^4 - T_amb^4)``.
    ``c`` are the clamped row sums; T may be n or n x r."""
    T = np.asarray(T, dtype=np.float64)
    w = (1.0 - c) if T.ndim == 1 else (1.0 - c)[:, None]
    return -sigma * w * (T**4 - T_amb**4)


class DenseRadiosity:
    """Dense LU of the reflection matrix of one cavity, reused for every
    right-hand side (as the paper reuses its factorisation)."""

    def __init__(self, F, eps, sigma=SIGMA, keep_c=True):
        self.F = F
        self.eps = np.asarray(eps, dtype=np.float64)
        self.sigma = sigma
        C = reflection_matrix(F, self.eps)
        # keep_c=False factorises C in place (large cavities: one n x n array
        # fewer); the factors are the same either way
        self.C = C if keep_c else None
        self.lu = sla.lu_factor(C, overwrite_a=not keep_c)
        # w = C^-1 eps and g = F w, used by the O(n) evaluation of eq. (12)
        self.w = sla.lu_solve(self.lu, self.eps)
        self.g = F @ self.w

    def solve(self, b):
        return sla.lu_solve(self.lu, b)

    def radiosity(self, T):
        return self.solve(emission(self.eps, T, self.sigma))

    def flux(self, T, J=None, T_amb=None):
        """Eq. (12) rewritten with the radiosity J:
        ``q_i = sigma eps_i [ (F C^-1 (eps eta))_i - eta_i (F C^-1 eps)_i ]``
        ``    = eps_i [ (F J)_i - sigma eta_i g_i ]``,  ``g = F C^-1 eps``;
        with ``T_amb`` (open cavity) plus the ambient exchange of eq. (35)."""
        T = np.asarray(T, dtype=np.float64)
        if J is None:
            J = self.radiosity(T)
        eta = T**4
        if T.ndim == 1:
            q = self.eps * (self.F @ J - self.sigma * eta * self.g)
        else:
            q = self.eps[:, None] * (self.F @ J - self.sigma * eta * self.g[:, None])
        if T_amb is not None:
            q = q + ambient_flux(clamped_row_sums(self.F), T, T_amb, self.sigma)
        return q


def flux_eq12_literal(F, eps, area, T, sigma=SIGMA):
    """Eq. (12) term by term with the paper's area-weighted view factor
    ``F_paper = diag(A) F`` and ``C = I - Lambda F_paper``.  O(n^3); small n."""
    eps = np.asarray(eps, dtype=np.float64)
    A = np.asarray(area, dtype=np.float64)
    Fp = A[:, None] * F
    Lam = (1.0 - eps) / A
    C = np.eye(F.shape[0]) - Lam[:, None] * Fp
    M = Fp @ np.linalg.inv(C)            # M_ij = sum_k F_paper_ik C^-1_kj
    eta = np.asarray(T, dtype=np.float64) ** 4
    diff = eta[None, :] - eta[:, None]   # (eta_j - eta_i)
    return (sigma * eps / A) * np.sum(eps[None, :] * M * diff, axis=1)


def relative_l2(a, b, axis=0):
    """``|a - b|_2 / |b|_2`` per right-hand side (the error measure of
    eq. (36), applied to J, q or T)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b, axis=axis) / np.linalg.norm(b, axis=axis)
