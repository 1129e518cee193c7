"""Closed forms that pin the oracle (test infrastructure only).

* Two infinite gray plates (Sec. 2.2): the net flux between them is
  ``sigma eps1 eps2 (T1^4 - T2^4) / (1 - (1 - eps1)(1 - eps2))``.
* Points on a sphere with inward radial normals: for any two of them the
  centroid-rule kernel gives ``F_ij = A_j / (4 pi R^2)`` exactly, because both
  cosines equal ``r / (2R)``.  The radiosity system then has a closed
  solution (derived below).
* Two aligned parallel rectangles a x b a distance c apart: the textbook
  exact view factor (Howell's catalogue, configuration C-11).
"""
from __future__ import annotations

import math

import numpy as np

SIGMA = 5.670374e-8


def two_plates_flux(eps1, eps2, T1, T2, sigma=SIGMA):
    """Net flux INTO plate 1 (positive when plate 2 is hotter)."""
    return sigma * eps1 * eps2 * (T2**4 - T1**4) / (1.0 - (1.0 - eps1) * (1.0 - eps2))


def two_plates_radiosity(eps1, eps2, T1, T2, sigma=SIGMA):
    """Radiosity of plate 1 for two infinite plates: solving
    ``J1 = eps1 sigma T1^4 + (1 - eps1) J2`` together with the same relation
    for plate 2 gives ``J1 = sigma (eps1 T1^4 + (1 - eps1) eps2 T2^4) /
    (1 - (1 - eps1)(1 - eps2))``."""
    return sigma * (eps1 * T1**4 + (1.0 - eps1) * eps2 * T2**4) / (1.0 - (1.0 - eps1) * (1.0 - eps2))


def sphere_points_F(weights, radius):
    """Exact ``F`` for points on a sphere with inward radial normals:
    ``F_ij = w_j / (4 pi R^2)`` off the diagonal, 0 on it."""
    As = 4.0 * math.pi * radius**2
    n = weights.size
    F = np.tile(weights[None, :] / As, (n, 1))
    np.fill_diagonal(F, 0.0)
    return F


def sphere_points_solve(weights, eps, b, radius):
    """Solve ``(I - diag(1 - eps) F) J = b`` for ``F = (1 w^T - diag(w)) / A_s``.

    Row i reads ``J_i - (1 - eps_i)(S - w_i J_i) / A_s = b_i`` with
    ``S = sum_j w_j J_j``, so ``J_i = (b_i + (1 - eps_i) S / A_s) / d_i`` with
    ``d_i = 1 + (1 - eps_i) w_i / A_s``.  Summing ``w_i J_i`` gives
    ``S = [sum_i w_i b_i / d_i] / [1 - sum_i w_i (1 - eps_i) / (d_i A_s)]``.
    """
    As = 4.0 * math.pi * radius**2
    d = 1.0 + (1.0 - eps) * weights / As
    S = np.sum(weights * b / d) / (1.0 - np.sum(weights * (1.0 - eps) / (d * As)))
    return (b + (1.0 - eps) * S / As) / d


def sphere_points_apply_F(weights, x, radius):
    """``F x`` for the sphere-point F in O(n): ``(sum_j w_j x_j - w_i x_i)/A_s``."""
    As = 4.0 * math.pi * radius**2
    return (np.sum(weights * x) - weights * x) / As


def sphere_points_flux(weights, eps, T, radius, sigma=SIGMA):
    """Facet flux of eq. (12) for the sphere-point cavity in O(n), through
    ``q = eps (F J - sigma eta g)``, ``g = F C^-1 eps``."""
    eta = T**4
    J = sphere_points_solve(weights, eps, sigma * eps * eta, radius)
    w = sphere_points_solve(weights, eps, eps, radius)
    g = sphere_points_apply_F(weights, w, radius)
    return eps * (sphere_points_apply_F(weights, J, radius) - sigma * eta * g), J


def parallel_rectangles(a, b, c):
    """Exact view factor between two aligned parallel a x b rectangles a
    distance c apart."""
    X = a / c
    Y = b / c
    t1 = 0.5 * math.log((1 + X * X) * (1 + Y * Y) / (1 + X * X + Y * Y))
    t2 = X * math.sqrt(1 + Y * Y) * math.atan(X / math.sqrt(1 + Y * Y))
    t3 = Y * math.sqrt(1 + X * X) * math.atan(Y / math.sqrt(1 + X * X))
    t4 = X * math.atan(X) + Y * math.atan(Y)
    return 2.0 / (math.pi * X * Y) * (t1 + t2 + t3 - t4)
