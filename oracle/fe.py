"""Finite-element coupling of conduction and cavity radiation (oracle; test
infrastructure only).

Sec. 3.1-3.4 couple a Galerkin finite-element heat equation to the cavity:
nodal temperatures T_M, nodal radiation power eta_M = T_M^4, facet power by
the projection P_iM = (1/A_i) int_{Gamma_i} phi_M (eqs. for P and eta_i),
the facet-to-facet exchange R and its row-sum-corrected form R_bar (eqs.
(Rdef), (Rbardef)), the nodal operator S = P^T R_bar P (eq. (S_def_matrix)),
the radiation load Q = S eta, and implicit Euler with the residual of eq.
(SVF_Galerkin_time), solved by Newton's method.

This oracle uses linear (P1) triangles on the cavity surface itself: a
conducting shell of thickness h whose elements are the radiating facets
(the paper leaves the element type open; the cavity operators do not depend
on it).  Then P_iM = 1/3 for the three vertices of facet i, the consistent
mass matrix is rho c h A/12 [[2,1,1],[1,2,1],[1,1,2]] per element, and the
stiffness is k h (e_a . e_b) / (4 A) per element (e_a the edge opposite
vertex a).  A facet source f_i (W/m^2) gives the load f_N = sum_i f_i A_i / 3.

Conventions: F is this build's view factor (rows sum to 1 in a closed
cavity), so the paper's area-weighted F_ij is A_i F_ij here, and
    R = sigma diag(eps A) F C^-1 diag(eps),   C = I - diag(1 - eps) F,
which makes R_bar eta = A q (q the facet flux of eq. (12) for facet power
eta).  The residual is
    Res(T) = M (T - T^n) / dt + K T - S T^4 - f
and its Jacobian dRes/dT = M/dt + K - 4 S diag(T^3): the paper's J^cav =
dQ/dT enters with the sign the residual gives it.  The step's result is the
root of Res, found by Newton's method with that dense Jacobian to rounding.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .radiosity import SIGMA, reflection_matrix


def surface_p1(v, tri, k_h, rho_c_h):
    """Consistent mass M, stiffness K (n_nodes x n_nodes, dense) and the
    projection P (n_facets x n_nodes) of P1 triangles; facet i is triangle
    tri[i] (vertices v)."""
    v = np.asarray(v, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.int64)
    nn, nf = v.shape[0], tri.shape[0]
    M = np.zeros((nn, nn))
    K = np.zeros((nn, nn))
    P = np.zeros((nf, nn))
    for i, t in enumerate(tri):
        p = v[t]
        e = [p[2] - p[1], p[0] - p[2], p[1] - p[0]]  # edge opposite vertex a
        area = 0.5 * np.linalg.norm(np.cross(e[2], -e[1]))
        for a in range(3):
            P[i, t[a]] += 1.0 / 3.0
            for b in range(3):
                M[t[a], t[b]] += rho_c_h * area / 12.0 * (2.0 if a == b else 1.0)
                K[t[a], t[b]] += k_h * np.dot(e[a], e[b]) / (4.0 * area)
    return M, K, P


def nodal_load(tri, area, f_facet, n_nodes):
    """f_N = sum over the facets i around node N of f_i A_i / 3."""
    f = np.zeros(n_nodes)
    for i, t in enumerate(np.asarray(tri)):
        for a in range(3):
            f[t[a]] += f_facet[i] * area[i] / 3.0
    return f


def exchange_matrix(F, eps, area, sigma=SIGMA):
    """R_bar of eq. (Rbardef): R = sigma diag(eps A) F C^-1 diag(eps) (eq.
    (Rdef) with the area-weighted F of the paper), minus its row sums on the
    diagonal."""
    C = reflection_matrix(F, eps)
    FCi = sla.solve(C.T, F.T).T  # F C^-1
    R = sigma * (eps * area)[:, None] * FCi * eps[None, :]
    return R - np.diag(R.sum(axis=1))


def cavity_operator(P, Rbar):
    """S = P^T R_bar P (eq. (S_def_matrix))."""
    return P.T @ Rbar @ P


def residual(T, Tn, dt, M, K, S, f):
    return M @ (T - Tn) / dt + K @ T - S @ T**4 - f


def newton_step(T_n, dt, M, K, S, f, tol=1e-13, max_newton=50):
    """Implicit Euler step from T_n (n_nodes, or n_nodes x r): the root of
    Res by Newton's method with the exact Jacobian M/dt + K - 4 S diag(T^3).
    Stops when |Res|_2 <= tol |M T_n / dt|_2 (per column).  Returns (T,
    iterations, final residual norms)."""
    Tn = np.array(T_n, dtype=np.float64)
    one = Tn.ndim == 1
    if one:
        Tn = Tn[:, None]
    f = np.asarray(f, dtype=np.float64)
    f = f[:, None] if f.ndim == 1 else f
    T = Tn.copy()
    its = np.zeros(T.shape[1], dtype=np.int64)
    rns = np.zeros(T.shape[1])
    for c in range(T.shape[1]):
        x = T[:, c]
        scale = np.linalg.norm(M @ Tn[:, c] / dt)
        for it in range(max_newton + 1):
            r = residual(x, Tn[:, c], dt, M, K, S, f[:, c])
            rns[c] = np.linalg.norm(r)
            if rns[c] <= tol * scale or it == max_newton:
                break
            J = M / dt + K - 4.0 * S * (x**3)[None, :]
            x = x - np.linalg.solve(J, r)
            its[c] = it + 1
        T[:, c] = x
    return (T[:, 0] if one else T), its, rns
