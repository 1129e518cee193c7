"""Lumped transient radiative exchange (oracle; test infrastructure only).

Analogue of Sec. 3.3 on a per-facet lumped model: every facet carries a heat
capacity per unit area ``m_c`` (rho c thickness) and a source ``s`` (W/m^2),
and exchanges radiation with the cavity through the flux of eq. (12):

    m_c dT/dt = q(T) + s.

Implicit Euler gives the residual ``R(T) = m_c (T - T^n)/dt - q(T) - s``
(the analogue of the paper's time residual), driven to zero by Newton's
method.  The Jacobian is replaced by its local (diagonal) part
``D_i = m_c/dt + 4 sigma eps_i g_i T_i^3`` with ``g = F C^-1 eps`` (the
``-d q_i / d T_i`` term of eq. (12) without the reflected part, which is of
order ``(1 - eps) F^2``); the update is ``T <- T - R / D``.  The iteration
stops when ``|R|_2 <= tol |m_c T^n / dt|_2`` per right-hand side, or after
``max_newton`` updates.
"""
from __future__ import annotations

import numpy as np

from .radiosity import SIGMA, DenseRadiosity


def newton_step(rad: DenseRadiosity, Tn, src, mc, dt, tol=1e-12, max_newton=60, T_amb=None):
    """One implicit Euler step from ``Tn`` (n x r).  Returns (T, iterations,
    final residual norms).  With ``T_amb`` the cavity is open: the flux gains
    the ambient exchange of eq. (35), and the local Jacobian its derivative
    ``4 sigma (1 - c_i) T_i^3``."""
    T = np.array(Tn, dtype=np.float64, copy=True)
    scale = np.linalg.norm(mc * Tn / dt, axis=0)
    eps = rad.eps[:, None]
    g = rad.g[:, None]
    amb = 0.0
    if T_amb is not None:
        amb = (1.0 - np.clip(rad.F.sum(axis=1), 0.0, 1.0))[:, None]
    it = 0
    while True:
        q = rad.flux(T) if T_amb is None else rad.flux(T, T_amb=T_amb)
        R = mc * (T - Tn) / dt - q - src
        rn = np.linalg.norm(R, axis=0)
        if np.all(rn <= tol * scale) or it >= max_newton:
            return T, it, rn
        D = mc / dt + 4.0 * rad.sigma * (eps * g + amb) * T**3
        T = T - R / D
        it += 1


def run(rad: DenseRadiosity, T0, src, mc, dt, steps, tol=1e-12):
    """``steps`` implicit Euler steps; returns the list [T^0, T^1, ...]."""
    out = [np.array(T0, dtype=np.float64)]
    T = out[0]
    for _ in range(steps):
        T, _, _ = newton_step(rad, T, src, mc, dt, tol)
        out.append(T)
    return out
