"""Pins of the oracle's finite-element coupling (Sec. 3.1-3.4), CPU only.

* P1 triangles: on a flat patch the stiffness reproduces k h |grad u|^2 A
  for a linear field u (closed form) and gives zero at the interior node
  (patch test); the consistent mass integrates linear fields exactly.
* R of eq. (Rdef) is symmetric (reciprocity A_i F_ij = A_j F_ji makes
  diag(A) F C^-1 symmetric), so R_bar has zero row and column sums, and
  R_bar eta equals A q with q the flux of eq. (12) for facet power eta.
* S = P^T R_bar P conserves energy (1^T S = 0) and leaves a uniform
  temperature at rest; a step changes the heat content 1^T M T only by
  the sources (1^T K = 0 too).
* Facets as nodes (P = I), no conduction and a lumped mass m_c A: the step
  is the lumped transient's step (pinned by the two-plate closed form).
* Planted mistakes (flux sign, R instead of R_bar, a wrong stiffness
  factor) fail these pins.
"""
import numpy as np

from oracle import fe, geometry, radiosity, transient, viewfactor
from workloads import meshes

SIGMA = radiosity.SIGMA


def _cavity(level=2):
    v, f = meshes.icosphere(level)
    f = meshes.inward(f)
    c, n, a = geometry.facets_from_triangles(v, f)
    F = viewfactor.view_factor_matrix(c, n, a)
    eps = np.random.default_rng(7).uniform(0.2, 0.9, a.size)
    return v, f, a, F, eps


def _flat_patch():
    # 3 x 3 nodes on the unit square, 8 triangles
    xs = np.linspace(0.0, 1.0, 3)
    v = np.array([[x, y, 0.0] for y in xs for x in xs])
    tri = []
    for j in range(2):
        for i in range(2):
            a, b, c, d = 3 * j + i, 3 * j + i + 1, 3 * (j + 1) + i, 3 * (j + 1) + i + 1
            tri += [[a, b, d], [a, d, c]]
    return v, np.array(tri)


def test_p1_matrices_closed_forms():
    v, tri = _flat_patch()
    k_h, rc_h = 2.5, 3.0
    M, K, P = fe.surface_p1(v, tri, k_h, rc_h)
    g = np.array([0.7, -1.3])
    u = v[:, 0] * g[0] + v[:, 1] * g[1] + 0.4
    assert abs(u @ K @ u - k_h * (g @ g) * 1.0) <= 1e-12
    assert abs((K @ u)[4]) <= 1e-12  # interior node
    assert np.abs(K @ np.ones(9)).max() <= 1e-12
    # int u dA over the unit square = u at its centre
    assert abs(np.ones(9) @ M @ u - rc_h * (0.5 * g[0] + 0.5 * g[1] + 0.4)) <= 1e-12
    assert np.allclose(P.sum(axis=1), 1.0) and np.all((P > 0).sum(axis=1) == 3)


def test_exchange_matrix_symmetry_and_flux():
    v, f, a, F, eps = _cavity()
    Rbar = fe.exchange_matrix(F, eps, a)
    off = Rbar - np.diag(np.diag(Rbar))
    scale = np.abs(off).max()
    assert np.abs(off - off.T).max() <= 1e-12 * scale
    assert np.abs(Rbar.sum(axis=0)).max() <= 1e-11 * scale * a.size
    T = np.random.default_rng(3).uniform(300.0, 1200.0, a.size)
    q = radiosity.DenseRadiosity(F, eps).flux(T)
    assert np.linalg.norm(Rbar @ T**4 - a * q) <= 1e-12 * np.linalg.norm(a * q)


def test_cavity_operator_energy_rest_and_heat_content():
    v, f, a, F, eps = _cavity()
    M, K, P = fe.surface_p1(v, f, 1.0, 2e3)
    S = fe.cavity_operator(P, fe.exchange_matrix(F, eps, a))
    nn = v.shape[0]
    assert np.abs(np.ones(nn) @ S).max() <= 1e-12 * np.abs(S).max() * nn
    Tu = np.full(nn, 640.0)
    T1, it, _ = fe.newton_step(Tu, 0.5, M, K, S, np.zeros(nn))
    assert np.abs(T1 - Tu).max() <= 1e-9
    rng = np.random.default_rng(5)
    T0 = rng.uniform(300.0, 900.0, nn)
    src = rng.uniform(0.0, 500.0, a.size)
    fN = fe.nodal_load(f, a, src, nn)
    dt = 2.0
    T1, it, rn = fe.newton_step(T0, dt, M, K, S, fN)
    assert it.max() >= 2
    heat = np.ones(nn) @ M @ (T1 - T0) / dt
    assert abs(heat - fN.sum()) <= 1e-9 * abs(fN.sum())


def test_lumped_limit_is_the_transient_step():
    v, f, a, F, eps = _cavity()
    n = a.size
    mc, dt = 1e4, 1.0
    rng = np.random.default_rng(11)
    T0 = rng.uniform(300.0, 1500.0, n)
    s = rng.uniform(0.0, 500.0, n)
    S = fe.cavity_operator(np.eye(n), fe.exchange_matrix(F, eps, a))
    T1, it, _ = fe.newton_step(T0, dt, np.diag(mc * a), np.zeros((n, n)), S, a * s)
    Tl, _, _ = transient.newton_step(radiosity.DenseRadiosity(F, eps), T0[:, None], s[:, None], mc, dt)
    assert np.abs(T1 - Tl[:, 0]).max() <= 1e-9


def test_planted_mistakes_fail_the_pins(monkeypatch):
    v, f, a, F, eps = _cavity()
    n = a.size
    # 1. the radiation load with the wrong sign
    Rbar = fe.exchange_matrix(F, eps, a)
    T0 = np.random.default_rng(11).uniform(300.0, 1500.0, n)
    s = np.zeros(n)
    Tl, _, _ = transient.newton_step(radiosity.DenseRadiosity(F, eps), T0[:, None], s[:, None], 1e4, 1.0)
    bad = fe.newton_step(T0, 1.0, np.diag(1e4 * a), np.zeros((n, n)), -Rbar, a * s)[0]
    assert np.abs(bad - Tl[:, 0]).max() > 1e-3
    # 2. R without the row-sum correction: a uniform temperature moves
    orig = fe.exchange_matrix

    def no_bar(F_, e_, a_, sigma=SIGMA):
        C = radiosity.reflection_matrix(F_, e_)
        return sigma * (e_ * a_)[:, None] * (F_ @ np.linalg.inv(C)) * e_[None, :]

    monkeypatch.setattr(fe, "exchange_matrix", no_bar)
    M, K, P = fe.surface_p1(v, f, 1.0, 2e3)
    S = fe.cavity_operator(P, fe.exchange_matrix(F, eps, a))
    Tu = np.full(v.shape[0], 640.0)
    assert np.abs(fe.newton_step(Tu, 0.5, M, K, S, np.zeros(v.shape[0]))[0] - Tu).max() > 1e-3
    monkeypatch.setattr(fe, "exchange_matrix", orig)
    # 3. a stiffness off by a factor of two fails the closed form
    vp, tp = _flat_patch()
    M2, K2, _ = fe.surface_p1(vp, tp, 2.5, 3.0)
    g = np.array([0.7, -1.3])
    u = vp[:, 0] * g[0] + vp[:, 1] * g[1]
    assert abs(u @ (2.0 * K2) @ u - 2.5 * (g @ g)) > 1e-3
