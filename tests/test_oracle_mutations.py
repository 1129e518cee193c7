"""Planted mistakes in copies of oracle formulas must fail the pins.

Each test builds a deliberately wrong variant of one oracle step on the CPU
and shows that the closed form / invariant used to pin that step rejects it.
"""
import math

import numpy as np
import scipy.linalg as sla

from oracle import closed_forms, radiosity, viewfactor
from workloads import meshes


def _sphere_pin_error(vf_fn):
    p, n, w = meshes.projected_sphere_points(2, radius=1.3, seed=3)
    F = vf_fn(p, n, w)
    ref = closed_forms.sphere_points_F(w, 1.3)
    off = ~np.eye(w.size, dtype=bool)
    return np.max(np.abs(F[off] - ref[off]) / ref[off])


def _vf_variant(c, n, a, drop_area=False, wrong_power=False, sign_flip=False):
    d = c[None, :, :] - c[:, None, :]
    r2 = np.sum(d * d, axis=2)
    ci = np.einsum("ik,ijk->ij", n, d)
    cj = -np.einsum("jk,ijk->ij", n, d)
    if sign_flip:
        cj = -cj
    num = np.maximum(ci, 0) * np.maximum(cj, 0) * (1.0 if drop_area else a[None, :])
    den = math.pi * (r2 if wrong_power else r2 * r2)
    with np.errstate(divide="ignore", invalid="ignore"):
        F = np.where(r2 > 0, num / den, 0.0)
    np.fill_diagonal(F, 0.0)
    return F


def test_sphere_pin_accepts_oracle_and_rejects_mutants():
    assert _sphere_pin_error(viewfactor.view_factor_matrix) < 1e-13
    assert _sphere_pin_error(lambda c, n, a: _vf_variant(c, n, a)) < 1e-12
    assert _sphere_pin_error(lambda c, n, a: _vf_variant(c, n, a, drop_area=True)) > 0.1
    assert _sphere_pin_error(lambda c, n, a: _vf_variant(c, n, a, wrong_power=True)) > 0.1
    assert _sphere_pin_error(lambda c, n, a: _vf_variant(c, n, a, sign_flip=True)) > 0.1


def test_two_plate_pin_rejects_column_scaled_operator():
    """Scaling F by (1 - eps) on the wrong side leaves the two-plate flux
    unchanged (F is symmetric there) but breaks the radiosity closed form."""
    F = np.array([[0.0, 1.0], [1.0, 0.0]])
    eps = np.array([0.8, 0.3])
    T = np.array([400.0, 900.0])
    exact_J1 = closed_forms.two_plates_radiosity(0.8, 0.3, 400.0, 900.0)
    C_bad = np.eye(2) - F * (1.0 - eps)[None, :]
    J_bad = sla.solve(C_bad, radiosity.emission(eps, T))
    assert abs(J_bad[0] - exact_J1) > 1e-3 * abs(exact_J1)
    J_ok = radiosity.DenseRadiosity(F, eps).radiosity(T)
    assert abs(J_ok[0] - exact_J1) < 1e-13 * abs(exact_J1)


def test_literal_flux_pin_rejects_flux_without_g():
    v, f = meshes.cylinder(16, 8, 3, seed=2)
    from oracle import geometry
    c, n, a = geometry.facets_from_triangles(v, meshes.inward(f))
    rng = np.random.default_rng(0)
    eps = rng.uniform(0.1, 0.9, a.size)
    T = rng.uniform(300, 1500, a.size)
    F = viewfactor.view_factor_matrix(c, n, a)
    rad = radiosity.DenseRadiosity(F, eps)
    ql = radiosity.flux_eq12_literal(F, eps, a, T)
    J = rad.radiosity(T)
    q_bad = eps * (F @ J - radiosity.SIGMA * T**4)   # mutant: g replaced by 1
    assert np.linalg.norm(q_bad - ql) / np.linalg.norm(ql) > 1e-4
    assert np.linalg.norm(rad.flux(T) - ql) / np.linalg.norm(ql) < 1e-12


def _newton_step_plus_q(rad, Tn, src, mc, dt, tol=1e-15, max_newton=80):
    """Mutant of the implicit Euler step with the exchange term's sign
    flipped (``R = mc (T - T^n)/dt + q - s``, with the matching local
    Jacobian).  It conserves energy exactly like the oracle, so the energy
    invariant and the isothermal rest state both accept it."""
    T = np.array(Tn, dtype=np.float64, copy=True)
    scale = np.linalg.norm(mc * Tn / dt, axis=0)
    eps = rad.eps[:, None]
    g = rad.g[:, None]
    for _ in range(max_newton):
        R = mc * (T - Tn) / dt + rad.flux(T) - src
        if np.all(np.linalg.norm(R, axis=0) <= tol * scale):
            break
        T = T - R / (mc / dt - 4.0 * rad.sigma * eps * g * T**3)
    return T


def test_two_plate_transient_pin_rejects_flipped_exchange_sign():
    from tests.test_oracle_pins import _two_plate_step_exact

    F = np.array([[0.0, 1.0], [1.0, 0.0]])
    e1, e2, T1, T2, mc, dt = 0.8, 0.8, 400.0, 1200.0, 1.0e4, 1.0
    rad = radiosity.DenseRadiosity(F, np.array([e1, e2]))
    Tn = np.array([[T1], [T2]])
    x1, _ = _two_plate_step_exact(e1, e2, T1, T2, mc, dt)
    Tm = _newton_step_plus_q(rad, Tn, np.zeros_like(Tn), mc, dt)
    # the mutant passes the energy invariant ...
    assert abs((Tm[0, 0] + Tm[1, 0]) - (T1 + T2)) <= 1e-9 * (T1 + T2)
    # ... but heats the hot plate: the two-plate pin rejects it
    assert abs(Tm[0, 0] - x1) > 1.0
    from oracle import transient
    To, _, _ = transient.newton_step(rad, Tn, np.zeros_like(Tn), mc, dt, tol=1e-15, max_newton=80)
    assert abs(To[0, 0] - x1) <= 1e-12 * x1


def _mutant_matfree(tmp_path, name, old, new):
    """Builds ``oracle/vf_matfree.c`` with one planted change."""
    import os
    import subprocess

    from oracle import matfree
    src = open(os.path.join(os.path.dirname(matfree.__file__), "vf_matfree.c")).read()
    assert old in src
    path = tmp_path / ("%s.c" % name)
    path.write_text(src.replace(old, new, 1))
    so = tmp_path / ("%s.so" % name)
    subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-o", str(so), str(path)],
                   check=True)
    return matfree.load(str(so))


def test_matrix_free_pins_reject_planted_kernel_mistakes(tmp_path):
    """The large-n oracle's C product is pinned by the dense oracle and the
    projected-sphere closed form; a dropped area factor, a flipped cosine
    sign and a skipped last column each fail them."""
    from oracle import geometry, matfree
    v, f = meshes.ellipsoid(6, (3.0, 2.0, 1.0))
    f = meshes.inward(f)
    c, n, a = geometry.facets_from_triangles(v, f)
    F = viewfactor.view_factor_matrix(c, n, a)
    X = np.random.default_rng(4).uniform(0.5, 1.5, (a.size, 2))
    ref = F @ X
    p, nr, w = meshes.projected_sphere_points(2, radius=1.3, seed=3)
    sref = closed_forms.sphere_points_F(w, 1.3) @ np.ones(w.size)

    def errors(lib):
        mf = matfree.MatrixFreeF(c, n, a, lib=lib)
        e1 = np.max(np.abs(mf @ X - ref)) / np.max(np.abs(ref))
        ms = matfree.MatrixFreeF(p, nr, w, lib=lib)
        e2 = np.max(np.abs(ms @ np.ones(w.size) - sref)) / np.max(np.abs(sref))
        return e1, e2

    good = errors(None)
    assert max(good) < 1e-13
    for name, old, new in (("drop_area", "* aj;", ";"),
                           ("sign_flip", "const double cj = -((mx", "const double cj = ((mx"),
                           ("skip_last", "for (int64_t j = 0; j < n; ++j)", "for (int64_t j = 0; j < n - 1; ++j)")):
        e1, e2 = errors(_mutant_matfree(tmp_path, name, old, new))
        assert max(e1, e2) > 1e-3, name


def test_recompression_pins_reject_planted_mistakes():
    """A truncation on the largest discarded singular value instead of the
    Frobenius tail, a core without its singular values, and factors whose
    QR is taken on the wrong side each fail the Eckart-Young pin."""
    from oracle import aca

    # one dominant value and a flat tail: the Frobenius and the largest-value
    # criteria keep different ranks
    s = np.array([1.0] + [1e-2] * 10 + [1e-3])
    rng = np.random.default_rng(22)
    k = s.size
    Q1, _ = np.linalg.qr(rng.standard_normal((60, k)))
    Q2, _ = np.linalg.qr(rng.standard_normal((50, k)))
    Mx = np.eye(k) + 0.3 * rng.standard_normal((k, k))
    U, V = Q1 @ np.diag(s) @ Mx, Q2 @ np.linalg.inv(Mx).T
    X = U @ V.T
    tol = 2e-2
    tail = np.sqrt(np.cumsum((s**2)[::-1]))[::-1]
    r_exp = next(q for q in range(1, k) if tail[q] <= tol * np.linalg.norm(s))

    def pin_ok(fn):
        U2, V2 = fn(U, V, tol)
        err = np.linalg.norm(X - U2 @ V2.T)
        return U2.shape[1] == r_exp and abs(err - tail[r_exp]) <= 1e-10 * tail[r_exp]

    def spectral(U, V, tol):
        Qu, Ru = np.linalg.qr(U)
        Qv, Rv = np.linalg.qr(V)
        W, S, Zt = np.linalg.svd(Ru @ Rv.T)
        r = next((q for q in range(1, S.size) if S[q] <= tol * S[0]), S.size)
        return Qu @ (W[:, :r] * S[:r]), Qv @ Zt[:r].T

    def no_sigma(U, V, tol):
        U2, V2 = aca.recompress(U, V, tol)
        return U2 / np.linalg.norm(U2, axis=0), V2

    def wrong_side(U, V, tol):
        Qu, Ru = np.linalg.qr(U)
        Qv, Rv = np.linalg.qr(V)
        W, S, Zt = np.linalg.svd(Ru.T @ Rv)
        r = aca.recompress(U, V, tol)[0].shape[1]
        return Qu @ (W[:, :r] * S[:r]), Qv @ Zt[:r].T

    assert pin_ok(aca.recompress)
    for fn in (spectral, no_sigma, wrong_side):
        assert not pin_ok(fn), fn.__name__


def test_ambient_pins_reject_planted_mistakes():
    """The spherical-cap closed form rejects a flipped ambient sign and a
    dropped view fraction (1 - c); the closed icosphere rejects a row sum
    used without the clamp of eq. (33)."""
    R = 1.4
    p, nr, w = meshes.projected_sphere_points(3, radius=R, seed=31)
    cap = p[:, 2] > 0.25 * R
    p, nr, w = p[cap], nr[cap], w[cap]
    rng = np.random.default_rng(32)
    eps = rng.uniform(0.1, 0.9, w.size)
    T = rng.uniform(300.0, 1500.0, w.size)
    T_amb = 350.0
    F = viewfactor.view_factor_matrix(p, nr, w)
    rad = radiosity.DenseRadiosity(F, eps)
    q12 = rad.flux(T)
    s_exact = (w.sum() - w) / (4.0 * math.pi * R**2)
    q_exact = closed_forms.sphere_points_flux(w, eps, T, R)[0] - radiosity.SIGMA * (1.0 - s_exact) * (T**4 - T_amb**4)

    def cap_ok(q):
        return np.linalg.norm(q - q_exact) <= 1e-12 * np.linalg.norm(q_exact)

    c = radiosity.clamped_row_sums(F)
    assert cap_ok(q12 + radiosity.ambient_flux(c, T, T_amb))
    assert not cap_ok(q12 - radiosity.ambient_flux(c, T, T_amb))                       # sign
    assert not cap_ok(q12 - radiosity.SIGMA * (T**4 - T_amb**4))                       # no (1 - c)
    v, f = meshes.icosphere(2)
    f = meshes.inward(f)
    cc, nn, aa = __import__("oracle.geometry", fromlist=["x"]).facets_from_triangles(v, f)
    Fi = viewfactor.view_factor_matrix(cc, nn, aa)
    Ti = np.random.default_rng(33).uniform(300.0, 1500.0, aa.size)
    assert np.all(radiosity.ambient_flux(radiosity.clamped_row_sums(Fi), Ti, 400.0) == 0.0)
    assert np.any(radiosity.ambient_flux(Fi.sum(axis=1), Ti, 400.0) != 0.0)            # unclamped


def test_full_pivot_pins_reject_planted_mistakes():
    """A cross whose row is not divided by the pivot, and a pivot searched
    only in the first row of the residual, each fail the planted-rank pin or
    the skeleton identity of eq. (30)."""
    from oracle import aca

    rng = np.random.default_rng(41)
    X = rng.standard_normal((40, 5)) @ rng.standard_normal((5, 30))

    def run(undivided=False, row_only=False):
        R = X.copy()
        us, vs = [], []
        for _ in range(30):
            if row_only:
                i = 0
                j = int(np.argmax(np.abs(R[0])))
            else:
                i, j = divmod(int(np.argmax(np.abs(R))), R.shape[1])
            if R[i, j] == 0.0:
                break
            u = R[:, j].copy()
            v = R[i, :] if undivided else R[i, :] / R[i, j]
            R = R - np.outer(u, v)
            us.append(u)
            vs.append(v)
            if np.linalg.norm(R) <= 1e-13 * np.linalg.norm(X):
                break
        U, V = np.stack(us, axis=1), np.stack(vs, axis=1)
        return U.shape[1] == 5 and np.linalg.norm(X - U @ V.T) <= 1e-12 * np.linalg.norm(X)

    assert run()
    assert not run(undivided=True)
    assert not run(row_only=True)
