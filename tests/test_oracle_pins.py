"""Pins of the oracle against what the paper and the mathematics fix.

Every check here compares the oracle with something other than itself: a
closed form, an invariant, a hand-derived structure, a library routine or the
exact result within the paper's error bound.  CPU only.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import aca, clustering, closed_forms, geometry, radiosity, transient, viewfactor
from workloads import configs, meshes

SIGMA = 5.670374e-8


# --------------------------------------------------------------------------- geometry
def test_facet_geometry_right_triangle():
    v = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0], [0.0, 3.0, 0.0]])
    c, n, a = geometry.facets_from_triangles(v, np.array([[0, 1, 2]]))
    assert np.allclose(c[0], [2.0 / 3.0, 1.0, 0.0], rtol=0, atol=1e-15)
    assert np.allclose(n[0], [0.0, 0.0, 1.0], rtol=0, atol=1e-15)
    assert a[0] == pytest.approx(3.0, rel=1e-15)


def test_inward_normals_on_generated_cavities():
    for v, f in (meshes.icosphere(2), meshes.ellipsoid(6, (3, 2, 1)), meshes.cylinder(24, 16, 4)):
        c, n, a = geometry.facets_from_triangles(v, meshes.inward(f))
        # star-shaped about the origin: inward normals point back towards it
        assert np.all(np.einsum("ij,ij->i", n, c) < 0)
        assert np.all(a > 0)


# --------------------------------------------------------------------------- view factors, eq. (10)
def test_sphere_identity_projected_points():
    """Points on a sphere with inward radial normals: every off-diagonal
    centroid-rule entry equals A_j / (4 pi R^2) whatever the weights."""
    for R in (1.0, 2.5):
        p, n, w = meshes.projected_sphere_points(3, radius=R, seed=11)
        F = viewfactor.view_factor_matrix(p, n, w)
        ref = closed_forms.sphere_points_F(w, R)
        off = ~np.eye(w.size, dtype=bool)
        assert np.max(np.abs(F[off] - ref[off]) / ref[off]) < 1e-13
        assert np.all(np.diag(F) == 0.0)


def test_reciprocity_and_zero_diagonal():
    cav = configs.c1_icosphere()
    c, n, a = geometry.facets_from_triangles(cav.v, cav.tri)
    F = viewfactor.view_factor_matrix(c, n, a)
    G = a[:, None] * F
    assert np.max(np.abs(G - G.T)) <= 1e-15 * np.max(np.abs(G))
    assert np.all(np.diag(F) == 0.0)
    assert np.all(F >= 0.0)


def test_parallel_squares_converge_to_exact_view_factor():
    """Sec. 4.2 Example 2 geometry (two L x L plates a distance L apart): the
    centroid rule converges at O(h^2) to the exact 0.199825."""
    exact = closed_forms.parallel_rectangles(1.0, 1.0, 1.0)
    assert exact == pytest.approx(0.199825, abs=5e-7)
    errs = []
    for nps in (8, 16, 32):
        c, n, a = meshes.parallel_plates(nps)
        m = nps * nps
        F = viewfactor.view_factor_block(c, n, a, np.arange(m), np.arange(m, 2 * m))
        errs.append(abs(float(np.sum(a[:m, None] * F)) - exact))
    assert errs[2] < 1e-4
    for e0, e1 in zip(errs, errs[1:]):
        assert 3.5 < e0 / e1 < 4.5


def test_row_sums_tend_to_one_in_closed_convex_enclosure():
    """Sec. 6.1: in a closed cavity the true row sums are 1; the centroid
    rule misses by O(h^2) on recursive icospheres."""
    dev = []
    for lvl in (1, 2, 3):
        v, f = meshes.icosphere(lvl)
        c, n, a = geometry.facets_from_triangles(v, meshes.inward(f))
        s = viewfactor.row_sums(viewfactor.view_factor_matrix(c, n, a))
        dev.append(np.max(np.abs(s - 1.0)))
    assert dev[2] < 3e-3
    assert 3.0 < dev[1] / dev[2] < 5.0


def test_back_facing_pairs_are_zero():
    c = np.array([[0.0, 0, 0], [1.0, 0, 0]])
    n = np.array([[-1.0, 0, 0], [1.0, 0, 0]])  # facing away from each other
    F = viewfactor.view_factor_matrix(c, n, np.ones(2))
    assert np.all(F == 0.0)


def test_closed_cavity_scaling_clamps_and_rescales():
    F = np.array([[0.0, 0.25, 0.25], [0.6, 0.0, 0.6], [0.0, 0.0, 0.0]])
    out = viewfactor.closed_cavity_scaling(F)
    assert np.allclose(out[0], [0.0, 0.5, 0.5])   # s = 0.5 -> divided by 0.5
    assert np.allclose(out[1], F[1])              # s = 1.2 clamps to 1
    assert np.all(out[2] == 0.0)                  # c = 0: left alone


# --------------------------------------------------------------------------- radiosity and flux
@pytest.mark.parametrize("e1,e2,T1,T2", [(0.8, 0.3, 400.0, 900.0), (1.0, 0.5, 1200.0, 300.0), (0.05, 0.95, 700.0, 701.0)])
def test_two_infinite_plates(e1, e2, T1, T2):
    """Sec. 2.2 closed form: two facets that see only each other."""
    F = np.array([[0.0, 1.0], [1.0, 0.0]])
    rad = radiosity.DenseRadiosity(F, np.array([e1, e2]))
    q = rad.flux(np.array([T1, T2]))
    exact = closed_forms.two_plates_flux(e1, e2, T1, T2)
    tol = 1e-13 * SIGMA * max(T1, T2) ** 4   # absolute: the flux is a difference of T^4 terms
    assert q[0] == pytest.approx(exact, abs=tol)
    assert q[1] == pytest.approx(-exact, abs=tol)
    ql = radiosity.flux_eq12_literal(F, np.array([e1, e2]), np.ones(2), np.array([T1, T2]))
    assert ql[0] == pytest.approx(exact, abs=tol)
    J = rad.radiosity(np.array([T1, T2]))
    assert J[0] == pytest.approx(closed_forms.two_plates_radiosity(e1, e2, T1, T2), rel=1e-14)
    assert J[1] == pytest.approx(closed_forms.two_plates_radiosity(e2, e1, T2, T1), rel=1e-14)


def test_projected_sphere_closed_form_solution():
    p, n, w = meshes.projected_sphere_points(3, radius=1.7, seed=5)
    rng = np.random.default_rng(9)
    eps = rng.uniform(0.1, 0.9, w.size)
    T = rng.uniform(300.0, 1500.0, w.size)
    F = viewfactor.view_factor_matrix(p, n, w)
    rad = radiosity.DenseRadiosity(F, eps)
    J = rad.radiosity(T)
    q = rad.flux(T)
    q_ref, J_ref = closed_forms.sphere_points_flux(w, eps, T, 1.7)
    assert np.linalg.norm(J - J_ref) / np.linalg.norm(J_ref) < 1e-13
    assert np.linalg.norm(q - q_ref) / np.linalg.norm(q_ref) < 1e-12


def test_literal_eq12_equals_rewritten_flux_and_conserves_energy():
    v, f = meshes.cylinder(24, 12, 4, seed=3)
    c, n, a = geometry.facets_from_triangles(v, meshes.inward(f))
    rng = np.random.default_rng(1)
    eps = rng.uniform(0.1, 0.9, a.size)
    T = rng.uniform(300.0, 1500.0, a.size)
    F = viewfactor.view_factor_matrix(c, n, a)
    rad = radiosity.DenseRadiosity(F, eps)
    q = rad.flux(T)
    ql = radiosity.flux_eq12_literal(F, eps, a, T)
    assert np.linalg.norm(q - ql) / np.linalg.norm(ql) < 1e-12
    # energy: sum_i A_i q_i = 0 (A F symmetric makes diag(eps) A F C^-1 diag(eps) symmetric)
    assert abs(np.sum(a * q)) <= 1e-13 * np.sum(np.abs(a * q))
    # the textbook net-radiation form eps (FJ - sigma T^4) leaks energy when rows do not sum to 1
    J = rad.radiosity(T)
    q_naive = eps * (F @ J - SIGMA * T**4)
    assert abs(np.sum(a * q_naive)) > 1e-6 * np.sum(np.abs(a * q_naive))


def test_blackbody_and_isothermal_special_cases():
    cav = configs.c1_icosphere()
    c, n, a = geometry.facets_from_triangles(cav.v, cav.tri)
    F = viewfactor.view_factor_matrix(c, n, a)
    T = cav.T[:, 0]
    rad1 = radiosity.DenseRadiosity(F, np.ones(a.size))
    assert np.allclose(rad1.radiosity(T), SIGMA * T**4, rtol=1e-15, atol=0)
    rad = radiosity.DenseRadiosity(F, cav.eps)
    q_iso = rad.flux(np.full(a.size, 812.0))
    assert np.max(np.abs(q_iso)) <= 1e-12 * SIGMA * 812.0**4


def test_lu_solution_agrees_with_library_gmres():
    cav = configs.c1_icosphere()
    c, n, a = geometry.facets_from_triangles(cav.v, cav.tri)
    F = viewfactor.view_factor_matrix(c, n, a)
    rad = radiosity.DenseRadiosity(F, cav.eps)
    b = radiosity.emission(cav.eps, cav.T[:, 0])
    x, info = spla.gmres(rad.C, b, x0=b, rtol=1e-13, restart=30, maxiter=200)
    assert info == 0
    assert np.linalg.norm(x - rad.solve(b)) / np.linalg.norm(x) < 1e-12


# --------------------------------------------------------------------------- clustering, Alg. 1 and 2
def test_example1_line_block_structure():
    """Sec. 4.2 Example 1 with n = 8, n_min = 1 and c = 1 (hand-derived):
    diagonal singletons are dense; off-diagonal singleton pairs inside a pair
    cluster and all pairs of 2-clusters that are not on the diagonal are
    admissible; no larger block is."""
    root, perm = clustering.build_index_tree(meshes.line_points(8), 1)
    assert np.array_equal(perm, np.arange(8))
    dense, lr = clustering.build_block_tree(root, 1.0)
    assert dense == [(i, i + 1, i, i + 1) for i in range(8)]
    exp = []
    for i in range(0, 8, 2):
        exp += [(i, i + 1, i + 1, i + 2), (i + 1, i + 2, i, i + 1)]
    pairs = [(0, 2), (2, 4), (4, 6), (6, 8)]
    exp += [(a0, a1, b0, b1) for (a0, a1) in pairs for (b0, b1) in pairs if a0 != b0]
    assert sorted(lr) == sorted(exp)
    assert len(lr) == 20


def _cover_count(n, blocks):
    cov = np.zeros((n, n), dtype=np.int32)
    for r0, r1, c0, c1 in blocks:
        cov[r0:r1, c0:c1] += 1
    return cov


@pytest.mark.parametrize("n_min,eta", [(32, 2.0), (16, 1.5), (7, 0.8)])
def test_block_tree_partitions_and_admissible_blocks_are_far(n_min, eta):
    v, f = meshes.ellipsoid(7, (3.0, 2.0, 1.0))
    c, n, a = geometry.facets_from_triangles(v, meshes.inward(f))
    root, perm = clustering.build_index_tree(c, n_min)
    assert np.array_equal(np.sort(perm), np.arange(a.size))
    dense, lr = clustering.build_block_tree(root, eta)
    assert np.all(_cover_count(a.size, dense + lr) == 1)
    cp = c[perm]
    for r0, r1, c0, c1 in lr:
        P, Q = cp[r0:r1], cp[c0:c1]
        dmin = np.sqrt(np.min(np.sum((P[:, None, :] - Q[None, :, :]) ** 2, axis=2)))
        dP = np.sqrt(np.max(np.sum((P[:, None, :] - P[None, :, :]) ** 2, axis=2)))
        dQ = np.sqrt(np.max(np.sum((Q[:, None, :] - Q[None, :, :]) ** 2, axis=2)))
        assert min(dP, dQ) <= eta * dmin * (1 + 1e-12)
    for lf in clustering.leaves(root):
        assert 1 <= lf.size <= n_min


def test_median_split_is_balanced_and_contiguous():
    cav = configs.c1_icosphere()
    c, n, a = geometry.facets_from_triangles(cav.v, cav.tri)
    root, perm = clustering.build_index_tree(c, 32)
    lv = clustering.leaves(root)
    assert len(lv) == 64 and all(l.size == 20 for l in lv)

    def check(cl):
        if cl.children:
            l, r = cl.children
            assert l.begin == cl.begin and l.end == r.begin and r.end == cl.end
            assert r.size - l.size in (0, 1)
            for ch in cl.children:
                check(ch)
    check(root)


# --------------------------------------------------------------------------- ACA, eqs. (30)-(31)
def _far_block():
    cav = configs.c1_icosphere()
    c, n, a = geometry.facets_from_triangles(cav.v, cav.tri)
    root, perm = clustering.build_index_tree(c, 32)
    _, lr = clustering.build_block_tree(root, 2.0)
    cp, np_, ap = c[perm], n[perm], a[perm]
    big = max(lr, key=lambda b: (b[1] - b[0]) * (b[3] - b[2]))
    r0, r1, c0, c1 = big
    X = viewfactor.view_factor_block(cp, np_, ap, np.arange(r0, r1), np.arange(c0, c1))
    return X


def test_aca_cross_equals_skeleton_formula():
    """Eq. (30): the accumulated crosses equal X(:,C) X(R,C)^-1 X(R,:) for the
    pivot sets the algorithm picked."""
    X = _far_block()
    res = aca.aca_partial(lambda i: X[i], lambda j: X[:, j], *X.shape, 1e-6, 64)
    assert res.converged and 1 <= len(res.rows) < 20
    R, C = res.rows, res.cols
    skel = X[:, C] @ np.linalg.solve(X[np.ix_(R, C)], X[R, :])
    assert np.linalg.norm(res.U @ res.V.T - skel) <= 1e-12 * np.linalg.norm(X)
    # cross approximation interpolates the pivot rows and columns
    E = X - res.U @ res.V.T
    assert np.max(np.abs(E[R, :])) <= 1e-13 * np.max(np.abs(X))
    assert np.max(np.abs(E[:, C])) <= 1e-13 * np.max(np.abs(X))


def test_aca_meets_relative_tolerance_on_admissible_block():
    X = _far_block()
    for tol in (1e-4, 1e-6, 1e-8):
        res = aca.aca_partial(lambda i: X[i], lambda j: X[:, j], *X.shape, tol, 200)
        err = np.linalg.norm(X - res.U @ res.V.T) / np.linalg.norm(X)
        assert err <= 10 * tol


def test_aca_recovers_exact_low_rank_and_handles_zero_rows():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((40, 3)) @ rng.standard_normal((3, 30))
    X[0] = 0.0   # first row exactly zero: retried on the next unused row
    res = aca.aca_partial(lambda i: X[i], lambda j: X[:, j], 40, 30, 1e-12, 30)
    assert res.converged and 3 <= res.U.shape[1] <= 4
    assert res.rows[0] == 1
    assert np.linalg.norm(X - res.U @ res.V.T) <= 1e-13 * np.linalg.norm(X)
    Z = np.zeros((5, 6))
    rz = aca.aca_partial(lambda i: Z[i], lambda j: Z[:, j], 5, 6, 1e-6, 3)
    assert rz.converged and rz.U.shape[1] == 0


def test_sphere_points_blocks_have_rank_one():
    p, n, w = meshes.projected_sphere_points(3, seed=2)
    H = aca.build_hmatrix(p, n, w, 16, 1.5, 1e-10)
    assert len(H.lowrank) > 0 and H.fallback == 0
    # the first cross is exact; a second cross can only carry rounding noise
    for r0, r1, c0, c1, U, V in H.lowrank:
        assert U.shape[1] <= 2
        if U.shape[1] == 2:
            assert np.linalg.norm(U[:, 1]) * np.linalg.norm(V[:, 1]) <= 1e-12 * np.linalg.norm(U[:, 0]) * np.linalg.norm(V[:, 0])


def test_hmatrix_global_error_within_tolerance():
    """Eq. (31) per block implies the global Frobenius bound (paper Table 2
    reports ~0.1 eps_rel for its geometry)."""
    v, f = meshes.cylinder(40, 24, 6, seed=1)
    c, n, a = geometry.facets_from_triangles(v, meshes.inward(f))
    F = viewfactor.view_factor_matrix(c, n, a)
    for tol in (1e-3, 1e-5):
        H = aca.build_hmatrix(c, n, a, 24, 1.5, tol)
        err = np.linalg.norm(H.to_dense() - F) / np.linalg.norm(F)
        assert err <= tol
        x = np.random.default_rng(0).standard_normal(a.size)
        assert np.linalg.norm(H.matvec(x) - F @ x) <= 2 * tol * np.linalg.norm(F @ x) * 10


# --------------------------------------------------------------------------- transient
def test_transient_energy_invariant_and_isothermal_rest():
    v, f = meshes.ellipsoid(4, (2.0, 1.5, 1.0))
    c, n, a = geometry.facets_from_triangles(v, meshes.inward(f))
    F = viewfactor.view_factor_matrix(c, n, a)
    rad = radiosity.DenseRadiosity(F, np.full(a.size, 0.8))
    rng = np.random.default_rng(2)
    T0 = rng.uniform(300, 1000, (a.size, 2))
    src = rng.uniform(0, 500, (a.size, 2))
    mc, dt = 1.0e4, 1.0
    T1, it, rn = transient.newton_step(rad, T0, src, mc, dt, tol=1e-13)
    assert 2 <= it <= 30
    lhs = np.sum(a[:, None] * mc * (T1 - T0) / dt, axis=0)
    rhs = np.sum(a[:, None] * src, axis=0)
    assert np.allclose(lhs, rhs, rtol=1e-9)
    Tiso = np.full((a.size, 1), 600.0)
    T2, it2, _ = transient.newton_step(rad, Tiso, np.zeros_like(Tiso), mc, dt)
    assert np.max(np.abs(T2 - 600.0)) < 1e-9


def _two_plate_step_exact(e1, e2, T1, T2, mc, dt, sigma=SIGMA):
    """One implicit Euler step of two facing infinite gray plates (equal
    areas and heat capacities, no source), solved as a scalar equation.

    The plates exchange only with each other, so energy is conserved and the
    new temperatures satisfy T1' + T2' = T1 + T2.  The net flux into plate 1
    is the Sec. 2.2 closed form, so the step reduces to
    ``mc (T1' - T1)/dt = q1(T1', T1 + T2 - T1')``, whose left side increases
    and right side decreases with T1': one root, bracketed by the two
    initial temperatures."""
    from scipy.optimize import brentq

    S = T1 + T2

    def f(x):
        return mc * (x - T1) / dt - closed_forms.two_plates_flux(e1, e2, x, S - x, sigma)

    lo, hi = min(T1, T2), max(T1, T2)
    x = brentq(f, lo, hi, xtol=1e-14, rtol=4 * np.finfo(float).eps, maxiter=400)
    return x, S - x


@pytest.mark.parametrize("e1,e2,T1,T2,dt", [(0.8, 0.8, 400.0, 1200.0, 1.0), (0.3, 0.9, 1500.0, 350.0, 5.0),
                                            (1.0, 0.5, 700.0, 710.0, 0.5)])
def test_transient_two_plates_direction_of_exchange(e1, e2, T1, T2, dt):
    """Fixes the sign of the exchange term: heat flows from the hotter plate
    to the colder one at the two-plate rate of Sec. 2.2."""
    F = np.array([[0.0, 1.0], [1.0, 0.0]])
    rad = radiosity.DenseRadiosity(F, np.array([e1, e2]))
    mc = 1.0e4
    Tn = np.array([[T1], [T2]])
    T, it, _ = transient.newton_step(rad, Tn, np.zeros_like(Tn), mc, dt, tol=1e-15, max_newton=80)
    x1, x2 = _two_plate_step_exact(e1, e2, T1, T2, mc, dt)
    assert abs(T[0, 0] - x1) <= 1e-12 * x1
    assert abs(T[1, 0] - x2) <= 1e-12 * x2
    # the hotter plate cooled, the colder one warmed
    assert (T[0, 0] - T1) * (T2 - T1) > 0


# ---------------------------------------------------------------- recompression (Sec. 4.3 post-processing)
def _planted(m, n, svals, seed):
    """U V^T = Q1 diag(s) Q2^T with known singular values s, spread over a
    random (well-conditioned) non-orthogonal factor pair."""
    rng = np.random.default_rng(seed)
    k = len(svals)
    Q1, _ = np.linalg.qr(rng.standard_normal((m, k)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, k)))
    Mx = np.eye(k) + 0.3 * rng.standard_normal((k, k))
    U = Q1 @ np.diag(svals) @ Mx
    V = Q2 @ np.linalg.inv(Mx).T
    return U, V, Q1 @ np.diag(svals) @ Q2.T


def test_recompress_recovers_a_planted_rank():
    rng = np.random.default_rng(21)
    m, n, r, k = 90, 70, 5, 14
    U = rng.standard_normal((m, r)) @ rng.standard_normal((r, k))
    V = rng.standard_normal((n, r)) @ rng.standard_normal((r, k))
    U2, V2 = aca.recompress(U, V, 1e-10)
    X = U @ V.T
    assert U2.shape == (m, r) and V2.shape == (n, r)
    assert np.linalg.norm(U2 @ V2.T - X) <= 1e-13 * np.linalg.norm(X)
    assert np.allclose(V2.T @ V2, np.eye(r), atol=1e-13)


def test_recompress_truncates_at_the_eckart_young_error():
    """Known singular values (s_i = 10^(-i/2), and one dominant value over a
    flat tail): the kept rank is the smallest r with
    sqrt(sum_{i>=r} s_i^2) <= tol |s|, and the error of the truncated factors
    equals that tail (the best rank-r error, Eckart-Young)."""
    spectra = ((10.0 ** (-0.5 * np.arange(12)), (3e-1, 2e-2, 1e-3, 5e-5)),
               (np.array([1.0] + [1e-2] * 10 + [1e-3]), (2e-2, 5e-3)))
    for s, tols in spectra:
        U, V, X = _planted(60, 50, s, 22)
        tail = np.sqrt(np.cumsum((s**2)[::-1]))[::-1]
        for tol in tols:
            r_exp = next(q for q in range(1, s.size) if tail[q] <= tol * np.linalg.norm(s))
            U2, V2 = aca.recompress(U, V, tol)
            assert U2.shape[1] == r_exp
            err = np.linalg.norm(X - U2 @ V2.T)
            assert abs(err - tail[r_exp]) <= 1e-10 * tail[r_exp]
            assert err <= tol * np.linalg.norm(X)


def test_recompressed_hmatrix_meets_tolerance_with_fewer_entries():
    v, f = meshes.ellipsoid(9, (3.0, 2.0, 1.0))
    f = meshes.inward(f)
    c, n, a = geometry.facets_from_triangles(v, f)
    F = viewfactor.view_factor_matrix(c, n, a)
    H = aca.build_hmatrix(c, n, a, 32, 1.5, 1e-6)
    Hr = aca.build_hmatrix(c, n, a, 32, 1.5, 1e-6, recompress_tol=1e-6)
    e, er = (np.linalg.norm(h.to_dense() - F) / np.linalg.norm(F) for h in (H, Hr))
    assert er <= 1e-6 and e <= 1e-6
    assert Hr.stored_entries()[1] < 0.9 * H.stored_entries()[1]
    assert all(B[4].shape[1] <= A[4].shape[1] for A, B in zip(H.lowrank, Hr.lowrank))


# ---------------------------------------------------------------- open cavities (eqs. (32)-(35))
def test_open_cavity_flux_on_a_spherical_cap_matches_closed_form():
    """Sphere points with radial normals restricted to a cap: every entry is
    still w_j / (4 pi R^2), so the row sums are (W - w_i) / A_s < 1 in closed
    form, the eq. (12) flux follows the projected-sphere closed form over the
    cap's weights, and the ambient term of eq. (35) adds
    -sigma (1 - s_i)(T_i^4 - T_amb^4)."""
    R = 1.4
    p, nr, w = meshes.projected_sphere_points(3, radius=R, seed=31)
    cap = p[:, 2] > 0.25 * R
    p, nr, w = p[cap], nr[cap], w[cap]
    rng = np.random.default_rng(32)
    eps = rng.uniform(0.1, 0.9, w.size)
    T = rng.uniform(300.0, 1500.0, w.size)
    T_amb = 350.0
    F = viewfactor.view_factor_matrix(p, nr, w)
    As = 4.0 * math.pi * R**2
    s_exact = (w.sum() - w) / As
    assert np.max(np.abs(radiosity.clamped_row_sums(F) - s_exact)) <= 1e-13
    rad = radiosity.DenseRadiosity(F, eps)
    q = rad.flux(T, T_amb=T_amb)
    q12, _ = closed_forms.sphere_points_flux(w, eps, T, R)
    q_exact = q12 - radiosity.SIGMA * (1.0 - s_exact) * (T**4 - T_amb**4)
    assert np.linalg.norm(q - q_exact) <= 1e-12 * np.linalg.norm(q_exact)


def test_isolated_facet_exchanges_only_with_the_ambient():
    """A facet that sees nothing (its F row is zero, Sec. 6.1's isolated
    facets) has J = eps sigma T^4 and q = -sigma (T^4 - T_amb^4); one implicit
    Euler step of it is the scalar equation
    mc (T' - T)/dt = -sigma (T'^4 - T_amb^4) + s, solved here by bracketing."""
    from scipy.optimize import brentq
    # two facing pairs (0-1 and 2-3) and facet 4, which faces away from all
    c = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, -1.0], [5.0, 0.0, 0.0], [5.0, 0.0, 1.0], [10.0, 0.0, 0.0]])
    nrm = np.array([[0.0, 0.0, -1.0], [0.0, 0.0, 1.0], [0.0, 0.0, 1.0], [0.0, 0.0, -1.0], [1.0, 0.0, 0.0]])
    A = np.full(5, 0.1)
    F = viewfactor.view_factor_matrix(c, nrm, A)
    iso = np.where(~np.any(F != 0.0, axis=1))[0]
    assert list(iso) == [4]
    eps = np.array([0.7, 0.6, 0.5, 0.4, 0.3])
    T = np.array([900.0, 700.0, 500.0, 800.0, 650.0])
    T_amb = 300.0
    rad = radiosity.DenseRadiosity(F, eps)
    J = rad.radiosity(T)
    q = rad.flux(T, J, T_amb=T_amb)
    sig = radiosity.SIGMA
    assert J[4] == pytest.approx(eps[4] * sig * T[4] ** 4, rel=1e-15)
    assert q[4] == pytest.approx(-sig * (T[4] ** 4 - T_amb**4), rel=1e-13)
    mc, dt, s = 1e4, 1.0, 250.0
    Tn = T[:, None]
    src = np.full((5, 1), s)
    T1, _, _ = transient.newton_step(rad, Tn, src, mc, dt, tol=1e-14, T_amb=T_amb)
    root = brentq(lambda x: mc * (x - T[4]) / dt + sig * (x**4 - T_amb**4) - s, 300.0, 900.0, xtol=1e-13)
    assert T1[4, 0] == pytest.approx(root, rel=1e-12)


def test_ambient_term_vanishes_in_a_closed_convex_cavity():
    """On a recursive icosphere every centroid-rule row sum exceeds 1, so the
    clamp of eq. (33) gives c = 1 and the open-cavity flux equals eq. (12)."""
    v, f = meshes.icosphere(2)
    f = meshes.inward(f)
    c, n, a = geometry.facets_from_triangles(v, f)
    F = viewfactor.view_factor_matrix(c, n, a)
    assert np.all(F.sum(axis=1) > 1.0)
    rng = np.random.default_rng(33)
    eps = rng.uniform(0.1, 0.9, a.size)
    T = rng.uniform(300.0, 1500.0, a.size)
    rad = radiosity.DenseRadiosity(F, eps)
    assert np.array_equal(rad.flux(T, T_amb=400.0), rad.flux(T))


def test_fibonacci_spiral_is_an_open_cavity_with_isolated_facets():
    """The 13-sphere spiral (Sec. 6): centres follow the Fibonacci offsets
    (spheres 1-2 and 2-3 a diagonal of the unit square apart), every row sum
    is below 1 (open), facets of one sphere never see each other (convex
    spheres, back-face rule), and some 7-9% of the facets see no other facet
    at all (the paper reports about 7%)."""
    c = meshes.fibonacci_centers()
    assert np.allclose(c[1, :2], [1.0, 1.0]) and np.allclose(c[2, :2], [0.0, 2.0])
    assert np.allclose(c[12, :2], [-15.0, -3.0])
    v, f, sid = meshes.fibonacci_spheres(3)
    cc, nn, aa = geometry.facets_from_triangles(v, f)
    F = viewfactor.view_factor_matrix(cc, nn, aa)
    s = F.sum(axis=1)
    assert np.all(s < 1.0)
    same = sid[:, None] == sid[None, :]
    assert np.all(F[same] == 0.0)
    iso = ~np.any(F != 0.0, axis=1)
    assert 0.06 <= iso.mean() <= 0.10
    G = aa[:, None] * F
    assert np.max(np.abs(G - G.T)) <= 1e-15 * np.max(G)


# ---------------------------------------------------------------- fully pivoted ACA (Sec. 1, Sec. 4.3)
def test_full_pivot_aca_recovers_planted_rank_and_pivots_on_the_largest_entry():
    rng = np.random.default_rng(41)
    X = rng.standard_normal((40, 5)) @ rng.standard_normal((5, 30))
    res = aca.aca_full(X, 1e-13, 30)
    assert res.converged and res.U.shape[1] == 5
    assert np.linalg.norm(X - res.U @ res.V.T) <= 1e-12 * np.linalg.norm(X)
    i, j = np.unravel_index(np.argmax(np.abs(X)), X.shape)
    assert (res.rows[0], res.cols[0]) == (i, j)
    # cross = skeleton formula eq. (30) over the chosen rows and columns
    R, Cc = res.rows, res.cols
    S = X[:, Cc] @ np.linalg.solve(X[np.ix_(R, Cc)], X[R, :])
    assert np.linalg.norm(S - res.U @ res.V.T) <= 1e-10 * np.linalg.norm(X)


def test_full_pivot_aca_meets_eq31_on_every_block_where_partial_pivoting_fails():
    """The 13-sphere spiral: partial pivoting leaves whole zero-structured
    parts of some admissible blocks out (per-block errors of several percent),
    while full pivoting meets |X - U V^T|_F <= tol |X|_F on every block."""
    from workloads import configs
    cav = configs.fibonacci_spiral(nu=2)
    c, n, a = geometry.facets_from_triangles(cav.v, cav.tri)
    F = viewfactor.view_factor_matrix(c, n, a)
    tol = 1e-8
    Hf = aca.build_hmatrix(c, n, a, 16, 1.5, tol, pivot="full")
    Hp = aca.build_hmatrix(c, n, a, 16, 1.5, tol, pivot="partial")
    Fp = F[np.ix_(Hf.perm, Hf.perm)]
    worst = 0.0
    for r0, r1, c0, c1, U, V in Hf.lowrank:
        X = Fp[r0:r1, c0:c1]
        worst = max(worst, np.linalg.norm(X - U @ V.T) / max(np.linalg.norm(X), 1e-300))
    assert worst <= tol
    assert np.linalg.norm(Hf.to_dense() - F) <= tol * np.linalg.norm(F)
    assert np.linalg.norm(Hp.to_dense() - F) > 100 * tol * np.linalg.norm(F)
