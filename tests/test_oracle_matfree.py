"""Pins of the oracle's large-n mode (``oracle/matfree.py``, CPU only).

The matrix-free product evaluates the same centroid-rule entries as the
dense oracle (which the closed forms in ``test_oracle_pins.py`` pin), so:

* its products equal the dense matrix's on an ellipsoid and on a jittered
  cylinder (back-facing pairs present) to summation order;
* its GMRES solution equals the closed-form solution of the projected-sphere
  cavity (sphere points with radial normals, where every entry is
  ``A_j / (4 pi R^2)``) and the dense LU solution, J and the eq. (12) flux;
* one implicit Euler step of the lumped transient taken with it equals the
  step taken with the dense LU oracle.
"""
import numpy as np

from oracle import closed_forms, geometry, matfree, radiosity, transient, viewfactor
from workloads import meshes


def _facets(v, f):
    return geometry.facets_from_triangles(v, f)


def test_matrix_free_product_equals_dense():
    for v, f in (meshes.ellipsoid(9, (3.0, 2.0, 1.0)), meshes.cylinder(24, 16, 4, 1.0, 4.0, 0.05, seed=1)):
        f = meshes.inward(f)
        c, n, a = _facets(v, f)
        F = viewfactor.view_factor_matrix(c, n, a)
        mf = matfree.MatrixFreeF(c, n, a)
        X = np.random.default_rng(3).uniform(-1.0, 2.0, (a.size, 5))
        Yd, Ym = F @ X, mf @ X
        assert np.max(np.abs(Ym - Yd)) <= 1e-13 * np.max(np.abs(Yd))
        assert np.allclose(mf @ X[:, 0], Yd[:, 0], rtol=0, atol=1e-13 * np.max(np.abs(Yd)))


def test_matrix_free_gmres_matches_projected_sphere_closed_form():
    p, nr, w = meshes.projected_sphere_points(3, radius=1.3, seed=7)
    rng = np.random.default_rng(8)
    eps = rng.uniform(0.1, 0.9, w.size)
    T = rng.uniform(300.0, 1500.0, w.size)
    rad = matfree.MatrixFreeRadiosity(p, nr, w, eps, rtol=1e-13)
    J = rad.radiosity(T)
    qc, Jc = closed_forms.sphere_points_flux(w, eps, T, 1.3)
    assert np.linalg.norm(J - Jc) <= 1e-12 * np.linalg.norm(Jc)
    q = rad.flux(T, J)
    assert np.linalg.norm(q - qc) <= 1e-10 * np.linalg.norm(radiosity.emission(eps, T))


def test_matrix_free_solve_and_flux_equal_dense_lu():
    v, f = meshes.cylinder(24, 16, 4, 1.0, 4.0, 0.05, seed=1)
    f = meshes.inward(f)
    c, n, a = _facets(v, f)
    rng = np.random.default_rng(9)
    eps = rng.uniform(0.1, 0.9, a.size)
    T = rng.uniform(300.0, 1500.0, (a.size, 3))
    d = radiosity.DenseRadiosity(viewfactor.view_factor_matrix(c, n, a), eps)
    m = matfree.MatrixFreeRadiosity(c, n, a, eps, rtol=1e-13)
    Jd, Jm = d.radiosity(T), m.radiosity(T)
    assert np.all(radiosity.relative_l2(Jm, Jd) <= 1e-12)
    assert np.all(radiosity.relative_l2(m.flux(T, Jm), d.flux(T, Jd)) <= 1e-11)
    assert np.linalg.norm(m.g - d.g) <= 1e-12 * np.linalg.norm(d.g)


def test_matrix_free_transient_step_equals_dense():
    v, f = meshes.ellipsoid(6, (4.0, 2.0, 1.0))
    f = meshes.inward(f)
    c, n, a = _facets(v, f)
    rng = np.random.default_rng(10)
    eps = np.full(a.size, 0.8)
    T0 = rng.uniform(300.0, 1000.0, (a.size, 2))
    src = rng.uniform(0.0, 500.0, (a.size, 2))
    d = radiosity.DenseRadiosity(viewfactor.view_factor_matrix(c, n, a), eps)
    m = matfree.MatrixFreeRadiosity(c, n, a, eps, rtol=1e-13)
    Td, _, _ = transient.newton_step(d, T0, src, 1e4, 1.0, tol=1e-12)
    Tm, _, _ = transient.newton_step(m, T0, src, 1e4, 1.0, tol=1e-12)
    assert np.all(radiosity.relative_l2(Tm - T0, Td - T0) <= 1e-9)
