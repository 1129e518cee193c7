"""Pins of the oracle's hierarchical block LU (Sec. 5.1) and its
substitutions (Sec. 5.2), CPU only.

* With a tolerance below rounding every block stays exact: the H-LU is the
  dense LU without pivoting (L U = C to rounding) and its solutions are the
  dense solver's.
* At eps_rel = 1e-6 the factors reproduce C (|L U - C| <= eps_rel |C|), the
  solutions are within 10 eps_rel of the dense ones, and the factors keep
  the low-rank structure (fewer stored entries than n^2, Sec. 5.1's claim).
* The four steps hold at the top level: L11 U11 = C11, L11 U12 = C12,
  L21 U11 = C21, L21 U12 + L22 U22 = C22.
* Leaving out the Schur complement update of step 4, or the backward
  substitution of step 3, breaks L U = C (planted mistakes).
"""
import numpy as np
import pytest

from oracle import geometry, hlu, radiosity, viewfactor
from workloads import meshes


@pytest.fixture(scope="module")
def cavity():
    v, f = meshes.ellipsoid(8, (3.0, 2.0, 1.0))
    f = meshes.inward(f)
    c, n, a = geometry.facets_from_triangles(v, f)
    eps = np.random.default_rng(1).uniform(0.1, 0.9, a.size)
    C = radiosity.reflection_matrix(viewfactor.view_factor_matrix(c, n, a), eps)
    return c, n, a, eps, C


def _factor(cavity, tol, **kw):
    c, n, a, eps, C = cavity
    root, perm = hlu.build_reflection(c, n, a, eps, 32, 1.5, tol, **kw)
    Cp = C[np.ix_(perm, perm)]
    return root, perm, Cp


def test_exact_tolerance_gives_the_dense_lu(cavity):
    root, perm, Cp = _factor(cavity, 1e-15)
    hlu.factorize(root, 1e-15)
    L, U = hlu.lower_upper_dense(root)
    assert np.linalg.norm(L @ U - Cp) <= 1e-14 * np.linalg.norm(Cp)
    b = np.random.default_rng(2).uniform(size=(Cp.shape[0], 3))
    x = hlu.solve(root, b)
    xe = np.linalg.solve(Cp, b)
    assert np.linalg.norm(x - xe) <= 1e-13 * np.linalg.norm(xe)


def test_tolerance_bounds_factor_and_solution_errors(cavity):
    tol = 1e-6
    root, perm, Cp = _factor(cavity, tol)
    top = [[hlu.to_dense(root.ch[i][j]) for j in range(2)] for i in range(2)]
    hlu.factorize(root, tol)
    L, U = hlu.lower_upper_dense(root)
    assert np.linalg.norm(L @ U - Cp) <= tol * np.linalg.norm(Cp)
    b = np.random.default_rng(3).uniform(size=Cp.shape[0])
    x = hlu.solve(root, b)
    xe = np.linalg.solve(Cp, b)
    assert np.linalg.norm(x - xe) <= 10 * tol * np.linalg.norm(xe)
    n = Cp.shape[0]
    assert hlu.stored_entries(root) < 0.8 * n * n and hlu.max_rank(root) > 0
    # the four steps at the top level
    m0 = root.ch[0][0].m
    L11, L21, L22 = L[:m0, :m0], L[m0:, :m0], L[m0:, m0:]
    U11, U12, U22 = U[:m0, :m0], U[:m0, m0:], U[m0:, m0:]
    nc = np.linalg.norm(Cp)
    assert np.linalg.norm(L11 @ U11 - top[0][0]) <= tol * nc
    assert np.linalg.norm(L11 @ U12 - top[0][1]) <= tol * nc
    assert np.linalg.norm(L21 @ U11 - top[1][0]) <= tol * nc
    assert np.linalg.norm(L21 @ U12 + L22 @ U22 - top[1][1]) <= tol * nc


def test_planted_mistakes_break_the_factorisation(cavity, monkeypatch):
    tol = 1e-8
    for name in ("no_schur", "no_step3"):
        root, perm, Cp = _factor(cavity, tol)
        orig_gemm, orig_up = hlu.gemm, hlu.solve_upper_block

        def factorize_mutant(A, t, name=name):
            if A.kind == "dense":
                A.D = hlu._dense_lu_nopivot(A.D)
                return
            factorize_mutant(A.ch[0][0], t)
            hlu.solve_lower_block(A.ch[0][0], A.ch[0][1], t)
            if name != "no_step3":
                hlu.solve_upper_block(A.ch[0][0], A.ch[1][0], t)
            if name != "no_schur":
                hlu.gemm(A.ch[1][1], -1.0, A.ch[1][0], A.ch[0][1], t)
            factorize_mutant(A.ch[1][1], t)

        factorize_mutant(root, tol)
        L, U = hlu.lower_upper_dense(root)
        assert np.linalg.norm(L @ U - Cp) > 1e-4 * np.linalg.norm(Cp), name
