"""Host-side checks of the C-ABI library (no GPU needed).

* the shared library loads and exports every function ``include/hm.h``
  declares;
* facet geometry and the cluster / block trees computed by the library's C++
  host code agree with the oracle: trees and block lists bit-exactly
  (integers) and the facet geometry bit-exactly (same IEEE operations);
* argument validation returns HM_EINVAL.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import clustering, geometry
from workloads import configs, meshes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hm():
    from paper_2305_06891_amd import hm
    return hm


def test_library_exports_every_declared_function():
    hm = _hm()
    hdr = open(os.path.join(ROOT, "include", "hm.h")).read()
    names = set(re.findall(r"\b(hm_[a-z_0-9]+)\s*\(", hdr))
    assert len(names) >= 25
    for name in sorted(names):
        assert hasattr(hm.lib, name), name
    assert set(hm.EXPORTED) == names
    assert hm.lib.hm_version().startswith(b"hmrad")


def test_facets_match_oracle_geometry():
    hm = _hm()
    for v, f in (meshes.icosphere(2), meshes.cylinder(30, 12, 5, seed=4), meshes.ellipsoid(5, (3, 2, 1))):
        f = meshes.inward(f)
        c, n, a = hm.hm_facets_from_triangles(v, f, orient=1)
        co, no, ao = geometry.facets_from_triangles(v, f)
        # same IEEE operations in the same order on both sides: bit-exact
        assert np.array_equal(c, co) and np.array_equal(n, no) and np.array_equal(a, ao)
        # orientation: automatic mode points the normals into a star-shaped cavity
        c2, n2, _ = hm.hm_facets_from_triangles(v, meshes.inward(f), orient=0)
        assert np.all(np.einsum("ij,ij->i", n2, c2) < 0)


def _tree_case(c, n, a, leaf, eta):
    hm = _hm()
    t = hm.hm_build_cluster_tree(None, c, n, a, leaf, eta)
    st = t.stats()
    d, l = t.blocks()
    root, perm = clustering.build_index_tree(c, leaf)
    od, ol = clustering.build_block_tree(root, eta)
    assert np.array_equal(st["perm"], perm)
    assert st["n_nodes"] == clustering.count_nodes(root)
    assert [tuple(x) for x in d] == od
    assert [tuple(x) for x in l] == ol
    return st


def test_tree_matches_oracle_icosphere_c1():
    cav = configs.c1_icosphere()
    c, n, a = geometry.facets_from_triangles(cav.v, cav.tri)
    st = _tree_case(c, n, a, cav.leaf, cav.eta)
    assert st["n_dense"] == 560 and st["n_lowrank"] == 1376


@pytest.mark.parametrize("leaf,eta", [(64, 1.5), (16, 0.7), (100, 3.0)])
def test_tree_matches_oracle_cylinder_and_ellipsoid(leaf, eta):
    v, f = meshes.cylinder(60, 30, 8, seed=9)
    c, n, a = geometry.facets_from_triangles(v, meshes.inward(f))
    _tree_case(c, n, a, leaf, eta)
    v, f = meshes.ellipsoid(9, (4.0, 2.0, 1.0))
    c, n, a = geometry.facets_from_triangles(v, meshes.inward(f))
    _tree_case(c, n, a, leaf, eta)


def test_tree_matches_oracle_example1_and_example2():
    pts = meshes.line_points(37)
    nrm = np.tile([0.0, 0.0, 1.0], (37, 1))
    _tree_case(pts, nrm, np.ones(37), 1, 1.0)
    _tree_case(pts, nrm, np.ones(37), 3, 0.5)
    c, n, a = meshes.parallel_plates(40)     # Example 2: 3,200 facets, leaf size 128
    _tree_case(c, n, a, 128, 1.0)


def test_tree_full_size_cylinder_c2():
    cav = configs.c2_cylinder()
    c, n, a = geometry.facets_from_triangles(cav.v, cav.tri)
    st = _tree_case(c, n, a, cav.leaf, cav.eta)
    assert st["n_nodes"] == 1023


def test_invalid_arguments_are_rejected():
    hm = _hm()
    c = np.zeros((4, 3))
    c[:, 0] = np.arange(4)
    n = np.tile([0.0, 0.0, 1.0], (4, 1))
    with pytest.raises(hm.HMError) as e:
        hm.hm_build_cluster_tree(None, c, n, np.ones(4), 0, 1.0)
    assert e.value.status == hm.HM_EINVAL
    with pytest.raises(hm.HMError):
        hm.hm_build_cluster_tree(None, c, n, np.array([1.0, 0.0, 1.0, 1.0]), 2, 1.0)
    with pytest.raises(hm.HMError):
        hm.hm_build_cluster_tree(None, c, n, np.ones(4), 2, -1.0)
    bad = c.copy()
    bad[1, 1] = np.nan
    with pytest.raises(hm.HMError):
        hm.hm_build_cluster_tree(None, bad, n, np.ones(4), 2, 1.0)
    v = np.array([[0.0, 0, 0], [1.0, 0, 0], [2.0, 0, 0]])
    with pytest.raises(hm.HMError):
        hm.hm_facets_from_triangles(v, np.array([[0, 1, 2]]))   # degenerate triangle
    with pytest.raises(hm.HMError):
        hm.hm_facets_from_triangles(v, np.array([[0, 1, 5]]))   # index out of range


def test_entry_points_reject_missing_handles():
    # no GPU needed: every entry point checks its handles before any device call
    hm = _hm()
    tree = hm.hm_build_cluster_tree(None, *_small_cloud(), 2, 1.0)
    params = (hm.hm_assembly_params * 1)(hm.hm_assembly_params(1e-6, 16, hm.HM_F32, hm.HM_F32, 0, 0, 0))
    trees = (C.c_void_p * 1)(tree._h)
    out = (C.c_void_p * 1)()
    assert hm.lib.hm_assemble_hmatrix_batched(None, 1, trees, params, out) == hm.HM_EINVAL
    assert hm.lib.hm_matrix_set_tuning(None, None, 64, 0) == hm.HM_EINVAL
    assert hm.lib.hm_matrix_tuning(None, None, None, None) == hm.HM_EINVAL
    assert hm.lib.hm_matrix_set_tuning_phase2(None, None, 4) == hm.HM_EINVAL
    assert hm.lib.hm_matrix_tuning_phase2(None, None, None) == hm.HM_EINVAL
    assert hm.lib.hm_matrix_stats(None, None, None, None, None) == hm.HM_EINVAL
    assert out[0] is None


def _small_cloud():
    c = np.zeros((8, 3))
    c[:, 0] = np.arange(8)
    n = np.tile([0.0, 0.0, 1.0], (8, 1))
    return c, n, np.ones(8)
