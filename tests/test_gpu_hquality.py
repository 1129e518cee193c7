"""Accuracy of the H-matrix against eps_rel in the form of the paper's
Table 2 (Sec. 6.3): |F - F_eps|_F / |F|_F for eps_rel = 1e-1 ... 1e-6 on
the 13-sphere Fibonacci spiral with fully pivoted ACA (the paper's setting),
GPU-assembled and compared with the oracle's H-matrix of the same
tolerance.

* Each low-rank block stops on the exact residual of eq. (31) and dense
  blocks are exact, so the global ratio is at most eps_rel (the sum of the
  blocks' squared errors is at most eps_rel^2 |F|_F^2).
* The GPU's fully pivoted ACA takes the oracle's steps, so its ratio is
  the oracle's (within 25%: near-equal pivots may be taken in another order
  at loose tolerances).
* Recompressed at the same eps_rel, the ratio is at most 2 eps_rel (the
  ACA error plus the truncation error).

The table is printed; the paper's values on its own meshes are printed
beside it for context only (its ratios are about 0.094-0.097 eps_rel).
"""
import numpy as np
import pytest

from oracle import aca, geometry, viewfactor
from workloads import configs

from gpu_common import full_matrix, log, rel

pytestmark = pytest.mark.gpu

# Table 2 of the paper (its meshes; context, not a target)
PAPER = {1e-1: 9.529e-03, 1e-2: 9.668e-04, 1e-3: 9.416e-05, 1e-4: 9.399e-06, 1e-5: 9.372e-07, 1e-6: 9.415e-08}


@pytest.fixture(scope="module")
def hm():
    from paper_2305_06891_amd import hm as _hm
    return _hm


@pytest.fixture(scope="module")
def ctx(hm):
    return hm.Context(0)


def test_table2_error_against_eps_rel(hm, ctx):
    cav = configs.fibonacci_spiral(nu=4)
    leaf = 32
    log("case: H-matrix error against eps_rel, spiral %d facets, leaf %d, eta 1.5, full pivoting" % (cav.n, leaf))
    c, nr, a = geometry.facets_from_triangles(cav.v, cav.tri)
    F = viewfactor.view_factor_matrix(c, nr, a)
    cg, ng, ag = hm.hm_facets_from_triangles(cav.v, cav.tri, orient=1)
    tree = hm.hm_build_cluster_tree(ctx, cg, ng, ag, leaf, 1.5)
    log("eps_rel   |F-F_H|/|F| GPU   oracle      ratio/eps   recompressed  entries (recompr.)   paper")
    for tol in sorted(PAPER, reverse=True):
        M = hm.hm_assemble_hmatrix(ctx, tree, tol, 256, hm.HM_F64, hm.HM_F64, aca_pivot=1)
        Mr = hm.hm_assemble_hmatrix(ctx, tree, tol, 256, hm.HM_F64, hm.HM_F64, aca_pivot=1, recompress=1)
        e = rel(full_matrix(hm, ctx, M, cav.n), F)
        er = rel(full_matrix(hm, ctx, Mr, cav.n), F)
        eo = rel(aca.build_hmatrix(c, nr, a, leaf, 1.5, tol, pivot="full").to_dense(), F)
        s, sr = M.stats(), Mr.stats()
        ent = s["entries_dense"] + s["entries_lowrank"]
        entr = sr["entries_dense"] + sr["entries_lowrank"]
        log("%-8.0e  %.3e          %.3e   %.3f       %.3e     %d (%d)   %.3e"
            % (tol, e, eo, e / tol, er, ent, entr, PAPER[tol]))
        assert e <= tol and eo <= tol
        assert abs(e - eo) <= 0.25 * eo
        assert er <= 2 * tol and entr <= ent
        M.close()
        Mr.close()
