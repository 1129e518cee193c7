"""GPU tests of the finite-element coupling (Sec. 3.1-3.4) against the
oracle's dense definition (oracle/fe.py), FP64 H-matrix (ACA 1e-10).

* The radiation load Q = S T^4 of random nodal temperatures: relative L2
  <= 1e-8 (the H approximation, amplified by C^-1, is about 1e-10).
* One implicit Euler step with conduction, radiation and facet sources:
  T^{n+1} within 1e-9 (relative L2) of the oracle's Newton root; the GPU
  Newton-Krylov converges (status OK, at least two corrections).
* The step changes the heat content 1^T M T only by the sources (1^T K = 0
  and 1^T S = 0): to 1e-8 of the source power.
* A uniform temperature without sources stays at rest.

Geometries: an icosphere shell (level 3) and the bench's ellipsoid shell
family (axes 4, 2, 1) at 1,280 facets, 642 nodes each.
"""
import numpy as np
import pytest

from oracle import fe, geometry, viewfactor
from workloads import configs, meshes

from gpu_common import dt, log, rel, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hm():
    from paper_2305_06891_amd import hm as _hm
    return _hm


@pytest.fixture(scope="module")
def ctx(hm):
    return hm.Context(0)


@pytest.fixture(scope="module", params=["icosphere", "ellipsoid"])
def shell(hm, ctx, request):
    if request.param == "icosphere":
        v, f = meshes.icosphere(3)
        f = meshes.inward(f)
    else:
        cav = configs.fe_shell(nu=8)
        v, f = cav.v, cav.tri
    c, n, a = geometry.facets_from_triangles(v, f)
    F = viewfactor.view_factor_matrix(c, n, a)
    eps = np.random.default_rng(21).uniform(0.2, 0.9, a.size)
    cg, ng, ag = hm.hm_facets_from_triangles(v, f, orient=1)
    tree = hm.hm_build_cluster_tree(ctx, cg, ng, ag, 32, 2.0)
    M = hm.hm_assemble_hmatrix(ctx, tree, 1e-10, 256, hm.HM_F64, hm.HM_F64)
    return v, f, a, F, eps, tree, M


K_H, RC_H, DT = 5.0, 2e3, 1.0


def _fe(hm, ctx, shell):
    v, f, a, F, eps, tree, M = shell
    p = hm.fe_params(K_H, RC_H, DT, newton_rtol=1e-12, krylov_rtol=1e-11, pc_rtol=1e-13,
                     solve=hm.solve_params(rtol=1e-13, restart=30, max_iter=600))
    return hm.hm_fe_create(ctx, M, v, f, dt(eps), p)


def test_cavity_load_matches_oracle(hm, ctx, shell):
    import torch
    v, f, a, F, eps, tree, M = shell
    log("case: FE radiation load, shell %d facets %d nodes, FP64, ACA 1e-10" % (a.size, v.shape[0]))
    obj = _fe(hm, ctx, shell)
    T = np.random.default_rng(3).uniform(300.0, 1200.0, v.shape[0])
    Q = to_np(obj.cavity_load(dt(T)))
    torch.cuda.synchronize()
    Mm, Kk, P = fe.surface_p1(v, f, K_H, RC_H)
    S = fe.cavity_operator(P, fe.exchange_matrix(F, eps, a))
    Qo = S @ T**4
    e = rel(Q, Qo)
    log("e(Q) %.2e, sum Q / |Q| %.1e" % (e, abs(Q.sum()) / np.linalg.norm(Q)))
    assert e <= 1e-8


def test_step_matches_oracle_and_keeps_heat(hm, ctx, shell):
    import torch
    v, f, a, F, eps, tree, M = shell
    nn = v.shape[0]
    log("case: FE implicit Euler step, shell %d facets %d nodes, k h %g, rho c h %g, dt %g"
        % (a.size, nn, K_H, RC_H, DT))
    obj = _fe(hm, ctx, shell)
    rng = np.random.default_rng(9)
    T0 = rng.uniform(300.0, 1200.0, nn)
    src = rng.uniform(0.0, 500.0, a.size)
    T1, info = obj.step(dt(T0), dt(src))
    torch.cuda.synchronize()
    T1 = to_np(T1)
    Mm, Kk, P = fe.surface_p1(v, f, K_H, RC_H)
    S = fe.cavity_operator(P, fe.exchange_matrix(F, eps, a))
    fN = fe.nodal_load(f, a, src, nn)
    To, it, _ = fe.newton_step(T0, DT, Mm, Kk, S, fN)
    e = rel(T1, To)
    heat = np.ones(nn) @ Mm @ (T1 - T0) / DT
    log("info %s; oracle Newton %d; e(T) %.2e, |T1 - T0| / |T0| %.2e, heat balance %.2e"
        % (info, int(it[0]), e, rel(T1, T0), abs(heat - fN.sum()) / fN.sum()))
    assert info["status"] == 0 and info["newton"] >= 2
    assert e <= 1e-9
    assert abs(heat - fN.sum()) <= 1e-8 * fN.sum()


def test_uniform_temperature_stays(hm, ctx, shell):
    import torch
    v, f, a, F, eps, tree, M = shell
    obj = _fe(hm, ctx, shell)
    Tu = np.full(v.shape[0], 700.0)
    T1, info = obj.step(dt(Tu))
    torch.cuda.synchronize()
    log("uniform: max |T1 - T0| %.2e, info %s" % (np.abs(to_np(T1) - Tu).max(), info))
    assert np.abs(to_np(T1) - Tu).max() <= 1e-7
