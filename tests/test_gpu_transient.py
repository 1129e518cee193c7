"""GPU tests of the lumped transient (analogue of Sec. 3.3) with 16
scenarios per product (the matrix-core path), in the configuration the
bench times: FP32 factors (recompressed ACA crosses, product split tuned on
16-column products) and FP32 Krylov vectors (rtol 1e-7), FP64 flux and
Newton update, Newton tolerance 1e-9.

* 18,000-facet member (geodesic frequency 30) of the (4, 2, 1) ellipsoid
  family, 100 steps of 1 s: temperatures after steps 1 and 100 of scenarios
  0-3 against the oracle's dense-LU integration stored in
  ``tests/golden/c4_reference.npz`` (written by
  ``tests/golden/make_c4_reference.py`` from ``oracle/`` only):
  e(T) <= 1e-6 (per-step flux error ~1e-6 of |q| times dt / m_c, summed
  over 100 steps, is ~1e-7 of T).
* 200,000-facet ellipsoid, 2 steps: the energy balance of every step and
  scenario, sum_i A_i (m_c (T_i^{n+1} - T_i^n) / dt - s_i) = sum_i A_i q_i,
  vanishes for the dense operator (reciprocity) and up to the ACA error
  (1e-6) and the Newton tolerance here: relative to sum_i A_i |m_c dT_i/dt|
  it stays <= 1e-5.  Step 1 of scenarios 0-1 against the oracle's large-n
  mode (matrix-free FP64 products, GMRES to 1e-12; stored as the FP32
  increments T^1 - T^0 in ``tests/golden/c4_fullsize_reference.npz``,
  written by ``tests/golden/make_c4_fullsize_reference.py`` from
  ``oracle/`` only): e(T) <= 1e-6.
"""
import os

import numpy as np
import pytest

from oracle import geometry
from workloads import configs

from gpu_common import log, to_np

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
SIGMA = 5.670374e-8


@pytest.fixture(scope="module")
def hm():
    from paper_2305_06891_amd import hm as _hm
    return _hm


@pytest.fixture(scope="module")
def ctx(hm):
    return hm.Context(0)


def _setup(hm, ctx, cav):
    import torch
    c, n, a = hm.hm_facets_from_triangles(cav.v, cav.tri, orient=1)
    tree = hm.hm_build_cluster_tree(ctx, c, n, a, cav.leaf, cav.eta)
    M = hm.hm_assemble_hmatrix(ctx, tree, cav.aca_tol, 256, hm.HM_F32, hm.HM_F32, autotune=16, recompress=1)
    eps = torch.as_tensor(cav.eps, device="cuda")
    T = torch.as_tensor(np.asfortranarray(cav.T), device="cuda")
    src = torch.as_tensor(np.asfortranarray(cav.extra["source"]), device="cuda")
    return M, eps, T, src


def _params(hm):
    return hm.solve_params(rtol=1e-7, restart=30, max_iter=400, want_q=1, vec_dtype=hm.HM_F32)


def test_transient_family_member_matches_oracle_over_100_steps(hm, ctx):
    ref = np.load(os.path.join(HERE, "golden", "c4_reference.npz"))
    cav = configs.c4_ellipsoid(nu=int(ref["nu"]), scenarios=16)
    assert cav.n == int(ref["n"])
    log("case: transient ellipsoid %d facets, 16 scenarios, 100 steps" % cav.n)
    M, eps, T, src = _setup(hm, ctx, cav)
    T, i1 = hm.hm_transient_run(ctx, M, eps, T, src, mc=cav.extra["mc"], dt=cav.extra["dt"], steps=1,
                                newton_rtol=1e-9, params=_params(hm))
    T1 = to_np(T)[:, :4].copy()
    T, i2 = hm.hm_transient_run(ctx, M, eps, T, src, mc=cav.extra["mc"], dt=cav.extra["dt"], steps=99,
                                newton_rtol=1e-9, params=_params(hm))
    T100 = to_np(T)[:, :4]
    e1 = max(np.linalg.norm(T1[:, s] - ref["T1"][:, s]) / np.linalg.norm(ref["T1"][:, s]) for s in range(4))
    e100 = max(np.linalg.norm(T100[:, s] - ref["T100"][:, s]) / np.linalg.norm(ref["T100"][:, s]) for s in range(4))
    log("newton %d + %d (max %d per step), %.2f s; e(T) step 1 %.2e, step 100 %.2e"
        % (i1["newton_total"], i2["newton_total"], max(i1["newton_max"], i2["newton_max"]),
           i1["seconds"] + i2["seconds"], e1, e100))
    assert i2["steps_done"] == 99
    assert e1 <= 1e-6 and e100 <= 1e-6


def test_transient_full_size_energy_balance(hm, ctx):
    cav = configs.c4_ellipsoid()
    log("case: transient ellipsoid %d facets, 16 scenarios, 2 steps" % cav.n)
    M, eps, T, src = _setup(hm, ctx, cav)
    T0 = to_np(T).copy()
    T, i1 = hm.hm_transient_run(ctx, M, eps, T, src, mc=cav.extra["mc"], dt=cav.extra["dt"], steps=1,
                                newton_rtol=1e-9, params=_params(hm))
    T1 = to_np(T).copy()
    T, i2 = hm.hm_transient_run(ctx, M, eps, T, src, mc=cav.extra["mc"], dt=cav.extra["dt"], steps=1,
                                newton_rtol=1e-9, params=_params(hm))
    T2 = to_np(T)
    _, _, a = geometry.facets_from_triangles(cav.v, cav.tri)
    mc, dt = cav.extra["mc"], cav.extra["dt"]
    s = cav.extra["source"]
    worst = 0.0
    for Ta, Tb in ((T0, T1), (T1, T2)):
        rate = mc * (Tb - Ta) / dt
        imb = np.abs(a @ (rate - s)) / (a @ np.abs(rate))
        worst = max(worst, float(np.max(imb)))
    log("newton %d + %d, residual %.1e; worst energy imbalance %.2e" % (i1["newton_total"], i2["newton_total"],
                                                                      max(i1["max_rel_residual"],
                                                                          i2["max_rel_residual"]), worst))
    assert worst <= 1e-5
    ref_path = os.path.join(HERE, "golden", "c4_fullsize_reference.npz")
    ref = np.load(ref_path)
    assert int(ref["n"]) == cav.n
    for sc in range(int(ref["scenarios"])):
        T1o = T0[:, sc] + ref["dT1"][:, sc].astype(np.float64)
        e = np.linalg.norm(T1[:, sc] - T1o) / np.linalg.norm(T1o)
        ed = np.linalg.norm((T1[:, sc] - T0[:, sc]) - ref["dT1"][:, sc]) / np.linalg.norm(ref["dT1"][:, sc])
        log("scenario %d: e(T) step 1 %.2e (increment %.2e)" % (sc, e, ed))
        assert e <= 1e-6
