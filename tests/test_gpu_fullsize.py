"""GPU parity at the benchmark's full sizes, in the configurations bench.py
times (autotuned matrices, the same solve parameters).

* 20,176-facet cylinder, plain FP32 H-solve (ACA 1e-6, GMRES rtol 1e-7):
  J and q against the oracle's dense FP64 LU solution stored in
  ``tests/golden/c2_reference.npz`` (written by
  ``tests/golden/make_c2_reference.py`` from ``oracle/`` only): relative L2
  <= 1e-6 (FP32 Krylov floor ~ cond * 1e-7 plus the ACA error ~3e-7).
* 64-cavity batch (696,072 facets) assembled in one batched call (ACA
  crosses recompressed by truncated SVD at the ACA tolerance), BF16
  factors (dithered rounding) + FP64 refinement to a residual of 1e-7
  (inner FP32 GMRES to 2e-4), all cavities in one batched solve: the
  smallest cavity of
  each type against the dense oracle computed here, and the largest
  ellipsoid (35,280 facets) with an 18k-facet cavity of each type against the
  stored dense oracle solution (relative L2 <= 1e-6);
  every cavity against the batched FP32 solve of the same cavities (both
  within 1e-6 of the exact solution: <= 2e-6 apart); the largest cavity
  (35,280 facets) through the exact radiosity balance on 64 sampled rows
  evaluated by the oracle one row at a time (relative residual <= 1e-5: the
  H approximation error on single rows stays below 10x its global 3e-7);
  the energy balance sum_i A_i q_i ~ 0 on every cavity (exact for the dense
  operator; the ACA error breaks reciprocity at the 1e-6 level).
* Autotuned and fixed phase-1 splits give the same product up to the order
  of partial sums (FP64: 1e-13).
* The smallest and the largest cavity of the batch, solved alone with the
  same matrices and parameters, give the batch's radiosity and flux bit for
  bit (the batch's products run four-wave workgroups, a single cavity's
  eight; every row sum has the same order in both).
"""
import os

import numpy as np
import pytest

from oracle import geometry, radiosity, viewfactor
from workloads import configs

from gpu_common import dt, log, oracle_dense, rel, to_np

pytestmark = pytest.mark.gpu
SIGMA = 5.670374e-8
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def hm():
    from paper_2305_06891_amd import hm as _hm
    return _hm


@pytest.fixture(scope="module")
def ctx(hm):
    return hm.Context(0)


def _tree(hm, ctx, cav):
    c, n, a = hm.hm_facets_from_triangles(cav.v, cav.tri, orient=1)
    return hm.hm_build_cluster_tree(ctx, c, n, a, cav.leaf, cav.eta)


def test_c2_full_size_fp32_matches_golden(hm, ctx):
    import torch
    cav = configs.c2_cylinder()
    log("case: c2 cylinder %d facets, FP32 storage, autotuned, GMRES rtol 1e-7" % cav.n)
    ref = np.load(os.path.join(HERE, "golden", "c2_reference.npz"))
    assert int(ref["n"]) == cav.n
    M = hm.hm_assemble_hmatrix(ctx, _tree(hm, ctx, cav), cav.aca_tol, 256, hm.HM_F32, hm.HM_F32, autotune=1)
    p = hm.solve_params(rtol=1e-7, restart=30, max_iter=300, want_q=1, vec_dtype=hm.HM_F32)
    J, q, info = hm.hm_solve_radiosity(ctx, M, dt(cav.eps), dt(cav.T[:, 0]), SIGMA, p)
    torch.cuda.synchronize()
    eJ, eq = rel(to_np(J), ref["J"]), rel(to_np(q), ref["q"])
    log("c2: iters %d residual %.2e e(J) %.3e e(q) %.3e tuning %s" % (info["iters"], info["rel_residual"], eJ, eq,
                                                                      M.tuning()))
    assert info["status"] == hm.HM_OK
    assert eJ <= 1e-6 and eq <= 1e-6


@pytest.fixture(scope="module")
def c3(hm, ctx):
    import torch
    cavs = configs.c3_batch()
    log("case: c3 batch of %d cavities, %d facets" % (len(cavs), sum(c.n for c in cavs)))
    trees = [_tree(hm, ctx, c) for c in cavs]
    Mx = hm.hm_assemble_hmatrix_batched(ctx, trees, [c.aca_tol for c in cavs], 256, hm.HM_BF16, hm.HM_F32,
                                        keep_f32_copy=1, autotune=1, recompress=1, lowrank_rounding=1)
    M32 = [hm.hm_assemble_hmatrix(ctx, t, c.aca_tol, 256, hm.HM_F32, hm.HM_F32, autotune=1, recompress=1)
           for t, c in zip(trees, cavs)]
    eps = [dt(c.eps) for c in cavs]
    T = [dt(c.T[:, 0]) for c in cavs]
    pmx = hm.solve_params(rtol=1e-7, restart=30, max_iter=400, mixed_precision=1, ir_inner_rtol=2e-4, want_q=1)
    Jx, qx, ix = hm.hm_solve_radiosity_batched(ctx, Mx, eps, T, SIGMA, pmx)
    p32 = hm.solve_params(rtol=1e-7, restart=30, max_iter=400, want_q=1, vec_dtype=hm.HM_F32)
    J3, q3, i3 = hm.hm_solve_radiosity_batched(ctx, M32, eps, T, SIGMA, p32)
    torch.cuda.synchronize()
    # two cavities solved alone with the same matrices and parameters: the
    # batch's products run four-wave workgroups, a single cavity's eight
    alone = {}
    for k in (min(range(len(cavs)), key=lambda i: cavs[i].n), max(range(len(cavs)), key=lambda i: cavs[i].n)):
        Ja, qa, _ = hm.hm_solve_radiosity(ctx, Mx[k], eps[k], T[k], SIGMA, pmx)
        alone[k] = (to_np(Ja), to_np(qa))
    torch.cuda.synchronize()
    return (cavs, [to_np(j) for j in Jx], [to_np(q) for q in qx], ix, [to_np(j) for j in J3], [to_np(q) for q in q3],
            alone)


def test_c3_batch_smallest_of_each_type_match_oracle(c3):
    cavs, Jx, qx, ix, _, _, _ = c3
    assert all(i["status"] == 0 for i in ix)
    picked = {}
    for k, c in enumerate(cavs):
        kind = c.extra["kind"]
        if kind not in picked or c.n < cavs[picked[kind]].n:
            picked[kind] = k
    for kind, k in sorted(picked.items()):
        c = cavs[k]
        _, _, _, F = oracle_dense(c.v, c.tri)
        rad = radiosity.DenseRadiosity(F, c.eps)
        Jo = rad.radiosity(c.T[:, 0])
        qo = rad.flux(c.T[:, 0], Jo)
        eJ, eq = rel(Jx[k], Jo), rel(qx[k], qo)
        log("%s (%d facets): outer %d inner %d e(J) %.3e e(q) %.3e" % (c.name, c.n, ix[k]["outer_iters"],
                                                                       ix[k]["iters"], eJ, eq))
        assert eJ <= 1e-6 and eq <= 1e-6


def test_c3_batch_large_and_mid_cavities_match_golden(c3):
    """The largest ellipsoid (35,280 facets) and an 18,000-18,400-facet
    icosphere, ellipsoid and cylinder of the batch against the oracle's dense
    FP64 LU solution (``tests/golden/c3_reference.npz``, written by
    ``tests/golden/make_c3_reference.py`` from ``oracle/`` only): relative L2
    of J and q <= 1e-6."""
    cavs, Jx, qx, ix, _, _, _ = c3
    ref = np.load(os.path.join(HERE, "golden", "c3_reference.npz"))
    for k in ref["indices"]:
        k = int(k)
        c = cavs[k]
        assert int(ref["n_%d" % k]) == c.n
        eJ, eq = rel(Jx[k], ref["J_%d" % k]), rel(qx[k], ref["q_%d" % k])
        log("%s (%d facets): outer %d inner %d e(J) %.3e e(q) %.3e" % (c.name, c.n, ix[k]["outer_iters"],
                                                                       ix[k]["iters"], eJ, eq))
        assert eJ <= 1e-6 and eq <= 1e-6


def test_c3_batch_mixed_agrees_with_fp32_and_conserves_energy(c3):
    cavs, Jx, qx, ix, J3, q3, _ = c3
    worst_J = worst_q = worst_e = 0.0
    for k, c in enumerate(cavs):
        worst_J = max(worst_J, rel(Jx[k], J3[k]))
        worst_q = max(worst_q, rel(qx[k], q3[k]))
        _, _, a = geometry.facets_from_triangles(c.v, c.tri)
        worst_e = max(worst_e, abs(float(a @ qx[k])) / float(a @ np.abs(qx[k])))
    log("c3: mixed vs FP32 worst e(J) %.2e e(q) %.2e; energy imbalance worst %.2e" % (worst_J, worst_q, worst_e))
    assert worst_J <= 2e-6 and worst_q <= 2e-6
    assert worst_e <= 1e-5


def test_c3_largest_cavity_sampled_rows_satisfy_radiosity_balance(c3):
    cavs, Jx, _, _, _, _, _ = c3
    k = max(range(len(cavs)), key=lambda i: cavs[i].n)
    c = cavs[k]
    cc, nn, a = geometry.facets_from_triangles(c.v, c.tri)
    rows = np.random.default_rng(7).choice(c.n, 64, replace=False)
    Frows = viewfactor.view_factor_rows(cc, nn, a, rows)
    b = SIGMA * c.eps[rows] * c.T[rows, 0] ** 4
    J = Jx[k]
    r = b - J[rows] + (1.0 - c.eps[rows]) * (Frows @ J)
    e = float(np.linalg.norm(r) / np.linalg.norm(b))
    log("%s (%d facets): sampled-row residual of the exact balance %.2e" % (c.name, c.n, e))
    assert e <= 1e-5


def test_c3_batch_members_equal_their_alone_solves(c3):
    cavs, Jx, qx, _, _, _, alone = c3
    for k, (Ja, qa) in alone.items():
        log("%s (%d facets): batched vs alone max |dJ| %.1e" % (cavs[k].name, cavs[k].n, float(np.max(np.abs(Jx[k] - Ja)))))
        assert np.array_equal(Jx[k], Ja) and np.array_equal(qx[k], qa)


@pytest.mark.parametrize("width", [1, 16])
def test_autotuned_and_fixed_splits_give_the_same_product(hm, ctx, width):
    """The split tuned on products of 1 or 16 columns changes only the order
    of partial sums (16: FP32 storage, so the tuning times matrix-core
    products; compared with FP64 vectors on the FP32 entries)."""
    import torch
    cav = configs.c2_cylinder()
    t = _tree(hm, ctx, cav)
    st = hm.HM_F64 if width == 1 else hm.HM_F32
    log("case: c2 product, fixed vs phase-1 split autotuned on %d-column products" % width)
    Ma = hm.hm_assemble_hmatrix(ctx, t, cav.aca_tol, 256, st, st, autotune=width)
    Mf = hm.hm_assemble_hmatrix(ctx, t, cav.aca_tol, 256, st, st, autotune=0)
    x = torch.as_tensor(np.random.default_rng(3).uniform(0.5, 1.5, (cav.n, 16)), device="cuda").T.contiguous().T
    ya = torch.zeros_like(x)
    yf = torch.zeros_like(x)
    hm.hm_hmatvec(ctx, Ma, x, ya)
    hm.hm_hmatvec(ctx, Mf, x, yf)
    e = rel(to_np(ya), to_np(yf))
    log("tuning %s vs %s: rel diff %.2e" % (Ma.tuning(), Mf.tuning(), e))
    assert Mf.tuning()["p1_us"] == 0.0 and Ma.tuning()["p1_us"] > 0.0
    assert e <= 1e-13
    with pytest.raises(Exception):
        hm.hm_assemble_hmatrix(ctx, t, cav.aca_tol, 256, st, st, autotune=17)


def test_batched_profile_counts_the_bytes_of_every_matrix(hm, ctx):
    cavs = configs.c3_batch(count=3)
    log("case: profile entry over 3 cavities")
    Ms = [hm.hm_assemble_hmatrix(ctx, _tree(hm, ctx, c), c.aca_tol, 256, hm.HM_BF16, hm.HM_F32, keep_f32_copy=1)
          for c in cavs]
    each = [hm.hm_hmatvec_profile(ctx, M, 1, hm.HM_F32, reps=2, flush_bytes=0) for M in Ms]
    allp = hm.hm_hmatvec_profile(ctx, Ms, 1, hm.HM_F32, reps=2, flush_bytes=0)
    assert allp["bytes_phase1"] == sum(e["bytes_phase1"] for e in each)
    assert allp["bytes_phase2"] == sum(e["bytes_phase2"] for e in each)
    assert allp["ms_phase2"] > 0 and allp["ms_total"] >= allp["ms_phase2"]
