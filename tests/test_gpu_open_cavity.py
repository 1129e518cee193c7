"""GPU tests of the non-convex, open 13-sphere spiral (Sec. 6): isolated
facets (zero rows of F), fully pivoted ACA, the closed-cavity row scaling of
eqs. (32)-(34) and the open-cavity ambient exchange of eq. (35).  Every
matrix here is compressed with full pivoting (partial pivoting misses parts
of this geometry's blocks, see the second test).

* Fully pivoted ACA (2,340 facets, FP64, ACA 1e-8, with and without
  recompression): ranks sum to the oracle's, products within 1e-12 of the
  oracle's H-matrix, |F_H - F| / |F| <= 1e-8 (partial pivoting: above 1e-6).

* FP64 H-matrix (leaf 32, eta 1.5, ACA 1e-8) of the 4,160-facet spiral:
  |F_H - F| / |F| <= 1e-8 with about 8% zero rows; open-cavity J and q
  against the dense oracle with the same ambient term: relative L2 <= 1e-7
  (H error ~1e-8 times cond); every isolated facet has J = eps sigma T^4 and
  q = -sigma (T^4 - T_amb^4) to 1e-12.
* The same spiral treated as closed (the paper's experiment): rows with a
  clamped sum in (0, 1) rescaled, zero rows left alone; J and q against the
  oracle's scaled dense system: <= 1e-7.
* BF16 factors + FP64 refinement (leaf 64, eta 1.5, ACA 1e-6, the bench's
  solver settings) on the 9,360-facet spiral, open: J and q <= 1e-6.
* Two implicit Euler steps of the open FP64 transient (2,340 facets, four
  scenarios) against the oracle's: e(T) <= 1e-9.
* Fully pivoted ACA on sphere-to-sphere blocks of 1.6 M entries (16,640
  facets, the sliced passes for blocks of 262,144 entries and more): F_H x on
  sampled rows against the oracle's rows of F times x, <= 1e-5.
"""
import numpy as np
import pytest

from oracle import geometry, radiosity, transient, viewfactor
from workloads import configs

from gpu_common import dt, full_matrix, log, rel, to_np

pytestmark = pytest.mark.gpu
SIGMA = 5.670374e-8


@pytest.fixture(scope="module")
def hm():
    from paper_2305_06891_amd import hm as _hm
    return _hm


@pytest.fixture(scope="module")
def ctx(hm):
    return hm.Context(0)


def _dense(cav):
    c, n, a = geometry.facets_from_triangles(cav.v, cav.tri)
    return a, viewfactor.view_factor_matrix(c, n, a)


def _matrix(hm, ctx, cav, leaf, tol, lr, dense, keep=0, closed=0, pivot=1, recompress=0):
    c, n, a = hm.hm_facets_from_triangles(cav.v, cav.tri, orient=1)
    tree = hm.hm_build_cluster_tree(ctx, c, n, a, leaf, 1.5)
    return hm.hm_assemble_hmatrix(ctx, tree, tol, 256, lr, dense, keep, closed, aca_pivot=pivot,
                                  recompress=recompress)


def test_spiral_open_cavity_fp64(hm, ctx):
    import torch
    cav = configs.fibonacci_spiral(nu=4)
    T_amb = cav.extra["T_amb"]
    log("case: open spiral %d facets, FP64, leaf 32, ACA 1e-8, T_amb %g" % (cav.n, T_amb))
    M = _matrix(hm, ctx, cav, 32, 1e-8, hm.HM_F64, hm.HM_F64)
    _, F = _dense(cav)
    FH = full_matrix(hm, ctx, M, cav.n)
    eF = rel(FH, F)
    iso = ~np.any(F != 0.0, axis=1)
    assert np.all(FH[iso] == 0.0)
    T = cav.T[:, 0]
    p = hm.solve_params(rtol=1e-12, open_cavity=1, ambient_temperature=T_amb)
    J, q, info = hm.hm_solve_radiosity(ctx, M, dt(cav.eps), dt(T), SIGMA, p)
    torch.cuda.synchronize()
    J, q = to_np(J), to_np(q)
    rad = radiosity.DenseRadiosity(F, cav.eps)
    Jo = rad.radiosity(T)
    qo = rad.flux(T, Jo, T_amb=T_amb)
    eJ, eq = rel(J, Jo), rel(q, qo)
    qi = -SIGMA * (T[iso] ** 4 - T_amb**4)
    ei = float(np.max(np.abs(q[iso] - qi)) / (SIGMA * np.max(T) ** 4))
    eJi = float(np.max(np.abs(J[iso] - cav.eps[iso] * SIGMA * T[iso] ** 4) / (cav.eps[iso] * SIGMA * T[iso] ** 4)))
    log("|F_H - F| %.2e, %d isolated facets (%.1f%%), iters %d, e(J) %.2e e(q) %.2e; isolated: J %.1e q %.1e"
        % (eF, iso.sum(), 100 * iso.mean(), info["iters"], eJ, eq, eJi, ei))
    assert eF <= 1e-8 and iso.mean() > 0.05
    assert info["status"] == hm.HM_OK
    assert eJ <= 1e-7 and eq <= 1e-7
    assert ei <= 1e-12 and eJi <= 1e-12


@pytest.mark.parametrize("recompress", [0, 1])
def test_spiral_full_pivot_aca_matches_oracle(hm, ctx, recompress):
    """Fully pivoted ACA (the paper's) on the GPU takes the oracle's pivots
    (the same FP64 entries and updates): ranks sum to the oracle's and the
    products agree to rounding; every block meets eq. (31), so the global
    error is within the tolerance, where partial pivoting is 2e-4 off."""
    from oracle import aca
    cav = configs.fibonacci_spiral(nu=3)
    tol = 1e-8
    log("case: full-pivot ACA on the spiral, %d facets, tol %g, recompress %d" % (cav.n, tol, recompress))
    M = _matrix(hm, ctx, cav, 32, tol, hm.HM_F64, hm.HM_F64, pivot=1, recompress=recompress)
    Mp = _matrix(hm, ctx, cav, 32, tol, hm.HM_F64, hm.HM_F64, pivot=0)
    c, n, a = geometry.facets_from_triangles(cav.v, cav.tri)
    F = viewfactor.view_factor_matrix(c, n, a)
    Ho = aca.build_hmatrix(c, n, a, 32, 1.5, tol, pivot="full", recompress_tol=tol if recompress else None)
    FH = full_matrix(hm, ctx, M, cav.n)
    FHp = full_matrix(hm, ctx, Mp, cav.n)
    st = M.stats()
    ro = sum(b[4].shape[1] for b in Ho.lowrank)
    d, e, ep = rel(FH, Ho.to_dense()), rel(FH, F), rel(FHp, F)
    log("rank sum %d (oracle %d), fallbacks %d, |F_H - F_H,oracle| %.2e, |F_H - F| %.2e (partial pivoting %.2e)"
        % (st["rank_sum"], ro, st["n_fallback"], d, e, ep))
    assert st["rank_sum"] == ro
    assert d <= 1e-12
    assert e <= tol and ep > 100 * tol


def test_spiral_closed_treatment_fp64(hm, ctx):
    import torch
    cav = configs.fibonacci_spiral(nu=4)
    log("case: spiral %d facets treated as closed (eqs. (32)-(34)), FP64" % cav.n)
    M = _matrix(hm, ctx, cav, 32, 1e-8, hm.HM_F64, hm.HM_F64, closed=1)
    _, F = _dense(cav)
    Fs = viewfactor.closed_cavity_scaling(F)
    T = cav.T[:, 0]
    J, q, info = hm.hm_solve_radiosity(ctx, M, dt(cav.eps), dt(T), SIGMA, hm.solve_params(rtol=1e-12))
    torch.cuda.synchronize()
    rad = radiosity.DenseRadiosity(Fs, cav.eps)
    Jo = rad.radiosity(T)
    qo = rad.flux(T, Jo)
    eJ, eq = rel(to_np(J), Jo), rel(to_np(q), qo)
    log("iters %d, e(J) %.2e e(q) %.2e" % (info["iters"], eJ, eq))
    assert eJ <= 1e-7 and eq <= 1e-7


def test_spiral_open_cavity_mixed_precision(hm, ctx):
    import torch
    cav = configs.fibonacci_spiral(nu=6)
    T_amb = cav.extra["T_amb"]
    rng = np.random.default_rng(61)
    T = np.where(cav.extra["sphere"] == 0, 1000.0, 300.0)[:, None] + rng.uniform(0.0, 200.0, (cav.n, 2))
    log("case: open spiral %d facets, BF16 + refinement, leaf 64, ACA 1e-6, 2 columns" % cav.n)
    M = _matrix(hm, ctx, cav, 64, 1e-6, hm.HM_BF16, hm.HM_F32, keep=1)
    p = hm.solve_params(rtol=1e-7, restart=30, max_iter=400, mixed_precision=1, ir_inner_rtol=3e-3, want_q=1,
                        open_cavity=1, ambient_temperature=T_amb)
    Td = torch.as_tensor(np.asfortranarray(T), device="cuda")
    J, q, info = hm.hm_solve_radiosity(ctx, M, dt(cav.eps), Td, SIGMA, p)
    torch.cuda.synchronize()
    _, F = _dense(cav)
    rad = radiosity.DenseRadiosity(F, cav.eps)
    Jo = rad.radiosity(T)
    qo = rad.flux(T, Jo, T_amb=T_amb)
    eJ = radiosity.relative_l2(to_np(J), Jo)
    eq = radiosity.relative_l2(to_np(q), qo)
    log("outer %d inner %d, e(J) %s e(q) %s" % (info["outer_iters"], info["iters"], eJ, eq))
    assert np.all(eJ <= 1e-6) and np.all(eq <= 1e-6)


def test_spiral_open_transient_fp64(hm, ctx):
    import torch
    cav = configs.fibonacci_spiral(nu=3)
    T_amb = cav.extra["T_amb"]
    rng = np.random.default_rng(62)
    T0 = cav.T[:, 0][:, None] + rng.uniform(0.0, 100.0, (cav.n, 4))
    src = rng.uniform(0.0, 500.0, (cav.n, 4))
    log("case: open spiral transient %d facets, 4 scenarios, 2 steps, FP64" % cav.n)
    M = _matrix(hm, ctx, cav, 32, 1e-10, hm.HM_F64, hm.HM_F64)
    Td = torch.as_tensor(np.asfortranarray(T0), device="cuda")
    Sd = torch.as_tensor(np.asfortranarray(src), device="cuda")
    sp = hm.solve_params(rtol=1e-12, open_cavity=1, ambient_temperature=T_amb)
    Td, info = hm.hm_transient_run(ctx, M, dt(cav.eps), Td, Sd, mc=1e4, dt=1.0, steps=2, newton_rtol=1e-12,
                                   params=sp)
    torch.cuda.synchronize()
    _, F = _dense(cav)
    rad = radiosity.DenseRadiosity(F, cav.eps)
    To = T0
    for _ in range(2):
        To, _, _ = transient.newton_step(rad, To, src, 1e4, 1.0, tol=1e-12, T_amb=T_amb)
    e = float(np.max(radiosity.relative_l2(to_np(Td), To)))
    ed = float(np.max(radiosity.relative_l2(to_np(Td) - T0, To - T0)))
    log("newton %d, e(T) %.2e (of the change %.2e)" % (info["newton_total"], e, ed))
    assert e <= 1e-9 and ed <= 1e-7


def test_spiral_full_pivot_large_blocks(hm, ctx):
    """Fully pivoted ACA on large blocks: on the frequency-8 spiral (1,280
    facets per sphere) the sphere-to-sphere blocks hold 1.6 M entries, and
    blocks of 262,144 entries and more run their residual passes in slices
    over many workgroups.
    F_H x on 64 sampled rows against the oracle's rows of F (eq. (10)) times
    x: within 1e-5 of their norm at ACA 1e-6 (eq. (31) bounds each block's
    error by 1e-6 of its norm)."""
    cav = configs.fibonacci_spiral(nu=8)
    n = cav.n
    log("case: full-pivot ACA with sliced passes over large blocks, spiral %d facets, FP64, ACA 1e-6" % n)
    M = _matrix(hm, ctx, cav, 64, 1e-6, hm.HM_F64, hm.HM_F64, pivot=1)
    st = M.stats()
    x = np.random.default_rng(81).uniform(0.5, 1.5, n)
    y = to_np(hm.hm_hmatvec(ctx, M, dt(x), dt(np.zeros(n))))
    rows = np.sort(np.random.default_rng(82).choice(n, 64, replace=False))
    c, nr, a = geometry.facets_from_triangles(cav.v, cav.tri)
    yo = viewfactor.matvec_rows(c, nr, a, rows, x)
    e = rel(y[rows], yo)
    log("low-rank blocks %d, rank sum %d, max rank %d; sampled rows of F_H x vs the oracle: %.2e"
        % (st["n_lowrank_blocks"], st["rank_sum"], st["max_rank"], e))
    assert st["n_lowrank_blocks"] > 0
    assert e <= 1e-5
