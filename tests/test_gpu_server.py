"""GPU tests of the serving loop (continuous batching, HBM-budget admission).

* Each request gives the same radiosity and flux alone and in a mix with
  requests on other cavities submitted together (the batched kernels reduce
  every row and every system in a fixed order that does not depend on the
  other members of a batch): relative difference <= 1e-12.
* Results agree with the dense FP64 oracle within 1e-6 (BF16 factors, FP64
  refinement to a residual of 1e-9, ACA 1e-8).
* A budget too small for all cavities forces evictions and re-assembly, and
  results stay the same.
* Cold start: requests on cavities that are not resident, all submitted at
  once, are assembled on the server's assembler thread while the requests
  whose cavity is ready already run; every result equals the one of the same
  request served alone (bit for bit up to 1e-12).
* Requests of 9-16 columns (slots 16 wide: both products of the refinement,
  FP32 inner and FP64 residual, run on the matrix cores, over compositions
  of several cavities with inactive slots) meet the same two bars.
"""
import time

import numpy as np
import pytest

from oracle import radiosity
from workloads import meshes

from gpu_common import log, oracle_dense, rel

pytestmark = pytest.mark.gpu
SIGMA = 5.670374e-8


@pytest.fixture(scope="module")
def hm():
    from paper_2305_06891_amd import hm as _hm
    return _hm


@pytest.fixture(scope="module")
def ctx(hm):
    return hm.Context(0)


def _cavities():
    out = []
    for k, (v, f) in enumerate((meshes.icosphere(2), meshes.ellipsoid(7, (2.0, 1.5, 1.0)),
                                meshes.cylinder(30, 16, 5, seed=2))):
        f = meshes.inward(f)
        rng = np.random.default_rng(700 + k)
        out.append((v, f, rng.uniform(0.1, 0.9, f.shape[0])))
    return out


def _wait(srv, tickets, timeout=60.0):
    res = {}
    t0 = time.time()
    while len(res) < len(tickets):
        for tk, shape in tickets:
            if tk in res:
                continue
            r = srv.poll(tk, shape)
            if r is not None:
                res[tk] = r
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.002)
    return res


def _server(hm, ctx, cavs, budget, max_rhs=8):
    p = hm.solve_params(rtol=1e-9, restart=30, max_iter=400, mixed_precision=1, ir_inner_rtol=1e-3, want_q=1)
    srv = hm.Server(ctx, hbm_budget_bytes=budget, max_active=16, max_rhs_per_slot=max_rhs, params=p)
    for cid, (v, f, eps) in enumerate(cavs):
        c, n, a = hm.hm_facets_from_triangles(v, f, orient=1)
        tree = hm.hm_build_cluster_tree(ctx, c, n, a, 32, 1.5)
        srv.register_cavity(cid, tree, eps, aca_tol=1e-8)
    return srv


@pytest.mark.parametrize("wide", [False, True], ids=["narrow", "sixteen"])
def test_server_alone_vs_mix_and_oracle(hm, ctx, wide):
    cavs = _cavities()
    widths = ((0, 16), (1, 12), (2, 16), (1, 9)) if wide else ((0, 1), (1, 3), (2, 2), (0, 4), (1, 1))
    log("case: server, 3 cavities", [c[1].shape[0] for c in cavs], "requests (cavity, columns)", widths)
    rng = np.random.default_rng(11)
    reqs = []  # (cavity id, T n x nrhs)
    for cid, nr in widths:
        n = cavs[cid][1].shape[0]
        reqs.append((cid, rng.uniform(300.0, 1500.0, (n, nr))))
    srv = _server(hm, ctx, cavs, 8 << 30, max_rhs=16 if wide else 8)
    alone = []
    for cid, T in reqs:
        tk = srv.submit(cid, T)
        alone.append(_wait(srv, [tk])[tk[0]])
    tks = [srv.submit(cid, T) for cid, T in reqs]
    mix = _wait(srv, tks)
    st = srv.stats()
    srv.close()
    log("stats", st)
    assert st["completed"] == 2 * len(reqs) and st["assemblies"] == 3
    refs = {}
    for (cid, T), a, tk in zip(reqs, alone, tks):
        m = mix[tk[0]]
        dJ, dq = rel(m[0], a[0]), rel(m[1], a[1])
        if cid not in refs:
            v, f, eps = cavs[cid]
            _, _, _, F = oracle_dense(v, f)
            refs[cid] = radiosity.DenseRadiosity(F, eps)
        Jo = refs[cid].radiosity(T)
        qo = refs[cid].flux(T, Jo)
        eJ, eq = rel(a[0], Jo), rel(a[1], qo)
        log("cavity %d nrhs %d: alone vs mix dJ %.1e dq %.1e; vs oracle e(J) %.2e e(q) %.2e; latency %.1f ms"
            % (cid, T.shape[1], dJ, dq, eJ, eq, 1e3 * m[2]["latency"]))
        assert dJ <= 1e-12 and dq <= 1e-12
        assert eJ <= 1e-6 and eq <= 1e-6


def _cavity_bytes(hm, ctx, cavs):
    """Device bytes of each cavity's H-matrix as the server assembles it."""
    out = []
    for v, f, eps in cavs:
        c, n, a = hm.hm_facets_from_triangles(v, f, orient=1)
        tree = hm.hm_build_cluster_tree(ctx, c, n, a, 32, 1.5)
        M = hm.hm_assemble_hmatrix(ctx, tree, 1e-8, 256, hm.HM_BF16, hm.HM_F32, 1, 0)
        out.append(M.stats()["bytes_device"] + 32 * f.shape[0])
    return out


def test_server_evicts_under_a_small_budget(hm, ctx):
    cavs = _cavities()
    sizes = _cavity_bytes(hm, ctx, cavs)
    # room for the largest cavity and one round of it, not for all three
    budget = max(sizes) + (2 << 20)
    log("case: server with a budget that holds the largest cavity: sizes", sizes, "budget", budget)
    assert sum(sizes) > budget
    rng = np.random.default_rng(12)
    T = [rng.uniform(300.0, 1500.0, (c[1].shape[0], 1)) for c in cavs]
    big = _server(hm, ctx, cavs, 8 << 30)
    tks = [big.submit(cid, T[cid]) for cid in range(3)]
    ref = _wait(big, tks)
    big.close()
    small = _server(hm, ctx, cavs, budget)
    out = {}
    for rnd in range(2):
        for cid in range(3):
            tk = small.submit(cid, T[cid])
            out[(rnd, cid)] = _wait(small, [tk])[tk[0]]
    st = small.stats()
    small.close()
    log("stats", st)
    assert st["evictions"] >= 1 and st["assemblies"] >= 4 and st["rejected"] == 0
    for (rnd, cid), r in out.items():
        want = ref[tks[cid][0]]
        assert rel(r[0], want[0]) <= 1e-12 and rel(r[1], want[1]) <= 1e-12


def test_server_cold_mix_assembles_while_serving(hm, ctx):
    cavs = _cavities()
    log("case: server cold start, 3 cavities submitted at once")
    rng = np.random.default_rng(13)
    reqs = []
    for cid, nr in ((2, 2), (0, 1), (1, 3), (2, 1), (0, 4), (1, 1), (2, 2)):
        reqs.append((cid, rng.uniform(300.0, 1500.0, (cavs[cid][1].shape[0], nr))))
    warm = _server(hm, ctx, cavs, 8 << 30)
    alone = []
    for cid, T in reqs:
        tk = warm.submit(cid, T)
        alone.append(_wait(warm, [tk])[tk[0]])
    warm.close()
    cold = _server(hm, ctx, cavs, 8 << 30)
    tks = [cold.submit(cid, T) for cid, T in reqs]
    mix = _wait(cold, tks)
    st = cold.stats()
    cold.close()
    log("stats", st)
    assert st["completed"] == len(reqs) and st["assemblies"] == 3
    for (cid, T), a, tk in zip(reqs, alone, tks):
        m = mix[tk[0]]
        assert rel(m[0], a[0]) <= 1e-12 and rel(m[1], a[1]) <= 1e-12, cid


def test_server_rejects_a_request_larger_than_its_budget(hm, ctx):
    """A cavity whose H-matrix alone exceeds the budget is built once (its
    size is unknown before), then its request fails with HM_ENOMEM and is
    counted as rejected; the server keeps serving."""
    cavs = _cavities()
    sizes = _cavity_bytes(hm, ctx, cavs)
    budget = sizes[2] // 2
    log("case: server budget %d below the cylinder's %d bytes" % (budget, sizes[2]))
    srv = _server(hm, ctx, cavs, budget)
    T = np.full((cavs[2][1].shape[0], 1), 600.0)
    tk = srv.submit(2, T)
    with pytest.raises(hm.HMError) as ei:
        _wait(srv, [tk])
    assert ei.value.status == hm.HM_ENOMEM
    st = srv.stats()
    srv.close()
    log("stats", st)
    assert st["rejected"] == 1 and st["completed"] == 0


def test_server_requires_one_set_of_storage_types(hm, ctx):
    """A round composes every active cavity into one product, so all cavities
    of a server share their storage types; BF16 factors need their FP32 copy
    (the FP64 residual reads it)."""
    cavs = _cavities()
    p = hm.solve_params(rtol=1e-9, mixed_precision=1, ir_inner_rtol=1e-3)
    srv = hm.Server(ctx, hbm_budget_bytes=1 << 30, max_active=4, params=p)
    trees = []
    for v, f, eps in cavs:
        c, n, a = hm.hm_facets_from_triangles(v, f, orient=1)
        trees.append(hm.hm_build_cluster_tree(ctx, c, n, a, 32, 1.5))
    with pytest.raises(hm.HMError) as e0:
        srv.register_cavity(0, trees[0], cavs[0][2], lowrank_dtype=hm.HM_BF16, keep_f32_copy=0)
    assert e0.value.status == hm.HM_EINVAL
    srv.register_cavity(0, trees[0], cavs[0][2], lowrank_dtype=hm.HM_BF16, keep_f32_copy=1)
    with pytest.raises(hm.HMError) as e1:
        srv.register_cavity(1, trees[1], cavs[1][2], lowrank_dtype=hm.HM_F32, keep_f32_copy=0)
    assert e1.value.status == hm.HM_EINVAL
    with pytest.raises(hm.HMError) as e2:
        srv.register_cavity(1, trees[1], cavs[1][2], lowrank_dtype=hm.HM_BF16, dense_dtype=hm.HM_BF16,
                            keep_f32_copy=1)
    assert e2.value.status == hm.HM_EINVAL
    srv.register_cavity(1, trees[1], cavs[1][2], lowrank_dtype=hm.HM_BF16, keep_f32_copy=1)
    srv.close()


def test_server_bench_configuration_matches_dense_oracle(hm, ctx):
    """Three cavity ids of the serving workload (one of each type, 5,120 to
    11,534 facets) served with the bench's parameters: leaf 64, eta 1.5,
    ACA 1e-6, BF16 factors (dithered rounding) + FP32 near field + FP32
    copy, FP64 refinement to a residual of 1e-7 (inner FP32 GMRES to 2e-4),
    all three requests
    submitted together.  J and q against the oracle's dense FP64 LU solution
    of the same requests (``tests/golden/c5_reference.npz``, written by
    ``tests/golden/make_c5_reference.py`` from ``oracle/`` only): relative
    L2 <= 1e-6 per right-hand side."""
    import os

    from workloads import configs
    ref = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_reference.npz"))
    seed = int(ref["seed"])
    p = hm.solve_params(rtol=1e-7, restart=30, max_iter=400, mixed_precision=1, ir_inner_rtol=2e-4, want_q=1)
    srv = hm.Server(ctx, hbm_budget_bytes=64 << 30, max_active=64, max_rhs_per_slot=8, params=p)
    reqs = []
    for cid, nrhs, idx in ref["requests"]:
        cav = configs.c5_cavity(int(cid))
        c, n, a = hm.hm_facets_from_triangles(cav.v, cav.tri, orient=1)
        tree = hm.hm_build_cluster_tree(ctx, c, n, a, cav.leaf, cav.eta)
        srv.register_cavity(int(cid), tree, cav.eps, aca_tol=cav.aca_tol, lowrank_dtype=hm.HM_BF16,
                            dense_dtype=hm.HM_F32, keep_f32_copy=1, lowrank_rounding=1)
        reqs.append((int(cid), configs.request_temperatures(cav.n, int(nrhs), seed, int(idx))))
    log("case: serving configuration, ids %s" % [(cid, T.shape) for cid, T in reqs])
    tks = [srv.submit(cid, T) for cid, T in reqs]
    res = _wait(srv, tks, timeout=120.0)
    srv.close()
    for (cid, T), tk in zip(reqs, tks):
        J, q, info = res[tk[0]]
        eJ = radiosity.relative_l2(J, ref["J_%d" % cid])
        eq = radiosity.relative_l2(q, ref["q_%d" % cid])
        log("id %d (%d facets, %d columns): residual %.1e, e(J) max %.2e, e(q) max %.2e" %
            (cid, T.shape[0], T.shape[1], info["rel_residual"], eJ.max(), eq.max()))
        assert info["rel_residual"] <= 1e-7
        assert np.all(eJ <= 1e-6) and np.all(eq <= 1e-6)
