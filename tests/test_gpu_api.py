"""GPU tests of the C ABI's state handling: cached compositions after a new
work split, products and solves of one matrix on two streams, and the
stream-ordered reuse of the library's device memory.

* After hm_matrix_set_tuning every cached composition, batch and captured
  graph of the matrix is rebuilt: products and solves (also a batched solve
  that was cached under another matrix) equal the ones before the change up
  to the order of partial sums (1e-13 relative, FP64 vectors).
* The autotuner also picks the second kernel's waves per workgroup (2, 4
  or 8) and reports its time; every shape (2, 4, 8, or by tile count) gives
  the same bits for one and two columns, FP32 and FP64 vectors.
* Two contexts on two streams in one thread, issuing products of the same
  matrices and solves interleaved without synchronising in between, give
  the same bits as the same calls issued one by one with a synchronisation
  after each.
"""
import numpy as np
import pytest

from workloads import meshes

from gpu_common import build, log, rel, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hm():
    from paper_2305_06891_amd import hm as _hm
    return _hm


def _cavity(hm, ctx, nu=14, axes=(3.0, 2.0, 1.0), lr=None):
    v, f = meshes.ellipsoid(nu, axes)
    f = meshes.inward(f)
    lr = hm.HM_F32 if lr is None else lr
    _, M = build(hm, ctx, v, f, 64, 1.5, 1e-6, lr, hm.HM_F32)
    return f.shape[0], M


def test_set_tuning_rebuilds_cached_state(hm):
    import torch
    ctx = hm.Context(0)
    n, M = _cavity(hm, ctx)
    n2, M2 = _cavity(hm, ctx, nu=10, axes=(2.0, 1.0, 1.0))
    log("case: set_tuning after cached products and solves, ellipsoids %d and %d facets" % (n, n2))
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(5)
    X = torch.as_tensor(rng.uniform(0.5, 1.5, n), dtype=torch.float64, device=dev)
    eps = torch.as_tensor(rng.uniform(0.1, 0.9, n), dtype=torch.float64, device=dev)
    T = torch.as_tensor(rng.uniform(300.0, 1500.0, n), dtype=torch.float64, device=dev)
    eps2 = torch.as_tensor(rng.uniform(0.1, 0.9, n2), dtype=torch.float64, device=dev)
    T2 = torch.as_tensor(rng.uniform(300.0, 1500.0, n2), dtype=torch.float64, device=dev)
    p = hm.solve_params(rtol=1e-12)

    def run():
        y = to_np(hm.hm_hmatvec(ctx, M, X, torch.zeros_like(X)))
        J, q, info = hm.hm_solve_radiosity(ctx, M, eps, T, params=p)
        Jb, qb, _ = hm.hm_solve_radiosity_batched(ctx, [M2, M], [eps2, eps], [T2, T], params=p)
        torch.cuda.synchronize()
        return y, to_np(J), to_np(q), to_np(Jb[1]), to_np(qb[1])

    before = run()
    old = M.tuning()
    M.set_tuning(ctx, 64, 0)
    assert M.tuning()["p1_rows"] == 64
    after = run()
    log("tuning %s -> %s" % (old, M.tuning()))
    errs = [rel(a, b) for a, b in zip(after, before)]
    log("rel differences after set_tuning:", ["%.1e" % e for e in errs])
    assert errs[0] <= 1e-13
    assert max(errs[1:]) <= 1e-11


def test_phase2_shape_is_tuned_and_changes_no_bits(hm):
    import torch
    ctx = hm.Context(0)
    v, f = meshes.ellipsoid(14, (3.0, 2.0, 1.0))
    f = meshes.inward(f)
    c, nrm, a = hm.hm_facets_from_triangles(v, f, orient=1)
    tree = hm.hm_build_cluster_tree(ctx, c, nrm, a, 64, 1.5)
    M = hm.hm_assemble_hmatrix(ctx, tree, 1e-6, 256, hm.HM_BF16, hm.HM_F32, 1, autotune=1)
    n = f.shape[0]
    t = M.tuning()
    log("case: phase-2 shapes, ellipsoid %d facets, autotuned: %s" % (n, t))
    assert t["p2_waves"] in (2, 4, 8) and t["p2_us"] > 0.0
    dev = torch.device("cuda:0")
    outs = {}
    for w in (2, 4, 8, 0):
        M.set_tuning_phase2(ctx, w)
        assert M.tuning()["p2_waves"] == w
        for dt in (torch.float32, torch.float64):
            for nr in (1, 2):
                X = torch.as_tensor(np.random.default_rng(nr).uniform(0.5, 1.5, (n, nr)), dtype=dt,
                                    device=dev).t().contiguous().t()
                Y = torch.zeros_like(X)
                hm.hm_hmatvec(ctx, M, X, Y)
                torch.cuda.synchronize()
                outs.setdefault((dt, nr), []).append(to_np(Y))
    for k, ys in outs.items():
        assert all(np.array_equal(ys[0], y) for y in ys[1:]), k


def test_two_streams_interleaved_equal_sequential(hm):
    import torch
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    ca = hm.Context(0, stream=sa.cuda_stream)
    cb = hm.Context(0, stream=sb.cuda_stream)
    n1, M1 = _cavity(hm, ca)
    n2, M2 = _cavity(hm, ca, nu=11, axes=(2.0, 2.0, 1.0), lr=hm.HM_BF16)
    log("case: two contexts on two streams, ellipsoids %d and %d facets, interleaved products" % (n1, n2))
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(9)
    # (matrix, n, width, vector type) per call; widths grow so that the
    # matrices' permuted buffers are reallocated between the two streams
    calls = []
    for k, w in enumerate((1, 2, 4, 16, 1, 8, 16, 3)):
        M, n = (M1, n1) if k % 3 != 2 else (M2, n2)
        tdt = torch.float64 if k % 2 == 0 else torch.float32
        X = torch.as_tensor(np.asfortranarray(rng.uniform(0.5, 1.5, (n, w))), dtype=tdt, device=dev)
        calls.append((M, X))
    torch.cuda.synchronize()
    # sequential: one context, synchronised after each call
    seq = []
    for M, X in calls:
        Y = torch.zeros_like(X)
        sa.wait_stream(torch.cuda.current_stream())
        hm.hm_hmatvec(ca, M, X, Y)
        torch.cuda.synchronize()
        seq.append(to_np(Y))
    # interleaved over the two streams, no synchronisation in between
    outs = []
    for k, (M, X) in enumerate(calls):
        Y = torch.zeros_like(X)
        ctx, st = (ca, sa) if k % 2 == 0 else (cb, sb)
        # the output buffer is zeroed on torch's current stream: order it
        st.wait_stream(torch.cuda.current_stream())
        hm.hm_hmatvec(ctx, M, X, Y)
        outs.append(Y)
    torch.cuda.synchronize()
    worst = max(float(np.max(np.abs(to_np(Y) - s))) for Y, s in zip(outs, seq))
    log("interleaved vs sequential: max abs difference %.3e" % worst)
    assert worst == 0.0
    # solves on both contexts, alternating, against the same solves alone
    eps = torch.as_tensor(rng.uniform(0.1, 0.9, n1), dtype=torch.float64, device=dev)
    T = torch.as_tensor(rng.uniform(300.0, 1500.0, n1), dtype=torch.float64, device=dev)
    p = hm.solve_params(rtol=1e-12)
    torch.cuda.synchronize()
    J0, q0, _ = hm.hm_solve_radiosity(ca, M1, eps, T, params=p)
    torch.cuda.synchronize()
    res = []
    for k in range(4):
        ctx, st = (ca, sa) if k % 2 == 0 else (cb, sb)
        st.wait_stream(torch.cuda.current_stream())
        J, q, info = hm.hm_solve_radiosity(ctx, M1, eps, T, params=p)
        res.append((J, q))
    torch.cuda.synchronize()
    for J, q in res:
        assert float(np.max(np.abs(to_np(J) - to_np(J0)))) == 0.0
        assert float(np.max(np.abs(to_np(q) - to_np(q0)))) == 0.0
