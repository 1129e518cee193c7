"""GPU tests of the batched assembly entry point (shared ACA launches over
several cavities).

* Cavities of different sizes, precisions and ACA tolerances assembled in one
  call give the same statistics (blocks, ranks, fallbacks, entries) and the
  same products, bit for bit, as the same cavities assembled one at a time:
  each block's ACA depends only on the block, and with the fixed work split
  the plans are the same.  The cavities are large enough for both ACA
  kernels (one wave per block up to 64 x 64, one workgroup above).
* With autotuning, every tuned matrix of the call gets the same split, timed
  on their batched product; blocks and ranks are those of the fixed split
  (only the work lists, and so the device bytes, differ) and the product
  equals the fixed-split product up to the order of FP32 partial sums.
"""
import numpy as np
import pytest

from workloads import meshes

from gpu_common import log, rel, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hm():
    from paper_2305_06891_amd import hm as _hm
    return _hm


@pytest.fixture(scope="module")
def ctx(hm):
    return hm.Context(0)


def _cavities(hm, ctx):
    out = []
    specs = ((meshes.icosphere(4), 64, 1.5, 1e-6, hm.HM_F32, hm.HM_F32, 0),
             (meshes.ellipsoid(16, (3.0, 2.0, 1.0)), 32, 2.0, 1e-8, hm.HM_F64, hm.HM_F64, 0),
             (meshes.cylinder(60, 40, 12, seed=5), 64, 1.5, 1e-6, hm.HM_BF16, hm.HM_F32, 1),
             (meshes.icosphere(2), 32, 2.0, 1e-7, hm.HM_F32, hm.HM_F32, 0))
    for (v, f), leaf, eta, tol, lr, dn, keep in specs:
        f = meshes.inward(f)
        c, n, a = hm.hm_facets_from_triangles(v, f, orient=1)
        out.append((hm.hm_build_cluster_tree(ctx, c, n, a, leaf, eta), tol, lr, dn, keep, f.shape[0]))
    return out


def _x(n, dtype, seed):
    import torch
    return torch.as_tensor(np.random.default_rng(seed).uniform(0.5, 1.5, n), dtype=dtype, device="cuda")


def test_batched_assembly_equals_one_at_a_time(hm, ctx):
    import torch
    cavs = _cavities(hm, ctx)
    log("case: batched assembly of %d cavities" % len(cavs), [c[5] for c in cavs])
    alone = [hm.hm_assemble_hmatrix(ctx, t, tol, 256, lr, dn, keep) for t, tol, lr, dn, keep, _ in cavs]
    batch = hm.hm_assemble_hmatrix_batched(ctx, [c[0] for c in cavs], aca_tol=[c[1] for c in cavs],
                                           lowrank_dtype=[c[2] for c in cavs], dense_dtype=[c[3] for c in cavs],
                                           keep_f32_copy=[c[4] for c in cavs])
    for q, (a, b) in enumerate(zip(alone, batch)):
        sa, sb = a.stats(), b.stats()
        log("cavity %d: %s" % (q, sa))
        assert sa == sb
        assert a.tuning() == b.tuning()
        n = cavs[q][5]
        for dtype in (torch.float64, torch.float32):
            x = _x(n, dtype, 10 + q)
            ya = torch.zeros_like(x)
            yb = torch.zeros_like(x)
            hm.hm_hmatvec(ctx, a, x, ya)
            hm.hm_hmatvec(ctx, b, x, yb)
            torch.cuda.synchronize()
            assert torch.equal(ya, yb), (q, dtype)
        if cavs[q][4]:
            x = _x(n, torch.float64, 20 + q)
            ya = torch.zeros_like(x)
            yb = torch.zeros_like(x)
            hm.hm_hmatvec(ctx, a, x, ya, use_f32_copy=True)
            hm.hm_hmatvec(ctx, b, x, yb, use_f32_copy=True)
            torch.cuda.synchronize()
            assert torch.equal(ya, yb), (q, "f32 copy")
    assert any(s.stats()["max_rank"] > 32 for s in batch)  # blocks for the workgroup kernel


def test_batched_assembly_tunes_one_split(hm, ctx):
    import torch
    cavs = _cavities(hm, ctx)[:3]
    log("case: joint autotuning of %d cavities" % len(cavs))
    fixed = hm.hm_assemble_hmatrix_batched(ctx, [c[0] for c in cavs], aca_tol=[c[1] for c in cavs],
                                           lowrank_dtype=hm.HM_F32, dense_dtype=hm.HM_F32)
    tuned = hm.hm_assemble_hmatrix_batched(ctx, [c[0] for c in cavs], aca_tol=[c[1] for c in cavs],
                                           lowrank_dtype=hm.HM_F32, dense_dtype=hm.HM_F32, autotune=1)
    tn = [m.tuning() for m in tuned]
    log("tunings", tn)
    assert all(t == tn[0] for t in tn) and tn[0]["p1_us"] > 0
    for q, (a, b) in enumerate(zip(fixed, tuned)):
        # the device bytes include the work lists of the split
        sa, sb = a.stats(), b.stats()
        sa.pop("bytes_device")
        sb.pop("bytes_device")
        assert sa == sb
        x = _x(cavs[q][5], torch.float32, 30 + q)
        ya = torch.zeros_like(x)
        yb = torch.zeros_like(x)
        hm.hm_hmatvec(ctx, a, x, ya)
        hm.hm_hmatvec(ctx, b, x, yb)
        e = rel(to_np(yb), to_np(ya))
        log("cavity %d: fixed vs tuned split rel diff %.2e" % (q, e))
        assert e <= 2e-6
