"""GPU test of the allocation-free product (hm_hmatvec_noalloc).

The entry point runs the same kernels as hm_hmatvec with every workspace in
the library's fixed device array, so its result must equal hm_hmatvec's bit
for bit.  Two calls in a row, the second on a smaller matrix and fewer
columns, check that the array's leftover contents from the first call do not
leak into the second; a product that needs more than the fixed array is
refused with HM_ENOMEM.
"""
import numpy as np
import pytest

from workloads import meshes

from gpu_common import build, log, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hm():
    from paper_2305_06891_amd import hm as _hm
    return _hm


def _cavity(hm, ctx, nu, axes, lr, dense):
    v, f = meshes.ellipsoid(nu, axes)
    f = meshes.inward(f)
    _, M = build(hm, ctx, v, f, 64, 1.5, 1e-6, lr, dense, keep=1 if lr == hm.HM_BF16 else 0)
    return f.shape[0], M


def _pair(hm, ctx, M, n, ncol, tdt, seed, alpha, beta):
    import torch
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(seed)
    shape = (n,) if ncol == 1 else (ncol, n)
    X = torch.as_tensor(rng.uniform(0.5, 1.5, shape), dtype=tdt, device=dev)
    Y0 = torch.as_tensor(rng.uniform(-1.0, 1.0, shape), dtype=tdt, device=dev)
    if ncol > 1:  # column-major n x ncol
        X, Y0 = X.T, Y0.T
    Ya = Y0.clone()
    Yb = Y0.clone()
    hm.hm_hmatvec(ctx, M, X, Ya, alpha, beta)
    hm.hm_hmatvec_noalloc(ctx, M, X, Yb, alpha, beta)
    torch.cuda.synchronize()
    return to_np(Ya), to_np(Yb)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_noalloc_equals_hmatvec_on_two_calls(hm, storage):
    import torch
    ctx = hm.Context(0)
    lr = hm.HM_F32 if storage == "f32" else hm.HM_BF16
    n1, M1 = _cavity(hm, ctx, 22, (3.0, 2.0, 1.0), lr, hm.HM_F32)
    n2, M2 = _cavity(hm, ctx, 10, (2.0, 1.5, 1.0), lr, hm.HM_F32)
    assert n2 < n1
    cases = [(M1, n1, 16, torch.float32, 0.7, 0.3),   # matrix cores, large input
             (M2, n2, 3, torch.float64, 1.0, 0.0),    # smaller matrix, fewer columns
             (M1, n1, 1, torch.float64, -0.5, 2.0),
             (M2, n2, 16, torch.float64, 1.0, 1.0)]
    for k, (M, n, ncol, tdt, a, b) in enumerate(cases):
        log("case: noalloc %s call %d n=%d ncol=%d %s alpha=%g beta=%g" % (storage, k, n, ncol, tdt, a, b))
        ya, yb = _pair(hm, ctx, M, n, ncol, tdt, 100 + k, a, b)
        assert np.all(np.isfinite(ya))
        assert np.array_equal(ya, yb), "max diff %g" % float(np.max(np.abs(ya - yb)))


def test_noalloc_refuses_a_product_beyond_its_scratch(hm):
    import torch
    ctx = hm.Context(0)
    n, M = _cavity(hm, ctx, 60, (3.0, 2.0, 1.0), hm.HM_F32, hm.HM_F32)
    log("case: noalloc beyond the scratch, n=%d, 16 columns" % n)
    X = torch.ones((16, n), dtype=torch.float64, device=torch.device("cuda:0")).T
    Y = torch.zeros_like(X)
    with pytest.raises(hm.HMError) as ei:
        hm.hm_hmatvec_noalloc(ctx, M, X, Y)
    assert ei.value.status == hm.HM_ENOMEM
    assert "scratch" in str(ei.value)
    # the refused call queued nothing: a product that fits still works
    y1 = torch.ones(n, dtype=torch.float64, device=X.device)
    ya = hm.hm_hmatvec(ctx, M, y1, torch.zeros_like(y1))
    yb = hm.hm_hmatvec_noalloc(ctx, M, y1, torch.zeros_like(y1))
    torch.cuda.synchronize()
    assert np.array_equal(to_np(ya), to_np(yb))
