"""Helpers shared by the GPU tests: build cavities through the C ABI and run
the oracle on the same seeded inputs."""
import sys

import numpy as np

from oracle import aca, geometry, radiosity, viewfactor


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def device():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch.device("cuda:0")


def dt(x, dev=None):
    import torch
    return torch.as_tensor(np.asfortranarray(x), dtype=torch.float64, device=dev or device())


def to_np(t):
    return t.detach().cpu().numpy()


def build(hm, ctx, v, tri, leaf, eta, tol, lr=None, dense=None, keep=0, k_max=256, closed=0):
    lr = hm.HM_F64 if lr is None else lr
    dense = hm.HM_F64 if dense is None else dense
    c, n, a = hm.hm_facets_from_triangles(v, tri, orient=1)
    tree = hm.hm_build_cluster_tree(ctx, c, n, a, leaf, eta)
    M = hm.hm_assemble_hmatrix(ctx, tree, tol, k_max, lr, dense, keep, closed)
    return tree, M


def oracle_dense(v, tri):
    c, n, a = geometry.facets_from_triangles(v, tri)
    return c, n, a, viewfactor.view_factor_matrix(c, n, a)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def full_matrix(hm, ctx, M, n, dtype="float64", nrhs=16):
    """F_H expanded column by column with unit vectors (exact: each output
    entry is one stored value times 1 plus zeros)."""
    import torch
    tdt = torch.float64 if dtype == "float64" else torch.float32
    F = np.empty((n, n))
    for j0 in range(0, n, nrhs):
        k = min(nrhs, n - j0)
        X = torch.zeros((k, n), dtype=tdt, device=device()).T  # column-major n x k
        for q in range(k):
            X[j0 + q, q] = 1.0
        Y = torch.zeros((k, n), dtype=tdt, device=device()).T
        hm.hm_hmatvec(ctx, M, X, Y)
        F[:, j0:j0 + k] = to_np(Y)
    return F
