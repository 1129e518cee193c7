"""Writes ``c5_reference.npz``: the oracle's radiosity J and flux q (FP64,
dense centroid-rule F of eq. (10), LU of the reflection system of eq. (11),
flux of eq. (12)) for three cavity ids of the serving workload (one of each
type, 5,000-12,000 facets) with the temperatures of three seeded requests.
Calls only ``oracle/`` and the seeded input recipe; a few minutes.

    python tests/golden/make_c5_reference.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import geometry, radiosity, viewfactor  # noqa: E402
from workloads import configs  # noqa: E402

# (cavity id, right-hand sides, request index) of each stored request;
# temperatures from configs.request_temperatures(n, nrhs, SEED, index)
REQUESTS = ((0, 3, 0), (4, 1, 1), (5, 4, 2))
SEED = 5999


def main():
    out = {"requests": np.array(REQUESTS, dtype=np.int64), "seed": np.int64(SEED)}
    for cid, nrhs, idx in REQUESTS:
        cav = configs.c5_cavity(cid)
        c, n, a = geometry.facets_from_triangles(cav.v, cav.tri)
        t0 = time.time()
        rad = radiosity.DenseRadiosity(viewfactor.view_factor_matrix(c, n, a), cav.eps, keep_c=False)
        T = configs.request_temperatures(cav.n, nrhs, SEED, idx)
        J = rad.radiosity(T)
        q = rad.flux(T, J)
        out["J_%d" % cid] = J
        out["q_%d" % cid] = q
        print("%s: n=%d, %d right-hand sides, %.1f s" % (cav.name, cav.n, nrhs, time.time() - t0), flush=True)
    path = os.path.join(HERE, "c5_reference.npz")
    np.savez_compressed(path, **out)
    print("wrote", path)


if __name__ == "__main__":
    main()
