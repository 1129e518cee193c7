"""Writes ``c3_reference.npz``: the oracle's radiosity J and flux q (FP64,
dense centroid-rule F of eq. (10), LU of the reflection system of eq. (11),
flux of eq. (12)) for four cavities of the 64-cavity batching workload with
their seeded emissivities and temperatures: the 35,280-facet ellipsoid (one
of the two largest) and an 18,000-18,400-facet icosphere, ellipsoid and
cylinder.  Calls only ``oracle/`` and the seeded input recipe; about 15
minutes on 8 cores and 25 GB of host memory at the largest cavity.

    python tests/golden/make_c3_reference.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import geometry, radiosity, viewfactor  # noqa: E402
from workloads import configs  # noqa: E402

INDICES = (15, 3, 54, 27)


def main():
    cavs = configs.c3_batch()
    out = {"indices": np.array(INDICES, dtype=np.int64)}
    for i in INDICES:
        cav = cavs[i]
        c, n, a = geometry.facets_from_triangles(cav.v, cav.tri)
        t0 = time.time()
        F = viewfactor.view_factor_matrix(c, n, a)
        t1 = time.time()
        rad = radiosity.DenseRadiosity(F, cav.eps, keep_c=False)
        T = cav.T[:, 0]
        J = rad.radiosity(T)
        q = rad.flux(T, J)
        t2 = time.time()
        out["J_%d" % i] = J
        out["q_%d" % i] = q
        out["n_%d" % i] = np.int64(cav.n)
        print("%s: n=%d, assembly %.1f s, LU + solves %.1f s" % (cav.name, cav.n, t1 - t0, t2 - t1), flush=True)
        del F, rad
    path = os.path.join(HERE, "c3_reference.npz")
    np.savez_compressed(path, **out)
    print("wrote", path)


if __name__ == "__main__":
    main()
