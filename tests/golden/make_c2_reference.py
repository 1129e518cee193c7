"""Writes ``c2_reference.npz``: the oracle's radiosity J and flux q (FP64,
dense centroid-rule F of eq. (10), LU of the reflection system of eq. (11),
flux of eq. (12)) for the 20,176-facet jittered cylinder with its seeded
emissivities and temperatures.  Calls only ``oracle/`` and the seeded input
recipe; about 2-3 minutes and 10 GB of host memory.

    python tests/golden/make_c2_reference.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import geometry, radiosity, viewfactor  # noqa: E402
from workloads import configs  # noqa: E402


def main():
    cav = configs.c2_cylinder()
    c, n, a = geometry.facets_from_triangles(cav.v, cav.tri)
    t0 = time.time()
    F = viewfactor.view_factor_matrix(c, n, a)
    t1 = time.time()
    rad = radiosity.DenseRadiosity(F, cav.eps)
    T = cav.T[:, 0]
    J = rad.radiosity(T)
    q = rad.flux(T, J)
    t2 = time.time()
    out = os.path.join(HERE, "c2_reference.npz")
    np.savez_compressed(out, J=J, q=q, n=np.int64(cav.n), area=a)
    print("wrote %s (n=%d, assembly %.1f s, LU + solves %.1f s)" % (out, cav.n, t1 - t0, t2 - t1))


if __name__ == "__main__":
    main()
