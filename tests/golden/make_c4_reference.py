"""Writes ``c4_reference.npz``: the oracle's lumped backward-Euler transient
(dense centroid-rule F of eq. (10), LU of the reflection system of eq. (11),
flux of eq. (12), diagonal Newton update; ``oracle/transient.py``) on the
18,000-facet member (geodesic frequency 30) of the (4, 2, 1) ellipsoid
family of the many-right-hand-side workload: 16 scenarios, 100 steps of
1 s, m_c = 1e4.  Stored: temperatures after steps 1 and 100 of scenarios
0-3 (all 16 are integrated; each is independent of the others).  Calls only
``oracle/`` and the seeded input recipe; a few minutes and 8 GB of memory.

    python tests/golden/make_c4_reference.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import geometry, radiosity, transient, viewfactor  # noqa: E402
from workloads import configs  # noqa: E402

NU, STEPS, KEEP = 30, 100, 4


def main():
    cav = configs.c4_ellipsoid(nu=NU, scenarios=16)
    c, n, a = geometry.facets_from_triangles(cav.v, cav.tri)
    t0 = time.time()
    rad = radiosity.DenseRadiosity(viewfactor.view_factor_matrix(c, n, a), cav.eps)
    t1 = time.time()
    T = cav.T.copy()
    src = cav.extra["source"]
    keep = {}
    for k in range(1, STEPS + 1):
        T, it, rn = transient.newton_step(rad, T, src, cav.extra["mc"], cav.extra["dt"], tol=1e-12)
        if k in (1, STEPS):
            keep[k] = T[:, :KEEP].copy()
    t2 = time.time()
    out = os.path.join(HERE, "c4_reference.npz")
    np.savez_compressed(out, T1=keep[1], T100=keep[STEPS], n=np.int64(cav.n), nu=np.int64(NU), steps=np.int64(STEPS))
    print("wrote %s (n=%d, LU %.1f s, %d steps %.1f s)" % (out, cav.n, t1 - t0, STEPS, t2 - t1))


if __name__ == "__main__":
    main()
