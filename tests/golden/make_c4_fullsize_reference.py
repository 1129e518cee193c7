"""Writes ``c4_fullsize_reference.npz``: the first backward-Euler step of
scenarios 0 and 1 of the many-right-hand-side transient workload at full
size (the 200,000-facet (4, 2, 1) ellipsoid, eps 0.8, m_c = 1e4, dt = 1 s),
computed by the oracle's large-n mode (``oracle/matfree.py``: the dense
definition of eqs. (10)-(12) with F applied on the fly in FP64 and GMRES to
a relative residual of 1e-12) and the lumped implicit Euler step of
``oracle/transient.py`` (Newton to a residual of 1e-11 of |m_c T^0 / dt|).
Stored: the temperature increments T^1 - T^0 of the two scenarios rounded
to FP32 (each increment is a few kelvin, so the rounding is below 1e-9 of
|T^1|).  Calls only ``oracle/`` and the seeded input recipe; about 1-2 hours
on 8 cores, 1 GB of memory.

    python tests/golden/make_c4_fullsize_reference.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import geometry, matfree, transient  # noqa: E402
from workloads import configs  # noqa: E402

SCEN = 2


def main():
    cav = configs.c4_ellipsoid(nu=100, scenarios=SCEN)
    c, n, a = geometry.facets_from_triangles(cav.v, cav.tri)
    t0 = time.time()
    rad = matfree.MatrixFreeRadiosity(c, n, a, cav.eps, rtol=1e-12)
    t1 = time.time()
    print("g: %d GMRES iterations, %.0f s" % (rad.iterations, t1 - t0), flush=True)
    T0 = cav.T[:, :SCEN]
    T1, it, rn = transient.newton_step(rad, T0, cav.extra["source"][:, :SCEN], cav.extra["mc"], cav.extra["dt"],
                                       tol=1e-11)
    t2 = time.time()
    print("step 1: %d Newton updates, residuals %s, %d products in all, %.0f s" %
          (it, rn, rad.F.products, t2 - t1), flush=True)
    out = os.path.join(HERE, "c4_fullsize_reference.npz")
    np.savez_compressed(out, dT1=(T1 - T0).astype(np.float32), n=np.int64(cav.n), scenarios=np.int64(SCEN))
    print("wrote", out)


if __name__ == "__main__":
    main()
