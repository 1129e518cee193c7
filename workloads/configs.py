"""Seeded recipes of the five synthetic workloads (input data only).

Each recipe returns triangles already wound inward (normals into the cavity),
per-facet emissivities and temperatures, and the tree / compression
parameters of the workload.  Nothing here computes view factors, radiosities
or fluxes.

Seeds: numpy ``default_rng``.  C1 temperature seed 0; C2 jitter seed 1 and
emissivity/temperature seed 2 (emissivity drawn first, then temperature);
C3 cavity list seed 3, cavity ``i`` uses ``default_rng([3, i])``; C4 scenario
``s`` uses seed ``400 + s``; C5 cavity id ``c`` uses seed ``5000 + c``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import meshes

SIGMA = 5.670374e-8  # Stefan-Boltzmann constant, W m^-2 K^-4


@dataclass
class Cavity:
    name: str
    v: np.ndarray            # vertices (nv, 3) float64
    tri: np.ndarray          # triangles (nt, 3) int32, inward winding
    eps: np.ndarray          # (nt,) emissivity in (0, 1]
    T: np.ndarray            # (nt, nrhs) temperatures in K
    leaf: int = 64           # n_min
    eta: float = 1.5         # admissibility constant
    aca_tol: float = 1e-6
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.tri.shape[0])


def c1_icosphere() -> Cavity:
    """Unit icosphere, recursive level 3 (1,280 facets); eps = 0.8;
    T ~ U[300, 1000] K from seed 0; leaf 32, eta 2, ACA 1e-8 (all FP64)."""
    v, f = meshes.icosphere(3)
    n = f.shape[0]
    T = np.random.default_rng(0).uniform(300.0, 1000.0, n)
    return Cavity("c1_icosphere_1280", v, meshes.inward(f), np.full(n, 0.8), T[:, None],
                  leaf=32, eta=2.0, aca_tol=1e-8)


def c2_cylinder() -> Cavity:
    """Jittered closed cylinder r=1, h=4, 20,176 facets (jitter seed 1);
    eps ~ U[0.1, 0.9], T ~ U[300, 1500] K (seed 2); leaf 64, eta 1.5, ACA 1e-6."""
    v, f = meshes.cylinder(104, 66, 16, 1.0, 4.0, 0.05, seed=1)
    n = f.shape[0]
    rng = np.random.default_rng(2)
    eps = rng.uniform(0.1, 0.9, n)
    T = rng.uniform(300.0, 1500.0, n)
    return Cavity("c2_cylinder_20176", v, meshes.inward(f), eps, T[:, None])


def _typed_cavity(kind: str, n_target: int, axes, rng_geo_seed) -> tuple:
    if kind == "icosphere":
        nu = max(1, int(round(math.sqrt(n_target / 20.0))))
        v, f = meshes.geodesic(nu)
    elif kind == "ellipsoid":
        nu = max(1, int(round(math.sqrt(n_target / 20.0))))
        v, f = meshes.ellipsoid(nu, axes)
    else:
        v, f = meshes.cylinder_for_count(n_target, seed=rng_geo_seed)
    return v, meshes.inward(f)


def c3_batch(count: int = 64, n_lo: int = 2000, n_hi: int = 40000) -> list:
    """``count`` convex cavities: type uniform over {icosphere, ellipsoid with
    axes ~ U[1,3]^3, cylinder r=1 h=4}; facet count log-uniform in
    [n_lo, n_hi]; eps ~ U[0.1, 0.9], T ~ U[300, 1500] K per facet.
    Low-rank factors BF16, near field FP32 (leaf 64, eta 1.5, ACA 1e-6)."""
    rng = np.random.default_rng(3)
    kinds = ("icosphere", "ellipsoid", "cylinder")
    out = []
    for i in range(count):
        kind = kinds[int(rng.integers(0, 3))]
        n_target = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        axes = tuple(rng.uniform(1.0, 3.0, 3))
        v, f = _typed_cavity(kind, n_target, axes, rng_geo_seed=int(1000 + i))
        n = f.shape[0]
        r2 = np.random.default_rng([3, i])
        eps = r2.uniform(0.1, 0.9, n)
        T = r2.uniform(300.0, 1500.0, n)
        out.append(Cavity(f"c3_{i:02d}_{kind}_{n}", v, f, eps, T[:, None],
                          extra={"kind": kind, "axes": axes}))
    return out


def c4_ellipsoid(nu: int = 100, scenarios: int = 16) -> Cavity:
    """Closed ellipsoid with semi-axes (4, 2, 1), geodesic frequency ``nu``
    (nu = 100 gives 200,000 facets); eps = 0.8; lumped heat capacity
    rho*c*thickness = 1e4 J m^-2 K^-1; ``scenarios`` right-hand sides, scenario
    ``s`` drawing T0 ~ U[300, 1000] K then a source ~ U[0, 500] W m^-2 from
    seed 400 + s.  Backward Euler, dt = 1 s."""
    v, f = meshes.ellipsoid(nu, (4.0, 2.0, 1.0))
    n = f.shape[0]
    T0 = np.empty((n, scenarios))
    src = np.empty((n, scenarios))
    for s in range(scenarios):
        r = np.random.default_rng(400 + s)
        T0[:, s] = r.uniform(300.0, 1000.0, n)
        src[:, s] = r.uniform(0.0, 500.0, n)
    return Cavity(f"c4_ellipsoid_{n}", v, meshes.inward(f), np.full(n, 0.8), T0,
                  extra={"source": src, "mc": 1.0e4, "dt": 1.0})


def fe_shell(nu: int = 32) -> Cavity:
    """Conducting ellipsoid shell (semi-axes 4, 2, 1; frequency ``nu``:
    20 nu^2 facets, 10 nu^2 + 2 nodes, watertight) for the finite-element
    coupling: eps ~ U[0.2, 0.9] per facet, nodal T0 ~ U[300, 1000] K and facet
    sources ~ U[0, 500] W m^-2 from seed 600; shell conductance k h = 5 W/K,
    capacity rho c h = 2e3 J m^-2 K^-1, implicit Euler with dt = 1 s.  The
    cavity's T field holds the nodal temperatures (one column)."""
    v, f = meshes.ellipsoid(nu, (4.0, 2.0, 1.0))
    # one node per position: the mesh generator repeats the vertices on the
    # seams between its patches, which would cut the conducting shell there
    uniq, inv = np.unique(np.round(v, 12), axis=0, return_inverse=True)
    v, f = uniq, inv.reshape(-1)[f].astype(f.dtype)
    rng = np.random.default_rng(600)
    eps = rng.uniform(0.2, 0.9, f.shape[0])
    T0 = rng.uniform(300.0, 1000.0, v.shape[0])
    src = rng.uniform(0.0, 500.0, f.shape[0])
    return Cavity(f"fe_shell_{f.shape[0]}", v, meshes.inward(f), eps, T0[:, None],
                  extra={"source": src, "conductance": 5.0, "capacity": 2.0e3, "dt": 1.0})


def c5_cavity(cid: int, n_lo: int = 1000, n_hi: int = 100000) -> Cavity:
    """Cavity id ``cid`` of the serving workload: type, facet count
    (log-uniform in [n_lo, n_hi]), axes and per-facet eps ~ U[0.1, 0.9] are
    fixed by seed 5000 + cid."""
    rng = np.random.default_rng(5000 + cid)
    kinds = ("icosphere", "ellipsoid", "cylinder")
    kind = kinds[int(rng.integers(0, 3))]
    n_target = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
    axes = tuple(rng.uniform(1.0, 3.0, 3))
    v, f = _typed_cavity(kind, n_target, axes, rng_geo_seed=int(7000 + cid))
    n = f.shape[0]
    eps = rng.uniform(0.1, 0.9, n)
    return Cavity(f"c5_{cid:03d}_{kind}_{n}", v, f, eps, np.zeros((n, 0)),
                  extra={"kind": kind, "axes": axes})


def c5_requests(count: int, rate_hz: float, n_ids: int = 256, zipf_s: float = 1.1,
                seed: int = 5999):
    """Poisson arrivals at ``rate_hz``; cavity id by Zipf(s) over ``n_ids``
    ids (rank r has weight r**-s, id = rank - 1); 1..8 right-hand sides
    (uniform); temperatures are drawn later per request from
    ``default_rng([seed, request_index])`` in U[300, 1500] K.
    Returns (arrival times, ids, nrhs)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, count)
    t = np.cumsum(gaps)
    w = np.arange(1, n_ids + 1, dtype=np.float64) ** (-zipf_s)
    ids = rng.choice(n_ids, size=count, p=w / w.sum())
    nrhs = rng.integers(1, 9, count)
    return t, ids, nrhs


def request_temperatures(n: int, nrhs: int, seed: int, index: int) -> np.ndarray:
    return np.random.default_rng([seed, index]).uniform(300.0, 1500.0, (n, nrhs))


def fibonacci_spiral(nu: int = 5, radius: float = 0.5, eps: float = 0.8, T_amb: float = 300.0) -> Cavity:
    """The 13-sphere spiral of the paper's experiments (Sec. 6) as a
    non-convex, open radiation surface: geodesic spheres of frequency ``nu``
    (20 nu^2 facets each; nu = 2, 3, 5, 6, 8, 10, 12 give 1,040-37,440 facets
    in all, spanning the paper's mesh levels) with outward normals;
    emissivity ``eps`` uniform; the central sphere at 1000 K and the others at
    300 K (the paper's initial state); ambient at ``T_amb``.  About 8% of the
    facets see no other facet (zero rows of F)."""
    v, tri, sid = meshes.fibonacci_spheres(nu, radius)
    n = tri.shape[0]
    T = np.where(sid == 0, 1000.0, 300.0)
    return Cavity(f"fibonacci_spiral_{n}", v, tri, np.full(n, eps), T[:, None],
                  extra={"sphere": sid, "T_amb": T_amb})
