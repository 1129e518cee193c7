"""Seeded synthetic cavity meshes.

This module only produces input data: vertex coordinates and triangle index
triples (or, for square facets, facet arrays given directly).  It holds none
of the view-factor / radiosity arithmetic; both the library and the oracle
derive centroids, normals and areas from these triangles on their own.

Winding convention: every generator emits triangles whose right-hand normal
points OUT of the enclosed volume.  ``inward(tri)`` swaps two corners so that
the right-hand normal points into the cavity, which is the orientation the
view-factor definition needs (the cosines are measured against the normal
facing the other facets).
"""
from __future__ import annotations

import math

import numpy as np

PHI = (1.0 + math.sqrt(5.0)) / 2.0


def inward(tri: np.ndarray) -> np.ndarray:
    """Reverse the winding of every triangle (outward -> inward normals)."""
    tri = np.asarray(tri)
    return np.ascontiguousarray(tri[:, [0, 2, 1]])


def _icosahedron():
    v = np.array(
        [
            [-1, PHI, 0], [1, PHI, 0], [-1, -PHI, 0], [1, -PHI, 0],
            [0, -1, PHI], [0, 1, PHI], [0, -1, -PHI], [0, 1, -PHI],
            [PHI, 0, -1], [PHI, 0, 1], [-PHI, 0, -1], [-PHI, 0, 1],
        ],
        dtype=np.float64,
    )
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array(
        [
            [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
            [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
            [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
            [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
        ],
        dtype=np.int64,
    )
    return v, _orient_outward_about_origin(v, f)


def _orient_outward_about_origin(v, f):
    """Make the winding of a star-shaped (about the origin) mesh outward."""
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    nrm = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", nrm, (a + b + c)) < 0
    f = f.copy()
    f[flip] = f[flip][:, [0, 2, 1]]
    return f


def icosphere(level: int, radius: float = 1.0):
    """Recursive icosphere: each level splits every triangle into four at the
    edge midpoints and pushes the new vertices back onto the sphere.
    ``20 * 4**level`` triangles, outward winding."""
    v, f = _icosahedron()
    verts = [tuple(p) for p in v]
    for _ in range(level):
        cache = {}

        def mid(i, j):
            key = (i, j) if i < j else (j, i)
            k = cache.get(key)
            if k is None:
                p = np.add(verts[i], verts[j]) * 0.5
                p /= np.linalg.norm(p)
                verts.append(tuple(p))
                k = len(verts) - 1
                cache[key] = k
            return k

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = np.array(nf, dtype=np.int64)
    v = np.array(verts, dtype=np.float64) * radius
    return v, f.astype(np.int32)


def geodesic(nu: int, radius: float = 1.0):
    """Geodesic sphere of frequency ``nu``: every icosahedron face is cut into
    ``nu**2`` triangles on the flat face and the grid points are then projected
    onto the sphere.  ``20 * nu**2`` triangles, outward winding.  Grid points on
    shared face edges are duplicated (identical coordinates)."""
    v0, f0 = _icosahedron()
    ii, jj = [], []
    for i in range(nu + 1):
        for j in range(nu + 1 - i):
            ii.append(i)
            jj.append(j)
    ii = np.array(ii)
    jj = np.array(jj)
    # local index of grid point (i, j)
    loc = -np.ones((nu + 1, nu + 1), dtype=np.int64)
    loc[ii, jj] = np.arange(ii.size)
    up = [(loc[i, j], loc[i + 1, j], loc[i, j + 1]) for i in range(nu) for j in range(nu - i)]
    dn = [
        (loc[i + 1, j], loc[i + 1, j + 1], loc[i, j + 1])
        for i in range(nu - 1)
        for j in range(nu - 1 - i)
    ]
    local_tri = np.array(up + dn, dtype=np.int64)
    npts = ii.size
    verts = np.empty((20 * npts, 3))
    tris = np.empty((20 * local_tri.shape[0], 3), dtype=np.int64)
    for fi, (a, b, c) in enumerate(f0):
        A, B, C = v0[a], v0[b], v0[c]
        p = A[None, :] + (ii[:, None] / nu) * (B - A)[None, :] + (jj[:, None] / nu) * (C - A)[None, :]
        p /= np.linalg.norm(p, axis=1, keepdims=True)
        verts[fi * npts:(fi + 1) * npts] = p
        tris[fi * local_tri.shape[0]:(fi + 1) * local_tri.shape[0]] = local_tri + fi * npts
    return verts * radius, tris.astype(np.int32)


def ellipsoid(nu: int, axes=(1.0, 1.0, 1.0)):
    """Geodesic sphere scaled by the semi-axes (a linear map keeps the
    winding and the convexity)."""
    v, f = geodesic(nu)
    return v * np.asarray(axes, dtype=np.float64)[None, :], f


def cylinder(n_theta=104, n_z=66, n_r=16, radius=1.0, height=4.0, jitter=0.05, seed=1):
    """Closed cylinder (side + two flat caps) from a structured grid.

    Side: ``n_theta`` x ``n_z`` quads, each cut on the (a,b)-(a+1,b+1)
    diagonal.  Caps: a centre fan of ``n_theta`` triangles, then ``n_r - 1``
    rings of quads cut on the same kind of diagonal.  Triangle count
    ``2*n_theta*n_z + 2*(n_theta + 2*n_theta*(n_r-1))`` (20,176 for the
    defaults).

    Every vertex that is neither on a rim circle nor a cap centre is moved by
    ``U[-jitter, jitter]`` times the local grid spacing in its parametric
    coordinates ((theta, z) on the side, (rho, theta) on a cap), so all
    vertices stay exactly on the cylinder surface.  Draws are taken from
    ``numpy.random.default_rng(seed)``, two per jittered vertex, in vertex
    index order.
    """
    rng = np.random.default_rng(seed)
    dth = 2.0 * math.pi / n_theta
    dz = height / n_z
    dr = radius / n_r
    z0 = -0.5 * height
    # --- vertex table in parametric form ------------------------------------
    # side rings b = 0..n_z, index side(a, b) = b*n_theta + a
    nside = (n_z + 1) * n_theta
    # bottom cap rings c = 1..n_r-1, top cap rings c = 1..n_r-1
    ncap = (n_r - 1) * n_theta
    nverts = nside + 2 * ncap + 2
    kind = np.zeros(nverts, dtype=np.int64)  # 0 side, 1 bottom cap, 2 top cap, 3 centre
    p0 = np.zeros(nverts)
    p1 = np.zeros(nverts)
    jit = np.zeros(nverts, dtype=bool)
    for b in range(n_z + 1):
        for a in range(n_theta):
            k = b * n_theta + a
            p0[k] = a * dth
            p1[k] = z0 + b * dz
            jit[k] = 0 < b < n_z
    for cap in (0, 1):
        base = nside + cap * ncap
        for c in range(1, n_r):
            for a in range(n_theta):
                k = base + (c - 1) * n_theta + a
                kind[k] = 1 + cap
                p0[k] = c * dr  # rho
                p1[k] = a * dth  # theta
                jit[k] = True
    cb = nside + 2 * ncap
    ct = cb + 1
    kind[cb] = 3
    kind[ct] = 3
    # --- jitter, two draws per jittered vertex in index order -----------------
    idx = np.nonzero(jit)[0]
    u = rng.uniform(-jitter, jitter, size=(idx.size, 2))
    side = kind[idx] == 0
    p0[idx[side]] += u[side, 0] * dth
    p1[idx[side]] += u[side, 1] * dz
    capm = ~side
    p0[idx[capm]] += u[capm, 0] * dr
    p1[idx[capm]] += u[capm, 1] * dth
    # --- Cartesian coordinates -------------------------------------------------
    v = np.zeros((nverts, 3))
    s = kind == 0
    v[s, 0] = radius * np.cos(p0[s])
    v[s, 1] = radius * np.sin(p0[s])
    v[s, 2] = p1[s]
    for cap, zc in ((1, z0), (2, z0 + height)):
        s = kind == cap
        v[s, 0] = p0[s] * np.cos(p1[s])
        v[s, 1] = p0[s] * np.sin(p1[s])
        v[s, 2] = zc
    v[cb] = (0.0, 0.0, z0)
    v[ct] = (0.0, 0.0, z0 + height)

    def side_v(a, b):
        return b * n_theta + (a % n_theta)

    def ring(cap, c, a):
        a %= n_theta
        if c == n_r:  # the rim is the side ring
            return side_v(a, 0 if cap == 0 else n_z)
        return nside + cap * ncap + (c - 1) * n_theta + a

    tris = []
    for b in range(n_z):
        for a in range(n_theta):
            v00, v10 = side_v(a, b), side_v(a + 1, b)
            v01, v11 = side_v(a, b + 1), side_v(a + 1, b + 1)
            tris.append((v00, v10, v11))
            tris.append((v00, v11, v01))
    for cap, centre in ((0, cb), (1, ct)):
        for a in range(n_theta):
            r0, r1 = ring(cap, 1, a), ring(cap, 1, a + 1)
            tris.append((centre, r1, r0) if cap == 0 else (centre, r0, r1))
        for c in range(1, n_r):
            for a in range(n_theta):
                p00, p01 = ring(cap, c, a), ring(cap, c, a + 1)
                p10, p11 = ring(cap, c + 1, a), ring(cap, c + 1, a + 1)
                if cap == 0:
                    tris.append((p00, p01, p11))
                    tris.append((p00, p11, p10))
                else:
                    tris.append((p00, p11, p01))
                    tris.append((p00, p10, p11))
    return v, np.array(tris, dtype=np.int32)


def cylinder_for_count(n_target: int, seed: int, jitter=0.05):
    """Cylinder r=1, h=4 whose grid is the 20,176-triangle grid scaled by
    sqrt(n_target / 20176) in every direction (rounded, at least 3)."""
    s = math.sqrt(n_target / 20176.0)
    nt = max(3, int(round(104 * s)))
    nz = max(1, int(round(66 * s)))
    nr = max(1, int(round(16 * s)))
    return cylinder(nt, nz, nr, 1.0, 4.0, jitter, seed)


def parallel_plates(n_per_side: int, length: float = 1.0, gap: float = 1.0):
    """Two aligned parallel L x L plates a distance ``gap`` apart, each cut into
    ``n_per_side**2`` square facets, facing each other.  Returned directly as
    facet arrays (centroid, unit normal into the gap, area) because the facets
    are squares, not triangles.  Facets of the bottom plate come first."""
    h = length / n_per_side
    c1 = (np.arange(n_per_side) + 0.5) * h
    X, Y = np.meshgrid(c1, c1, indexing="ij")
    X = X.ravel()
    Y = Y.ravel()
    m = X.size
    cen = np.zeros((2 * m, 3))
    nrm = np.zeros((2 * m, 3))
    cen[:m, 0], cen[:m, 1] = X, Y
    cen[m:, 0], cen[m:, 1], cen[m:, 2] = X, Y, gap
    nrm[:m, 2] = 1.0
    nrm[m:, 2] = -1.0
    area = np.full(2 * m, h * h)
    return cen, nrm, area


def line_points(n: int, spacing: float = 1.0):
    """``n`` equidistant points on the x axis (centroid cloud only)."""
    c = np.zeros((n, 3))
    c[:, 0] = np.arange(n) * spacing
    return c


def projected_sphere_points(n_level: int = 3, radius: float = 1.0, seed: int = 7):
    """A point set that lies exactly on a sphere: icosphere triangle centroids
    pushed radially onto the sphere, each with the inward radial unit normal
    and an arbitrary positive weight drawn from ``default_rng(seed)`` in
    ``U[0.5, 1.5] * 4*pi*R**2 / n``.  Returned as (points, normals, weights)."""
    v, tri = icosphere(n_level)
    p = (v[tri[:, 0]] + v[tri[:, 1]] + v[tri[:, 2]]) / 3.0
    d = p / np.linalg.norm(p, axis=1, keepdims=True)
    n = d.shape[0]
    w = np.random.default_rng(seed).uniform(0.5, 1.5, n) * (4.0 * math.pi * radius**2 / n)
    return radius * d, -d, w


def fibonacci_centers():
    """Centres (x, y, 0) of the 13 spheres of the spiral arrangement described
    in Sec. 6 (unit = the first Fibonacci offset), in sphere order 1..13.

    Sphere 1 sits at the origin; spheres 2, 3, 5, 7, 9, 11, 13 follow, each
    offset from the previous one of them by (+-a_n, +-a_n) with a_n the n-th
    Fibonacci number (1, 1, 2, 3, 5, 8, 13), the sign pairs turning by a
    quarter turn each time, (+,+), (-,+), (-,-), (+,-), ..., which winds the
    spiral counter-clockwise.  Consecutive ones of these are joined by
    quarter circles of radius a_n (the centre on the side that turns the arc
    counter-clockwise); spheres 4, 6, 8, 10, 12 sit at the midpoints of the
    arcs 3-5, 5-7, 7-9, 9-11, 11-13."""
    fib = [1, 1, 2, 3, 5, 8, 13]
    signs = [(1, 1), (-1, 1), (-1, -1), (1, -1)]
    main = [np.zeros(2)]
    arcs = []
    for k, a in enumerate(fib):
        sx, sy = signs[k % 4]
        prev = main[-1]
        nxt = prev + np.array([sx * a, sy * a], dtype=np.float64)
        for cen in (prev + np.array([sx * a, 0.0]), prev + np.array([0.0, sy * a])):
            u, w = prev - cen, nxt - cen
            if u[0] * w[1] - u[1] * w[0] > 0.0:  # counter-clockwise quarter turn
                mid = u + w
                arcs.append(cen + a * mid / np.linalg.norm(mid))
                break
        main.append(nxt)
    # main[0..7] are spheres 1, 2, 3, 5, 7, 9, 11, 13; arcs[k] joins main[k] and main[k+1]
    order = [main[0], main[1], main[2], arcs[2], main[3], arcs[3], main[4], arcs[4], main[5], arcs[5],
             main[6], arcs[6], main[7]]
    return np.array([[p[0], p[1], 0.0] for p in order])


def fibonacci_spheres(nu: int, radius: float = 0.5):
    """The 13-sphere spiral of Sec. 6 as one radiation surface: a geodesic
    sphere of frequency ``nu`` (20 nu^2 facets) at every centre of
    ``fibonacci_centers``, triangles wound outward (the cavity is the space
    between the spheres, so these normals already point into it).  Returns
    (vertices, triangles, sphere index of every triangle)."""
    vs, fs, ids = [], [], []
    sv, sf = geodesic(nu, radius)
    for k, cen in enumerate(fibonacci_centers()):
        fs.append(sf + sum(x.shape[0] for x in vs))
        vs.append(sv + cen[None, :])
        ids.append(np.full(sf.shape[0], k, dtype=np.int32))
    return np.concatenate(vs), np.concatenate(fs).astype(np.int32), np.concatenate(ids)
