"""Facet geometry from a triangle mesh (oracle; test infrastructure only).

The radiation surface is a set of flat facets (Sec. 3.1); the view factor of
eq. (10) needs each facet's area, centroid and plane normal (Sec. 3.2).
"""
from __future__ import annotations

import numpy as np


def facets_from_triangles(v: np.ndarray, tri: np.ndarray):
    """Centroid (mean of the corners), unit right-hand normal and area of
    every triangle, in FP64.

    The normal follows the triangle winding: (b - a) x (c - a), normalised.
    Returns (centroid (n,3), normal (n,3), area (n,)).
    """
    v = np.asarray(v, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.int64)
    a = v[tri[:, 0]]
    b = v[tri[:, 1]]
    c = v[tri[:, 2]]
    centroid = (a + b + c) / 3.0
    cr = np.cross(b - a, c - a)
    twice_area = np.sqrt(np.sum(cr * cr, axis=1))
    normal = cr / twice_area[:, None]
    return centroid, normal, 0.5 * twice_area
