"""Large-n mode of the oracle: the same dense definition without storing F
(test infrastructure only).

For cavities whose dense F does not fit in host memory (8 n^2 bytes: 320 GB
at 200,000 facets), products with the centroid-rule view factors of
eq. (10) are evaluated on the fly by a plain C kernel (``vf_matfree.c``,
FP64, every entry computed exactly as ``viewfactor.py`` computes it), and the
reflection system of eq. (11), ``C J = sigma eps T^4`` with
``C = I - diag(1 - eps) F``, is solved by restarted GMRES instead of LU.

GMRES(m) here is the textbook method: Arnoldi with classical Gram-Schmidt
applied twice (CGS2), Givens rotations on the Hessenberg matrix, restart
after m steps, and a stop when the TRUE residual ``|b - C x|_2`` is at most
``rtol |b|_2`` (checked at every restart and at the end).  Every column of a
multi-column right-hand side runs its own independent GMRES; the columns
only share the product calls.

The flux follows eq. (12) as in ``radiosity.DenseRadiosity``:
``q = eps (F J - sigma T^4 g)`` with ``g = F C^-1 eps``.
"""
from __future__ import annotations

import ctypes as C
import hashlib
import os
import subprocess
import tempfile

import numpy as np

from .radiosity import SIGMA

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vf_matfree.c")
_lib = None


def _host_tag() -> str:
    """The library is built with -march=native, so it is keyed by the host
    CPU's model and flags (a copy built on another machine is never loaded)."""
    try:
        with open("/proc/cpuinfo") as f:
            lines = [ln for ln in f if ln.startswith(("model name", "flags"))][:2]
    except OSError:
        lines = []
    with open(_SRC, "rb") as f:
        src = f.read()
    return hashlib.sha1(("".join(lines)).encode() + src).hexdigest()[:12]


def library_path() -> str:
    return os.path.join(_HERE, "_build", "vf_matfree_%s.so" % _host_tag())


def build(force: bool = False) -> str:
    """Compile ``vf_matfree.c`` for this host (gcc, OpenMP, no contraction)."""
    out = library_path()
    if os.path.exists(out) and not force:
        return out
    os.makedirs(os.path.dirname(out), exist_ok=True)
    fd, tmp = tempfile.mkstemp(suffix=".so", dir=os.path.dirname(out))
    os.close(fd)
    cmd = ["gcc", "-O2", "-march=native", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-o", tmp, _SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        os.unlink(tmp)
        raise RuntimeError("oracle build failed: %s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, out)
    return out


def load(path: str | None = None):
    """The product library (this host's build of ``vf_matfree.c`` unless
    ``path`` names another build of the same interface)."""
    global _lib
    if path is None and _lib is not None:
        return _lib
    lib = C.CDLL(path or build())
    dp = C.POINTER(C.c_double)
    lib.vf_matvec.restype = None
    lib.vf_matvec.argtypes = [C.c_int64] + [dp] * 7 + [C.c_int64, dp, dp]
    if path is None:
        _lib = lib
    return lib


class MatrixFreeF:
    """``Y = F X`` with the centroid-rule view factors, evaluated on the fly."""

    def __init__(self, c, nrm, area, lib=None):
        self.lib = lib
        self.n = int(c.shape[0])
        self._cols = [np.ascontiguousarray(a, dtype=np.float64)
                      for a in (c[:, 0], c[:, 1], c[:, 2], nrm[:, 0], nrm[:, 1], nrm[:, 2], area)]
        self.products = 0

    def __matmul__(self, X):
        X = np.asarray(X, dtype=np.float64)
        one = X.ndim == 1
        Xr = np.ascontiguousarray(X.reshape(self.n, -1))
        r = Xr.shape[1]
        Y = np.empty_like(Xr)
        lib = self.lib or load()
        dp = C.POINTER(C.c_double)
        for q0 in range(0, r, 16):
            Xq = np.ascontiguousarray(Xr[:, q0:q0 + 16])
            Yq = np.empty_like(Xq)
            lib.vf_matvec(self.n, *[a.ctypes.data_as(dp) for a in self._cols], Xq.shape[1],
                          Xq.ctypes.data_as(dp), Yq.ctypes.data_as(dp))
            Y[:, q0:q0 + 16] = Yq
        self.products += 1
        return Y[:, 0] if one else Y


def gmres(apply_a, B, X0=None, rtol=1e-13, restart=30, maxiter=1000):
    """Independent GMRES(restart) with CGS2 for every column of ``B``
    (n x r), sharing the calls of ``apply_a`` (which maps n x r to n x r).
    Returns (X, iterations, true relative residuals)."""
    B = np.asarray(B, dtype=np.float64)
    n, r = B.shape
    X = np.zeros_like(B) if X0 is None else np.array(X0, dtype=np.float64)
    bn = np.linalg.norm(B, axis=0)
    its = 0
    R = B - apply_a(X)
    rel = np.linalg.norm(R, axis=0) / bn
    while np.any(rel > rtol) and its < maxiter:
        m = min(restart, maxiter - its)
        act = rel > rtol
        beta = np.linalg.norm(R, axis=0)
        V = np.zeros((m + 1, n, r))
        H = np.zeros((r, m + 1, m))
        cs = np.zeros((r, m))
        sn = np.zeros((r, m))
        g = np.zeros((r, m + 1))
        g[:, 0] = beta
        V[0] = np.where(act, R / np.where(beta > 0, beta, 1.0), 0.0)
        done = ~act
        k_used = np.zeros(r, dtype=np.int64)
        for k in range(m):
            W = apply_a(V[k])
            its += 1
            for _ in range(2):  # classical Gram-Schmidt, twice
                h = np.einsum("jnr,nr->rj", V[:k + 1], W)
                W = W - np.einsum("jnr,rj->nr", V[:k + 1], h)
                H[:, :k + 1, k] += h
            hn = np.linalg.norm(W, axis=0)
            H[:, k + 1, k] = hn
            V[k + 1] = np.where(hn > 0, W / np.where(hn > 0, hn, 1.0), 0.0)
            for q in range(r):
                if done[q]:
                    continue
                for i in range(k):  # earlier rotations on the new column
                    a, b = H[q, i, k], H[q, i + 1, k]
                    H[q, i, k] = cs[q, i] * a + sn[q, i] * b
                    H[q, i + 1, k] = -sn[q, i] * a + cs[q, i] * b
                a, b = H[q, k, k], H[q, k + 1, k]
                d = np.hypot(a, b)
                cs[q, k], sn[q, k] = (a / d, b / d) if d > 0 else (1.0, 0.0)
                H[q, k, k] = d
                H[q, k + 1, k] = 0.0
                g[q, k + 1] = -sn[q, k] * g[q, k]
                g[q, k] = cs[q, k] * g[q, k]
                k_used[q] = k + 1
                if abs(g[q, k + 1]) <= rtol * bn[q] * 0.5:
                    done[q] = True
            if np.all(done):
                break
        for q in range(r):
            kq = k_used[q]
            if kq == 0:
                continue
            y = np.linalg.solve(np.triu(H[q, :kq, :kq]), g[q, :kq])
            X[:, q] += np.einsum("jn,j->n", V[:kq, :, q], y)
        R = B - apply_a(X)
        rel = np.linalg.norm(R, axis=0) / bn
    return X, its, rel


class MatrixFreeRadiosity:
    """Drop-in for ``radiosity.DenseRadiosity`` at large n: the same
    quantities (``eps``, ``sigma``, ``g``, ``radiosity``, ``flux``) with F
    applied on the fly and C^-1 by GMRES to ``rtol``.  A solve starts from the
    previous solution of the same shape (the result does not depend on the
    start beyond the tolerance)."""

    def __init__(self, c, nrm, area, eps, sigma=SIGMA, rtol=1e-13, restart=30):
        self.F = MatrixFreeF(c, nrm, area)
        self.eps = np.asarray(eps, dtype=np.float64)
        self.sigma = sigma
        self.rtol = rtol
        self.restart = restart
        self._last = None
        self.iterations = 0
        w = self.solve(self.eps)
        self.w = w
        self.g = self.F @ w
        self._last = None

    def apply_c(self, X):
        X = np.asarray(X, dtype=np.float64)
        return X - (1.0 - self.eps)[:, None] * (self.F @ X)

    def solve(self, b):
        b = np.asarray(b, dtype=np.float64)
        one = b.ndim == 1
        B = b.reshape(b.shape[0], -1)
        X0 = self._last if self._last is not None and self._last.shape == B.shape else B
        X, its, rel = gmres(self.apply_c, B, X0, self.rtol, self.restart)
        if np.any(rel > self.rtol):
            raise RuntimeError("matrix-free oracle: GMRES did not reach %g (%s)" % (self.rtol, rel))
        self.iterations += its
        self._last = X
        return X[:, 0] if one else X

    def radiosity(self, T):
        T = np.asarray(T, dtype=np.float64)
        e = self.eps if T.ndim == 1 else self.eps[:, None]
        return self.solve(self.sigma * e * T**4)

    def flux(self, T, J=None):
        """Eq. (12): ``q = eps (F J - sigma T^4 g)``."""
        T = np.asarray(T, dtype=np.float64)
        if J is None:
            J = self.radiosity(T)
        eta = T**4
        if T.ndim == 1:
            return self.eps * (self.F @ J - self.sigma * eta * self.g)
        return self.eps[:, None] * (self.F @ J - self.sigma * eta * self.g[:, None])
