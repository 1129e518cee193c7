"""ctypes binding of ``libhmrad.so`` (the C ABI declared in ``include/hm.h``).

Argument marshalling only: every step of the path runs in the library's HIP
kernels and C++ host code.  Device arrays are torch tensors on the GPU;
host arrays are numpy arrays.  Importing this module loads the library and
fails loudly when it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

# torch is imported before the library is opened: torch loads its own HIP
# runtime (SONAME libamdhip64.so.7), and the library's dependency on that
# SONAME then binds to the same runtime instead of loading a second copy.
import torch  # noqa: E402,F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhmrad.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libhmrad.so is not built; run `python -m paper_2305_06891_amd.build` "
        "(there is no fallback implementation)")
lib = C.CDLL(LIB_PATH)

HM_OK, HM_EINVAL, HM_ENOMEM, HM_ENOTCONV, HM_EDEVICE, HM_EBUSY, HM_ENOTFOUND = range(7)
HM_F64, HM_F32, HM_BF16 = 0, 1, 2
SIGMA = 5.670374e-8

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_vp = C.c_void_p


class hm_tree_params(C.Structure):
    _fields_ = [("leaf_size", C.c_int32), ("eta", C.c_double)]


class hm_assembly_params(C.Structure):
    _fields_ = [("aca_tol", C.c_double), ("k_max", C.c_int32), ("lowrank_dtype", C.c_int),
                ("dense_dtype", C.c_int), ("keep_f32_copy", C.c_int32), ("closed_row_scale", C.c_int32),
                ("autotune", C.c_int32), ("recompress", C.c_int32), ("aca_pivot", C.c_int32),
                ("lowrank_rounding", C.c_int32)]


class hm_solve_params(C.Structure):
    _fields_ = [("rtol", C.c_double), ("restart", C.c_int32), ("max_iter", C.c_int32),
                ("mixed_precision", C.c_int32), ("ir_inner_rtol", C.c_double), ("want_q", C.c_int32),
                ("vec_dtype", C.c_int32), ("use_graphs", C.c_int32), ("open_cavity", C.c_int32),
                ("ambient_temperature", C.c_double)]


class hm_fe_params(C.Structure):
    _fields_ = [("conductance", C.c_double), ("capacity", C.c_double), ("dt", C.c_double),
                ("newton_rtol", C.c_double), ("max_newton", C.c_int32), ("krylov_restart", C.c_int32),
                ("krylov_rtol", C.c_double), ("max_krylov", C.c_int32), ("pc_rtol", C.c_double),
                ("solve", hm_solve_params), ("sigma", C.c_double)]


class hm_fe_info(C.Structure):
    _fields_ = [("newton", C.c_int32), ("krylov", C.c_int32), ("cavity_solves", C.c_int32),
                ("pc_iterations", C.c_int32), ("residual", C.c_double), ("status", C.c_int32)]


class hm_solve_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer_iters", C.c_int32), ("matvecs", C.c_int32),
                ("rel_residual", C.c_double), ("seconds", C.c_double), ("bytes_moved", C.c_int64)]


class hm_transient_params(C.Structure):
    _fields_ = [("mc", C.c_double), ("dt", C.c_double), ("steps", C.c_int32), ("newton_rtol", C.c_double),
                ("max_newton", C.c_int32)]


class hm_transient_info(C.Structure):
    _fields_ = [("steps_done", C.c_int32), ("newton_total", C.c_int32), ("newton_max", C.c_int32),
                ("matvecs", C.c_int32), ("seconds", C.c_double), ("max_rel_residual", C.c_double)]


class hm_server_params(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("max_active", C.c_int32), ("max_rhs_per_slot", C.c_int32),
                ("solve", hm_solve_params), ("sigma", C.c_double)]


class hm_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("rejected", C.c_int64),
                ("assemblies", C.c_int64), ("evictions", C.c_int64), ("cache_hits", C.c_int64),
                ("rounds", C.c_int64), ("busy_seconds", C.c_double), ("resident_bytes", C.c_int64)]


# ---------------------------------------------------------------- prototypes
_PROTOS = {
    "hm_ctx_create": (C.c_int, [C.c_int, _vp, C.POINTER(_vp)]),
    "hm_ctx_destroy": (None, [_vp]),
    "hm_ctx_synchronize": (C.c_int, [_vp]),
    "hm_status_string": (C.c_char_p, [C.c_int]),
    "hm_last_error": (C.c_char_p, [_vp]),
    "hm_version": (C.c_char_p, []),
    "hm_facets_from_triangles": (C.c_int, [C.c_int64, _dp, C.c_int64, _ip, C.c_int, _dp, _dp, _dp]),
    "hm_build_cluster_tree": (C.c_int, [_vp, C.c_int64, _dp, _dp, _dp, C.POINTER(hm_tree_params), C.POINTER(_vp)]),
    "hm_tree_stats": (C.c_int, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64), _ip]),
    "hm_tree_blocks": (C.c_int, [_vp, _ip, _ip]),
    "hm_tree_destroy": (None, [_vp]),
    "hm_assemble_hmatrix": (C.c_int, [_vp, _vp, C.POINTER(hm_assembly_params), C.POINTER(_vp)]),
    "hm_assemble_hmatrix_batched": (C.c_int, [_vp, C.c_int32, C.POINTER(_vp), C.POINTER(hm_assembly_params),
                                              C.POINTER(_vp)]),
    "hm_matrix_stats": (C.c_int, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                  C.POINTER(C.c_int32)]),
    "hm_matrix_info": (C.c_int, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                 C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "hm_matrix_tuning": (C.c_int, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), _dp]),
    "hm_matrix_set_tuning": (C.c_int, [_vp, _vp, C.c_int32, C.c_int32]),
    "hm_matrix_tuning_phase2": (C.c_int, [_vp, C.POINTER(C.c_int32), _dp]),
    "hm_matrix_set_tuning_phase2": (C.c_int, [_vp, _vp, C.c_int32]),
    "hm_matrix_destroy": (None, [_vp]),
    "hm_hmatvec": (C.c_int, [_vp, _vp, C.c_int32, C.c_int, _vp, C.c_int64, _vp, C.c_int64, C.c_double,
                             C.c_double]),
    "hm_hmatvec_ex": (C.c_int, [_vp, _vp, C.c_int32, C.c_int, C.c_int32, _vp, C.c_int64, _vp, C.c_int64,
                                C.c_double, C.c_double]),
    "hm_hmatvec_noalloc": (C.c_int, [_vp, _vp, C.c_int32, C.c_int, _vp, C.c_int64, _vp, C.c_int64, C.c_double,
                                     C.c_double]),
    "hm_hmatvec_profile": (C.c_int, [_vp, C.c_int32, C.POINTER(_vp), C.c_int32, C.c_int, C.c_int32, C.c_int32,
                                     C.c_int64,
                                     _dp, _dp, _dp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "hm_solve_radiosity": (C.c_int, [_vp, _vp, _vp, C.c_int32, _vp, C.c_int64, C.c_double,
                                     C.POINTER(hm_solve_params), _vp, C.c_int64, _vp, C.c_int64,
                                     C.POINTER(hm_solve_info)]),
    "hm_solve_radiosity_batched": (C.c_int, [_vp, C.c_int32, C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp),
                                             C.c_double, C.POINTER(hm_solve_params), C.POINTER(_vp),
                                             C.POINTER(_vp), C.POINTER(hm_solve_info)]),
    "hm_transient_run": (C.c_int, [_vp, _vp, _vp, C.c_int32, _vp, C.c_int64, _vp, C.c_int64, C.c_double,
                                   C.POINTER(hm_transient_params), C.POINTER(hm_solve_params), _vp,
                                   C.POINTER(hm_transient_info)]),
    "hm_hlu_factor": (C.c_int, [_vp, _vp, _vp, C.POINTER(hm_assembly_params), C.POINTER(_vp)]),
    "hm_hlu_solve": (C.c_int, [_vp, _vp, C.c_int32, _vp, C.c_int64, _vp, C.c_int64]),
    "hm_hlu_stats": (C.c_int, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                               C.POINTER(C.c_double)]),
    "hm_hlu_destroy": (None, [_vp]),
    "hm_fe_create": (C.c_int, [_vp, _vp, C.c_int64, _dp, C.c_int64, C.POINTER(C.c_int32), _vp,
                               C.POINTER(hm_fe_params), C.POINTER(_vp)]),
    "hm_fe_cavity_load": (C.c_int, [_vp, _vp, _vp, _vp]),
    "hm_fe_step": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.POINTER(hm_fe_info)]),
    "hm_fe_destroy": (None, [_vp]),
    "hm_server_create": (C.c_int, [_vp, C.POINTER(hm_server_params), C.POINTER(_vp)]),
    "hm_server_register_cavity": (C.c_int, [_vp, C.c_uint64, _vp, _dp, C.POINTER(hm_assembly_params)]),
    "hm_submit": (C.c_int, [_vp, C.c_uint64, C.c_int32, _dp, C.POINTER(C.c_uint64)]),
    "hm_poll": (C.c_int, [_vp, C.c_uint64, C.POINTER(C.c_int32), _dp, _dp, C.POINTER(hm_solve_info),
                          C.POINTER(C.c_double)]),
    "hm_server_stats_get": (C.c_int, [_vp, C.POINTER(hm_server_stats)]),
    "hm_server_destroy": (None, [_vp]),
}

for _name, (_res, _args) in _PROTOS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_PROTOS)


class HMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (lib.hm_status_string(status).decode(), msg))
        self.status = status


def _check(st, ctx=None):
    if st != HM_OK:
        raise HMError(st, (lib.hm_last_error(ctx) or b"").decode())


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t)


def _dev_ptr(t, dtype=None):
    """Device pointer of a CUDA/HIP torch tensor (must be on the GPU)."""
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError("expected dtype %s, got %s" % (dtype, t.dtype))
    return C.c_void_p(t.data_ptr())


def _ld(t):
    """Leading dimension of an n or n x r column-major view (torch tensor)."""
    if t.dim() == 1:
        return t.shape[0]
    if t.stride(0) != 1:
        raise ValueError("right-hand sides must be column-major (stride(0) == 1)")
    return t.stride(1) if t.shape[1] > 1 else t.shape[0]


# ---------------------------------------------------------------- objects
class Context:
    """``hm_ctx`` bound to a GPU and (by default) torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        self.device = device
        self._h = _vp()
        _check(lib.hm_ctx_create(device, C.c_void_p(stream), C.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def synchronize(self):
        _check(lib.hm_ctx_synchronize(self._h), self._h)

    def close(self):
        if self._h:
            lib.hm_ctx_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hm_facets_from_triangles(v, tri, orient: int = 1):
    """Host FP64 facet centroid, unit normal and area of each triangle."""
    v = _f64(v)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    nt = tri.shape[0]
    c = np.empty((nt, 3))
    n = np.empty((nt, 3))
    a = np.empty(nt)
    _check(lib.hm_facets_from_triangles(v.shape[0], _ptr(v), nt, _ptr(tri, _ip), orient, _ptr(c), _ptr(n),
                                        _ptr(a)))
    return c, n, a


class Tree:
    """``hm_tree``: Algorithm 1 index tree and Algorithm 2 block tree (host)."""

    def __init__(self, handle, n):
        self._h = handle
        self.n = n

    def stats(self):
        nn, nd, nl = C.c_int64(), C.c_int64(), C.c_int64()
        perm = np.empty(self.n, dtype=np.int32)
        _check(lib.hm_tree_stats(self._h, C.byref(nn), C.byref(nd), C.byref(nl), _ptr(perm, _ip)))
        return {"n_nodes": nn.value, "n_dense": nd.value, "n_lowrank": nl.value, "perm": perm}

    def blocks(self):
        s = self.stats()
        d = np.empty((s["n_dense"], 4), dtype=np.int32)
        l = np.empty((s["n_lowrank"], 4), dtype=np.int32)
        _check(lib.hm_tree_blocks(self._h, _ptr(d, _ip), _ptr(l, _ip)))
        return d, l

    def close(self):
        if self._h:
            lib.hm_tree_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hm_build_cluster_tree(ctx, centroid, normal, area, leaf_size: int, eta: float) -> Tree:
    c = _f64(centroid)
    n = _f64(normal)
    a = _f64(area)
    p = hm_tree_params(int(leaf_size), float(eta))
    h = _vp()
    ch = ctx.handle if ctx is not None else None
    _check(lib.hm_build_cluster_tree(ch, a.shape[0], _ptr(c), _ptr(n), _ptr(a), C.byref(p), C.byref(h)), ch)
    return Tree(h, a.shape[0])


class HMatrix:
    """``hm_matrix``: the assembled H-matrix on the device."""

    def __init__(self, handle, ctx):
        self._h = handle
        self.ctx = ctx

    def stats(self):
        b, ed, el, mr = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int32()
        _check(lib.hm_matrix_stats(self._h, C.byref(b), C.byref(ed), C.byref(el), C.byref(mr)))
        n, nd, nl, nf, rs = (C.c_int64() for _ in range(5))
        _check(lib.hm_matrix_info(self._h, C.byref(n), C.byref(nd), C.byref(nl), C.byref(nf), C.byref(rs)))
        return {"bytes_device": b.value, "entries_dense": ed.value, "entries_lowrank": el.value,
                "max_rank": mr.value, "n": n.value, "n_dense_blocks": nd.value, "n_lowrank_blocks": nl.value,
                "n_fallback": nf.value, "rank_sum": rs.value}

    def tuning(self):
        """Work split of the product's first kernel (rows per item, bytes per
        wave task) and its measured time in microseconds (0: not timed)."""
        r, tb, us = C.c_int32(), C.c_int32(), C.c_double()
        _check(lib.hm_matrix_tuning(self._h, C.byref(r), C.byref(tb), C.byref(us)))
        w, us2 = C.c_int32(), C.c_double()
        _check(lib.hm_matrix_tuning_phase2(self._h, C.byref(w), C.byref(us2)))
        return {"p1_rows": r.value, "p1_task_bytes": tb.value, "p1_us": us.value, "p2_waves": w.value,
                "p2_us": us2.value}

    def set_tuning(self, ctx, p1_rows, p1_task_bytes):
        """Sets the work split of the product's first kernel (the values
        ``tuning()`` reports)."""
        _check(lib.hm_matrix_set_tuning(ctx._h, self._h, int(p1_rows), int(p1_task_bytes)))

    def set_tuning_phase2(self, ctx, p2_waves):
        """Sets the second kernel's waves per workgroup (0: by tile count,
        2, 4 or 8) for products of one or two columns."""
        _check(lib.hm_matrix_set_tuning_phase2(ctx._h, self._h, int(p2_waves)))

    def close(self):
        if self._h:
            lib.hm_matrix_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hm_assemble_hmatrix(ctx, tree: Tree, aca_tol=1e-6, k_max=256, lowrank_dtype=HM_F32, dense_dtype=HM_F32,
                        keep_f32_copy=0, closed_row_scale=0, autotune=0, recompress=0, aca_pivot=0,
                        lowrank_rounding=0) -> HMatrix:
    p = hm_assembly_params(float(aca_tol), int(k_max), int(lowrank_dtype), int(dense_dtype), int(keep_f32_copy),
                           int(closed_row_scale), int(autotune), int(recompress), int(aca_pivot),
                           int(lowrank_rounding))
    h = _vp()
    _check(lib.hm_assemble_hmatrix(ctx.handle, tree._h, C.byref(p), C.byref(h)), ctx.handle)
    return HMatrix(h, ctx)


def hm_assemble_hmatrix_batched(ctx, trees, aca_tol=1e-6, k_max=256, lowrank_dtype=HM_F32, dense_dtype=HM_F32,
                                keep_f32_copy=0, closed_row_scale=0, autotune=0, recompress=0, aca_pivot=0,
                                lowrank_rounding=0):
    """Matrices of several cavities assembled together (shared ACA launches;
    with autotune, one product split tuned on their batched product).  Every
    parameter is a scalar for all cavities or a sequence with one entry per
    tree."""
    trees = list(trees)
    k = len(trees)

    def each(v):
        return list(v) if isinstance(v, (list, tuple)) else [v] * k

    cols = [each(aca_tol), each(k_max), each(lowrank_dtype), each(dense_dtype), each(keep_f32_copy),
            each(closed_row_scale), each(autotune), each(recompress), each(aca_pivot), each(lowrank_rounding)]
    if any(len(c) != k for c in cols):
        raise ValueError("one parameter value per tree expected")
    ps = (hm_assembly_params * k)(*[hm_assembly_params(float(a), int(b), int(c), int(d), int(e), int(f), int(g),
                                                       int(h), int(i), int(j))
                                    for a, b, c, d, e, f, g, h, i, j in zip(*cols)])
    ts = (_vp * k)(*[t._h for t in trees])
    hs = (_vp * k)()
    _check(lib.hm_assemble_hmatrix_batched(ctx.handle, k, ts, ps, hs), ctx.handle)
    return [HMatrix(_vp(h), ctx) for h in hs]


def hm_hmatvec(ctx, M: HMatrix, X, Y, alpha=1.0, beta=0.0, use_f32_copy=False):
    """Y = alpha F_H X + beta Y; X, Y device tensors (n or n x r, float64/float32)."""
    import torch
    vt = {torch.float64: HM_F64, torch.float32: HM_F32}[X.dtype]
    nr = 1 if X.dim() == 1 else X.shape[1]
    _check(lib.hm_hmatvec_ex(ctx.handle, M._h, nr, vt, int(use_f32_copy), _dev_ptr(X), _ld(X), _dev_ptr(Y, X.dtype),
                             _ld(Y), float(alpha), float(beta)), ctx.handle)
    return Y


def hm_hmatvec_noalloc(ctx, M: HMatrix, X, Y, alpha=1.0, beta=0.0):
    """Y = alpha F_H X + beta Y with the library's fixed device scratch (no
    allocation); X, Y device tensors (n or n x r, float64/float32)."""
    import torch
    vt = {torch.float64: HM_F64, torch.float32: HM_F32}[X.dtype]
    nr = 1 if X.dim() == 1 else X.shape[1]
    _check(lib.hm_hmatvec_noalloc(ctx.handle, M._h, nr, vt, _dev_ptr(X), _ld(X), _dev_ptr(Y, X.dtype), _ld(Y),
                                  float(alpha), float(beta)), ctx.handle)
    return Y


def hm_hmatvec_profile(ctx, M, nrhs=1, vec_dtype=HM_F32, use_f32_copy=False, reps=20,
                       flush_bytes=512 << 20):
    """Average per-kernel times (HIP events on ctx's stream) and algorithmic
    bytes of the two product kernels; M is one HMatrix or a list of them
    (applied as one block-diagonal operator)."""
    Ms = list(M) if isinstance(M, (list, tuple)) else [M]
    marr = (C.c_void_p * len(Ms))(*[m._h for m in Ms])
    m1, m2, mt = C.c_double(), C.c_double(), C.c_double()
    b1, b2 = C.c_int64(), C.c_int64()
    _check(lib.hm_hmatvec_profile(ctx.handle, len(Ms), marr, int(nrhs), int(vec_dtype), int(use_f32_copy),
                                  int(reps), int(flush_bytes), C.byref(m1), C.byref(m2), C.byref(mt),
                                  C.byref(b1), C.byref(b2)), ctx.handle)
    return {"ms_phase1": m1.value, "ms_phase2": m2.value, "ms_total": mt.value, "bytes_phase1": b1.value,
            "bytes_phase2": b2.value}


def solve_params(rtol=1e-12, restart=30, max_iter=1000, mixed_precision=0, ir_inner_rtol=1e-4, want_q=1,
                 vec_dtype=HM_F64, use_graphs=1, open_cavity=0, ambient_temperature=0.0):
    return hm_solve_params(float(rtol), int(restart), int(max_iter), int(mixed_precision), float(ir_inner_rtol),
                           int(want_q), int(vec_dtype), int(use_graphs), int(open_cavity),
                           float(ambient_temperature))


def _info_dict(i: hm_solve_info):
    return {"iters": i.iters, "outer_iters": i.outer_iters, "matvecs": i.matvecs, "rel_residual": i.rel_residual,
            "seconds": i.seconds, "bytes_moved": i.bytes_moved}


def hm_solve_radiosity(ctx, M: HMatrix, eps, T, sigma=SIGMA, params=None, J=None, q=None, want_q=True):
    """Radiosity J (and flux q) for temperatures T (device float64, n or n x r)."""
    import torch
    p = params if params is not None else solve_params(want_q=int(want_q))
    if J is None:
        J = torch.empty_like(T)
    if q is None and want_q:
        q = torch.empty_like(T)
    nr = 1 if T.dim() == 1 else T.shape[1]
    info = hm_solve_info()
    st = lib.hm_solve_radiosity(ctx.handle, M._h, _dev_ptr(eps, torch.float64), nr, _dev_ptr(T, torch.float64),
                                _ld(T), float(sigma), C.byref(p), _dev_ptr(J, torch.float64), _ld(J),
                                _dev_ptr(q, torch.float64) if q is not None else None,
                                _ld(q) if q is not None else _ld(J), C.byref(info))
    if st not in (HM_OK, HM_ENOTCONV):
        _check(st, ctx.handle)
    d = _info_dict(info)
    d["status"] = st
    return J, q, d


def hm_solve_radiosity_batched(ctx, Ms, eps_list, T_list, sigma=SIGMA, params=None, J_list=None, q_list=None,
                               want_q=True):
    """One batched solve over several cavities (one right-hand side each)."""
    import torch
    k = len(Ms)
    p = params if params is not None else solve_params(want_q=int(want_q))
    if J_list is None:
        J_list = [torch.empty_like(t) for t in T_list]
    if q_list is None and want_q:
        q_list = [torch.empty_like(t) for t in T_list]
    arr = lambda xs: (C.c_void_p * k)(*[(C.c_void_p(x.data_ptr()) if x is not None else None) for x in xs])
    marr = (C.c_void_p * k)(*[m._h for m in Ms])
    infos = (hm_solve_info * k)()
    st = lib.hm_solve_radiosity_batched(ctx.handle, k, marr, arr(eps_list), arr(T_list), float(sigma), C.byref(p),
                                        arr(J_list), arr(q_list) if q_list is not None else None, infos)
    if st not in (HM_OK, HM_ENOTCONV):
        _check(st, ctx.handle)
    return J_list, q_list, [dict(_info_dict(i), status=st) for i in infos]


def hm_transient_run(ctx, M: HMatrix, eps, T, src, sigma=SIGMA, mc=1.0e4, dt=1.0, steps=1, newton_rtol=1e-9,
                     max_newton=30, params=None, history=None):
    """Implicit-Euler lumped transient; T (device float64 n x r) is updated in place."""
    import torch
    tp = hm_transient_params(float(mc), float(dt), int(steps), float(newton_rtol), int(max_newton))
    p = params if params is not None else solve_params(rtol=1e-12, want_q=1)
    nr = 1 if T.dim() == 1 else T.shape[1]
    info = hm_transient_info()
    _check(lib.hm_transient_run(ctx.handle, M._h, _dev_ptr(eps, torch.float64), nr, _dev_ptr(T, torch.float64),
                                _ld(T), _dev_ptr(src, torch.float64), _ld(src), float(sigma), C.byref(tp),
                                C.byref(p), _dev_ptr(history, torch.float64) if history is not None else None,
                                C.byref(info)), ctx.handle)
    return T, {"steps_done": info.steps_done, "newton_total": info.newton_total, "newton_max": info.newton_max,
               "matvecs": info.matvecs, "seconds": info.seconds, "max_rel_residual": info.max_rel_residual}


class HLU:
    """Factors C ~ L U of the reflection matrix (``hm_hlu_factor``)."""

    def __init__(self, h, ctx, n):
        self._h = h
        self.ctx = ctx
        self.n = n

    def solve(self, B, X=None):
        """X = U^-1 (L^-1 B) for a device float64 tensor B (n or n x r)."""
        import torch
        if X is None:
            X = torch.empty_like(B)
        nr = 1 if B.dim() == 1 else B.shape[1]
        _check(lib.hm_hlu_solve(self.ctx.handle, self._h, nr, _dev_ptr(B, torch.float64), _ld(B),
                                _dev_ptr(X, torch.float64), _ld(X)), self.ctx.handle)
        return X

    def stats(self):
        b, e, mr, sec = C.c_int64(), C.c_int64(), C.c_int32(), C.c_double()
        _check(lib.hm_hlu_stats(self._h, C.byref(b), C.byref(e), C.byref(mr), C.byref(sec)))
        return {"bytes_device": b.value, "entries": e.value, "max_rank": mr.value, "factor_seconds": sec.value}

    def close(self):
        if self._h:
            lib.hm_hlu_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FE:
    """Finite-element coupling of a conducting shell with the cavity
    (``hm_fe_create``): nodal temperatures, radiation load and implicit
    Euler steps."""

    def __init__(self, h, ctx, n_nodes, n_facets):
        self._h = h
        self.ctx = ctx
        self.n_nodes = n_nodes
        self.n_facets = n_facets

    def cavity_load(self, T, Q=None):
        """Q = S T^4 for device float64 nodal temperatures T."""
        import torch
        if Q is None:
            Q = torch.empty_like(T)
        _check(lib.hm_fe_cavity_load(self.ctx.handle, self._h, _dev_ptr(T, torch.float64),
                                     _dev_ptr(Q, torch.float64)), self.ctx.handle)
        return Q

    def step(self, T_n, f_facet=None, T_out=None, check=True):
        """One implicit Euler step; returns (T_out, info dict)."""
        import torch
        if T_out is None:
            T_out = torch.empty_like(T_n)
        info = hm_fe_info()
        fp = _dev_ptr(f_facet, torch.float64) if f_facet is not None else None
        st = lib.hm_fe_step(self.ctx.handle, self._h, _dev_ptr(T_n, torch.float64), fp,
                            _dev_ptr(T_out, torch.float64), C.byref(info))
        if check:
            _check(st, self.ctx.handle)
        return T_out, {"newton": info.newton, "krylov": info.krylov, "cavity_solves": info.cavity_solves,
                       "pc_iterations": info.pc_iterations, "residual": info.residual, "status": info.status}

    def close(self):
        if self._h:
            lib.hm_fe_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fe_params(conductance, capacity, dt, newton_rtol=1e-12, max_newton=20, krylov_restart=30, krylov_rtol=1e-10,
              max_krylov=200, pc_rtol=1e-12, solve=None, sigma=None) -> hm_fe_params:
    return hm_fe_params(float(conductance), float(capacity), float(dt), float(newton_rtol), int(max_newton),
                        int(krylov_restart), float(krylov_rtol), int(max_krylov), float(pc_rtol),
                        solve if solve is not None else solve_params(rtol=1e-12),
                        float(SIGMA if sigma is None else sigma))


def hm_fe_create(ctx, M: "HMatrix", vertices, triangles, eps, params: hm_fe_params) -> FE:
    """vertices (n_nodes x 3) and triangles (n_facets x 3) on the host, eps a
    device float64 vector in facet order; M the H-matrix of those facets."""
    import torch
    v = np.ascontiguousarray(vertices, dtype=np.float64)
    t = np.ascontiguousarray(triangles, dtype=np.int32)
    h = _vp()
    _check(lib.hm_fe_create(ctx.handle, M._h, v.shape[0], v.ctypes.data_as(_dp), t.shape[0],
                            t.ctypes.data_as(C.POINTER(C.c_int32)), _dev_ptr(eps, torch.float64),
                            C.byref(params), C.byref(h)), ctx.handle)
    return FE(h, ctx, v.shape[0], t.shape[0])


def hm_hlu_factor(ctx, tree: Tree, eps, aca_tol=1e-6, k_max=256, aca_pivot=0) -> HLU:
    """Hierarchical block LU of C = I - diag(1 - eps) F (eps: device float64,
    caller order)."""
    import torch
    p = hm_assembly_params(float(aca_tol), int(k_max), HM_F64, HM_F64, 0, 0, 0, 0, int(aca_pivot), 0)
    h = _vp()
    _check(lib.hm_hlu_factor(ctx.handle, tree._h, _dev_ptr(eps, torch.float64), C.byref(p), C.byref(h)), ctx.handle)
    return HLU(h, ctx, tree.n)


class Server:
    """``hm_server``: continuous-batching radiosity solves with resident H-matrices."""

    def __init__(self, ctx, hbm_budget_bytes=64 << 30, max_active=64, max_rhs_per_slot=8, params=None,
                 sigma=SIGMA):
        p = params if params is not None else solve_params(rtol=1e-7, want_q=1)
        sp = hm_server_params(int(hbm_budget_bytes), int(max_active), int(max_rhs_per_slot), p, float(sigma))
        self._h = _vp()
        self.ctx = ctx
        _check(lib.hm_server_create(ctx.handle, C.byref(sp), C.byref(self._h)), ctx.handle)
        self._n = {}

    def register_cavity(self, cavity_id, tree: Tree, eps_host, aca_tol=1e-6, k_max=256, lowrank_dtype=HM_BF16,
                        dense_dtype=HM_F32, keep_f32_copy=1, autotune=0, recompress=0, aca_pivot=0,
                        lowrank_rounding=0):
        e = _f64(eps_host)
        ap = hm_assembly_params(float(aca_tol), int(k_max), int(lowrank_dtype), int(dense_dtype),
                                int(keep_f32_copy), 0, int(autotune), int(recompress), int(aca_pivot),
                                int(lowrank_rounding))
        _check(lib.hm_server_register_cavity(self._h, C.c_uint64(cavity_id), tree._h, _ptr(e), C.byref(ap)))
        self._n[cavity_id] = tree.n

    def submit(self, cavity_id, T_host):
        T = np.asfortranarray(T_host, dtype=np.float64)
        if T.ndim == 1:
            T = T[:, None]
        t = C.c_uint64()
        _check(lib.hm_submit(self._h, C.c_uint64(cavity_id), T.shape[1], T.ctypes.data_as(_dp), C.byref(t)))
        return t.value, T.shape

    def poll(self, ticket, shape):
        done = C.c_int32()
        J = np.empty(shape, order="F")
        q = np.empty(shape, order="F")
        info = hm_solve_info()
        lat = C.c_double()
        st = lib.hm_poll(self._h, C.c_uint64(ticket), C.byref(done), J.ctypes.data_as(_dp), q.ctypes.data_as(_dp),
                         C.byref(info), C.byref(lat))
        if st == HM_EBUSY:
            return None
        _check(st)
        return J, q, dict(_info_dict(info), latency=lat.value)

    def stats(self):
        s = hm_server_stats()
        _check(lib.hm_server_stats_get(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in s._fields_}

    def close(self):
        if self._h:
            lib.hm_server_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
