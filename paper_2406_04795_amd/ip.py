"""Python binding of the C ABI in include/ip.h (argument marshalling only).

Every function named ip_* forwards to the entry point of the same name in
libip.so; all computation happens in the library's HIP kernels.  If the
library has not been built this module raises on import: there is no other
code path.  PyTorch is used only for device buffers and the current stream.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libip.so")

if not os.path.exists(LIBPATH):
    raise ImportError(f"{LIBPATH} is missing: build it with paper_2406_04795_amd/build.py "
                      "(or __graft_entry__.build()); there is no fallback path")

# torch first: the library then binds to the HIP runtime torch has loaded, so
# that both share one runtime (streams and device pointers pass between them)
import torch  # noqa: E402,F401

_lib = C.CDLL(LIBPATH)

IP_OK, IP_EINVAL, IP_ENOMEM, IP_ERANGE, IP_EDEVICE, IP_EAGAIN, IP_ECANCELED = 0, -1, -2, -3, -4, -5, -6
IP_FP64, IP_FP32_CERTIFY = 0, 1
IP_MAX_D = 7

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_vp = C.c_void_p


IP_KERNEL_POLY, IP_KERNEL_RBF = 0, 1


class ip_fparams(C.Structure):
    _fields_ = [("d", C.c_int32), ("degree", C.c_int32), ("n_sv", C.c_int64),
                ("gamma", C.c_double), ("coef0", C.c_double), ("bias", C.c_double),
                ("sv", _dp), ("alpha", _dp), ("kernel", C.c_int32)]


def _kernel_code(f):
    return IP_KERNEL_RBF if getattr(f, "kernel", "poly") == "rbf" else IP_KERNEL_POLY


class ip_space(C.Structure):
    _fields_ = [("d", C.c_int32), ("M", _dp), ("Minv", _dp), ("offset", _dp),
                ("lo", _dp), ("hi", _dp)]


class ip_scene(C.Structure):
    _fields_ = [("n_joints", C.c_int32), ("joint_T", _dp), ("joint_axis", _ip),
                ("n_lsph", C.c_int32), ("lsph_link", _ip), ("lsph_c", _dp), ("lsph_r", _dp),
                ("n_lcap", C.c_int32), ("lcap_link", _ip), ("lcap_p0", _dp), ("lcap_p1", _dp),
                ("lcap_r", _dp),
                ("n_osph", C.c_int32), ("osph_c", _dp), ("osph_r", _dp),
                ("n_obox", C.c_int32), ("obox_T", _dp), ("obox_l", _dp),
                ("n_ocyl", C.c_int32), ("ocyl_T", _dp), ("ocyl_rh", _dp)]


class ip_stats(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_vertices", C.c_int64), ("n_fallback", C.c_int64),
                ("n_settled64", C.c_int64),
                ("n_cofaces", C.c_int64), ("n_sigma", C.c_int64), ("n_batches", C.c_int64),
                ("n_template_edges", C.c_int64), ("levels", C.c_int32), ("regrows", C.c_int32),
                ("ms_total", C.c_double), ("ms_feval", C.c_double), ("ms_expand", C.c_double),
                ("ms_points", C.c_double), ("ms_check", C.c_double), ("ms_subdivide", C.c_double),
                ("subdivide_launches", C.c_int64), ("n_edge_hits", C.c_int64),
                ("n_coarse_edges", C.c_int64), ("n_shared_probes", C.c_int64),
                ("ms_sigma", C.c_double), ("n_ncofaces", C.c_int64), ("n_hip_malloc", C.c_int64), ("hip_malloc_bytes", C.c_int64),
                ("ms_refine", C.c_double), ("refine_iters", C.c_int32), ("pad0", C.c_int32),
                ("ms_prep", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ip_request(C.Structure):
    _fields_ = [("f", C.POINTER(ip_fparams)), ("sp", C.POINTER(ip_space)), ("seeds", _dp),
                ("n_seeds", C.c_int64), ("coarse_k", C.c_int32), ("precision", C.c_int32),
                ("scene", C.POINTER(ip_scene)), ("batch_budget", C.c_uint64),
                ("mem_bytes", C.c_uint64), ("flags", C.c_uint32)]


class ip_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("d", C.c_int32), ("stats", ip_stats),
                ("n_cells", C.c_int64), ("n_free", C.c_int64), ("digest", C.c_uint64 * 2),
                ("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double),
                ("free_pts", _dp), ("cells", C.c_void_p), ("error", C.c_char * 160),
                ("admitted_bytes", C.c_uint64), ("n_probe_edges", C.c_int64), ("t_admit", C.c_double)]


IP_KEEP_CELLS = 1


class ip_batch_summary(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_free", C.c_int64), ("batches", C.c_int64),
                ("digest", C.c_uint64 * 2), ("stats", ip_stats)]


# int fn(void *user, int64_t batch, const double *free_pts, int64_t n_free, int64_t n_cells)
ip_batch_fn = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int64, _dp, C.c_int64, C.c_int64)


def IP_REFINE(n: int) -> int:
    """ip_trace flag: n (0..15) iterations of the iterative intersection."""
    return (int(n) & 15) << 4

_P = C.POINTER
_sig = {
    "ip_create": (C.c_int, [_P(_vp), C.c_int, _vp]),
    "ip_destroy": (None, [_vp]),
    "ip_last_error": (C.c_char_p, [_vp]),
    "ip_problem_create": (C.c_int, [_vp, _P(ip_fparams), _P(ip_space), _dp, C.c_int64, C.c_int32,
                                    _P(_vp)]),
    "ip_problem_free": (None, [_vp]),
    "ip_trace": (C.c_int, [_vp, _vp, C.c_uint64, C.c_int32, C.c_uint32, _P(_vp)]),
    "ip_cells_count": (C.c_int64, [_vp]),
    "ip_cells_stats": (C.c_int, [_vp, _P(ip_stats)]),
    "ip_cells_download": (C.c_int, [_vp, _vp, _ip, C.POINTER(C.c_uint32), _dp]),
    "ip_cells_points": (C.c_int, [_vp, _P(_vp), _P(C.c_int64)]),
    "ip_cells_digest": (C.c_int, [_vp, _vp, C.POINTER(C.c_uint64)]),
    "ip_cells_gather": (C.c_int, [_vp, _vp, C.POINTER(C.c_int64), C.c_int64, _ip, C.POINTER(C.c_uint32), _dp,
                                  C.POINTER(C.c_uint8)]),
    "ip_cells_free": (None, [_vp]),
    "ip_check": (C.c_int, [_vp, _P(ip_scene), _vp, C.c_int64, C.c_int64, _vp]),
    "ip_check_cells": (C.c_int, [_vp, _vp, _P(ip_scene), _P(C.c_int64)]),
    "ip_cells_download_check": (C.c_int, [_vp, _vp, C.POINTER(C.c_uint8), _dp]),
    "ip_trace_check_batches": (C.c_int, [_vp, _vp, C.c_uint64, C.c_int32, C.c_uint32, _P(ip_scene), ip_batch_fn,
                                         _vp, _P(ip_batch_summary)]),
    "ip_cells_download_free": (C.c_int, [_vp, _vp, _vp]),
    "ip_feval": (C.c_int, [_vp, _vp, _vp, C.c_int64, C.c_int32, _vp, _vp]),
    "ip_feval_noalloc": (C.c_int, [_vp, _vp, _vp, C.c_int64, C.c_int32, _vp, _vp]),
    "ip_region_eval": (C.c_int, [_vp, _vp, _vp, C.c_int64, _vp, _vp, _vp, _P(C.c_int32)]),
    "ip_cells_key_layout": (C.c_int, [_vp, _P(C.c_int32), _P(C.c_int32)]),
    "ip_seed_search": (C.c_int, [_vp, _vp, _vp, C.c_int64, C.c_int32, _vp, _vp]),
    "ip_problem_set_seeds": (C.c_int, [_vp, _vp, _dp, C.c_int64]),
    "ip_server_create": (C.c_int, [_P(_vp), C.c_int, C.c_uint64, C.c_int32]),
    "ip_server_submit": (C.c_int, [_vp, _P(ip_request), _P(C.c_uint64)]),
    "ip_server_poll": (C.c_int, [_vp, C.c_uint64, _P(_P(ip_result))]),
    "ip_server_wait": (C.c_int, [_vp, C.c_uint64, _P(_P(ip_result))]),
    "ip_result_free": (None, [_P(ip_result)]),
    "ip_server_destroy": (None, [_vp]),
    "ip_server_clock": (C.c_double, [_vp]),
}
for _name, (_res, _args) in _sig.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_sig)


class IPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ip error {code}: {msg}")
        self.code = code


def _chk(ctx, rc):
    if rc != IP_OK:
        msg = _lib.ip_last_error(ctx).decode() if ctx else ""
        raise IPError(rc, msg)


def _d(keep, a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    keep.append(a)
    return a.ctypes.data_as(_dp)


def _i(keep, a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    keep.append(a)
    return a.ctypes.data_as(_ip)


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


# --------------------------------------------------------------------------
# Same-name wrappers
# --------------------------------------------------------------------------
def ip_create(device: int = 0, stream=None):
    h = _vp()
    _chk(None, _lib.ip_create(C.byref(h), device, _stream_handle(stream)))
    return h


def ip_destroy(ctx):
    _lib.ip_destroy(ctx)


def ip_last_error(ctx) -> str:
    return _lib.ip_last_error(ctx).decode()


def ip_problem_create(ctx, f, lat, dom, seeds, coarse_k=1):
    """f: inputs.Manifold, lat: inputs.Lattice, dom: inputs.Domain."""
    keep = []
    fp = ip_fparams(f.d, f.p, f.S, f.gamma, f.coef0, f.bias, _d(keep, f.sv), _d(keep, f.alpha), _kernel_code(f))
    sp = ip_space(f.d, _d(keep, lat.M), _d(keep, lat.Minv), _d(keep, lat.o), _d(keep, dom.lo),
                  _d(keep, dom.hi))
    seeds = np.ascontiguousarray(seeds, dtype=np.float64)
    h = _vp()
    _chk(ctx, _lib.ip_problem_create(ctx, C.byref(fp), C.byref(sp), seeds.ctypes.data_as(_dp),
                                     seeds.shape[0], coarse_k, C.byref(h)))
    return h


def ip_problem_free(p):
    _lib.ip_problem_free(p)


def ip_trace(ctx, prob, budget=0, precision=IP_FP64, flags=0):
    h = _vp()
    _chk(ctx, _lib.ip_trace(ctx, prob, budget, precision, flags, C.byref(h)))
    return h


def ip_cells_count(cells) -> int:
    return int(_lib.ip_cells_count(cells))


def ip_cells_stats(cells) -> dict:
    st = ip_stats()
    _chk(None, _lib.ip_cells_stats(cells, C.byref(st)))
    return st.as_dict()


def ip_cells_download(ctx, cells, d, points=True):
    """(v (n, d) int32, mask (n,) uint32, points (n, d) or None)."""
    n = ip_cells_count(cells)
    v = np.empty((n, d), np.int32)
    m = np.empty(n, np.uint32)
    p = np.empty((n, d), np.float64) if points else None
    _chk(ctx, _lib.ip_cells_download(ctx, cells, v.ctypes.data_as(_ip),
                                     m.ctypes.data_as(C.POINTER(C.c_uint32)),
                                     p.ctypes.data_as(_dp) if points else None))
    return v, m, p


def ip_cells_digest(ctx, cells):
    out = (C.c_uint64 * 2)()
    _chk(ctx, _lib.ip_cells_digest(ctx, cells, out))
    return int(out[0]), int(out[1])


def ip_cells_gather(ctx, cells, d, idx, verdict=False):
    """Rows idx of the cells: (v (n, d) int32, mask (n,), points (n, d),
    verdicts (n,) uint8 or None)."""
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    n = len(idx)
    v = np.zeros((n, d), np.int32)
    m = np.zeros(n, np.uint32)
    p = np.zeros((n, d), np.float64)
    vv = np.zeros(n, np.uint8) if verdict else None
    _chk(ctx, _lib.ip_cells_gather(ctx, cells, idx.ctypes.data_as(C.POINTER(C.c_int64)), n, v.ctypes.data_as(_ip),
                                   m.ctypes.data_as(C.POINTER(C.c_uint32)), p.ctypes.data_as(_dp),
                                   vv.ctypes.data_as(C.POINTER(C.c_uint8)) if verdict else None))
    return v, m, p, vv


def ip_cells_points(cells):
    ptr = _vp()
    ld = C.c_int64()
    _chk(None, _lib.ip_cells_points(cells, C.byref(ptr), C.byref(ld)))
    return ptr.value, ld.value


def ip_cells_free(cells):
    _lib.ip_cells_free(cells)


def _scene_struct(sc, keep):
    n = int(sc.joint_T.shape[0])
    return ip_scene(n, _d(keep, sc.joint_T), _i(keep, sc.joint_axis),
                    len(sc.lsph_r), _i(keep, sc.lsph_link), _d(keep, sc.lsph_c), _d(keep, sc.lsph_r),
                    len(sc.lcap_r), _i(keep, sc.lcap_link), _d(keep, sc.lcap_p0),
                    _d(keep, sc.lcap_p1), _d(keep, sc.lcap_r),
                    len(sc.osph_r), _d(keep, sc.osph_c), _d(keep, sc.osph_r),
                    len(sc.obox_l), _d(keep, sc.obox_T), _d(keep, sc.obox_l),
                    len(sc.ocyl_rh), _d(keep, sc.ocyl_T), _d(keep, sc.ocyl_rh))


def ip_check(ctx, scene, q_dev_ptr: int, n: int, ld: int, verdict_dev_ptr: int):
    keep = []
    s = _scene_struct(scene, keep)
    _chk(ctx, _lib.ip_check(ctx, C.byref(s), q_dev_ptr, n, ld, verdict_dev_ptr))


def ip_check_cells(ctx, cells, scene) -> int:
    keep = []
    s = _scene_struct(scene, keep)
    nf = C.c_int64()
    _chk(ctx, _lib.ip_check_cells(ctx, cells, C.byref(s), C.byref(nf)))
    return nf.value


def ip_cells_download_check(ctx, cells, d, n_free):
    n = ip_cells_count(cells)
    ver = np.zeros(n, np.uint8)
    fp = np.zeros((n_free, d), np.float64)
    _chk(ctx, _lib.ip_cells_download_check(ctx, cells, ver.ctypes.data_as(C.POINTER(C.c_uint8)),
                                           fp.ctypes.data_as(_dp)))
    return ver, fp


def ip_cells_download_free(ctx, cells, host_ptr: int):
    """Free points as d host columns of n_free doubles at host_ptr."""
    _chk(ctx, _lib.ip_cells_download_free(ctx, cells, host_ptr))


def ip_feval(ctx, prob, v_dev_ptr: int, n: int, precision, f_dev_ptr: int, bound_dev_ptr: int = 0):
    _chk(ctx, _lib.ip_feval(ctx, prob, v_dev_ptr, n, precision, f_dev_ptr, bound_dev_ptr or None))


def ip_region_eval(ctx, prob, simplex_dev_ptr: int, n: int, y_dev_ptr: int = 0, f_dev_ptr: int = 0,
                   bound_dev_ptr: int = 0) -> int:
    """Returns NP, the template points per coarse simplex."""
    np_out = C.c_int32()
    _chk(ctx, _lib.ip_region_eval(ctx, prob, simplex_dev_ptr or None, n, y_dev_ptr or None, f_dev_ptr or None,
                                  bound_dev_ptr or None, C.byref(np_out)))
    return np_out.value


def ip_seed_search(ctx, prob, q0_dev_ptr: int, n: int, iters: int, q_dev_ptr: int, f_dev_ptr: int):
    _chk(ctx, _lib.ip_seed_search(ctx, prob, q0_dev_ptr, n, iters, q_dev_ptr, f_dev_ptr))


def ip_problem_set_seeds(ctx, prob, seeds):
    seeds = np.ascontiguousarray(seeds, dtype=np.float64)
    _chk(ctx, _lib.ip_problem_set_seeds(ctx, prob, seeds.ctypes.data_as(_dp), seeds.shape[0]))


def ip_cells_key_layout(cells, d):
    bits = C.c_int32()
    vmin = np.zeros(8, np.int32)
    _chk(None, _lib.ip_cells_key_layout(cells, C.byref(bits), vmin.ctypes.data_as(_ip)))
    return bits.value, vmin[:d].copy()


IP_NOALLOC_MAX_VERTICES = 1048576


def ip_feval_noalloc(ctx, prob, v_dev_ptr: int, n: int, precision, f_dev_ptr: int, bound_dev_ptr: int = 0):
    _chk(ctx, _lib.ip_feval_noalloc(ctx, prob, v_dev_ptr, n, precision, f_dev_ptr, bound_dev_ptr or None))


# --------------------------------------------------------------------------
# Small conveniences over the same calls (still marshalling only)
# --------------------------------------------------------------------------
class Context:
    def __init__(self, device=0, stream=None):
        self.h = ip_create(device, stream)

    def close(self):
        if self.h:
            ip_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def ip_trace_check_batches(ctx, prob, scene, d, budget=0, precision=IP_FP64, flags=0, on_batch=None,
                           collect=False):
    """Per-batch trace + check with the C_free points handed to the host
    batch by batch.  on_batch(batch, free_pts (n_free x d, a view valid only
    during the call), n_cells) may return True to stop (IPError
    IP_ECANCELED).  Returns (summary dict, list of per-batch copies of the
    free points if collect else None)."""
    keep = []
    s = _scene_struct(scene, keep)
    got = [] if collect else None
    err = []

    def cb(_user, batch, pts, n_free, n_cells):
        try:
            view = (np.ctypeslib.as_array(pts, shape=(n_free * d,)).reshape(n_free, d) if n_free > 0
                    else np.zeros((0, d)))
            if got is not None:
                got.append(view.copy())
            if on_batch is not None and on_batch(batch, view, n_cells):
                return 1
            return 0
        except Exception as e:  # an exception stops the trace and is re-raised
            err.append(e)
            return 1

    fn = ip_batch_fn(cb)
    out = ip_batch_summary()
    rc = _lib.ip_trace_check_batches(ctx, prob, budget, precision, flags, C.byref(s), fn, None, C.byref(out))
    if err:
        raise err[0]
    _chk(ctx, rc)
    summ = {"n_cells": out.n_cells, "n_free": out.n_free, "batches": out.batches,
            "digest": (out.digest[0], out.digest[1]), "stats": out.stats.as_dict()}
    return summ, got


class Problem:
    def __init__(self, ctx: Context, wl, coarse_k=None):
        self.ctx = ctx
        self.d = wl.f.d
        self.h = ip_problem_create(ctx.h, wl.f, wl.lat, wl.dom, wl.seeds,
                                   wl.k if coarse_k is None else coarse_k)

    def trace_check_batches(self, scene, budget=0, precision=IP_FP64, flags=0, on_batch=None, collect=False):
        return ip_trace_check_batches(self.ctx.h, self.h, scene, self.d, budget, precision, flags, on_batch,
                                      collect)

    def close(self):
        if self.h:
            ip_problem_free(self.h)
            self.h = None


class Cells:
    def __init__(self, ctx: Context, prob: Problem, budget=0, precision=IP_FP64, flags=0):
        self.ctx = ctx
        self.d = prob.d
        self.h = ip_trace(ctx.h, prob.h, budget, precision, flags)
        self.n_free = None

    @property
    def n(self):
        return ip_cells_count(self.h)

    def stats(self):
        return ip_cells_stats(self.h)

    def download(self, points=True):
        return ip_cells_download(self.ctx.h, self.h, self.d, points)

    def check(self, scene):
        self.n_free = ip_check_cells(self.ctx.h, self.h, scene)
        return self.n_free

    def digest(self):
        return ip_cells_digest(self.ctx.h, self.h)

    def key_layout(self):
        return ip_cells_key_layout(self.h, self.d)

    def gather(self, idx, verdict=False):
        return ip_cells_gather(self.ctx.h, self.h, self.d, idx, verdict)

    def download_check(self):
        return ip_cells_download_check(self.ctx.h, self.h, self.d, self.n_free)

    def close(self):
        if self.h:
            ip_cells_free(self.h)
            self.h = None


# --------------------------------------------------------------------------
# Serving loop
# --------------------------------------------------------------------------
def ip_server_create(device=0, pool_bytes=0, max_slots=4):
    h = _vp()
    _chk(None, _lib.ip_server_create(C.byref(h), device, pool_bytes, max_slots))
    return h


def ip_server_submit(server, wl, precision=IP_FP64, scene=None, budget=0, mem_bytes=0, flags=0,
                     coarse_k=None):
    """Queue workload wl (inputs.Workload); returns the request id."""
    keep = []
    f = wl.f
    fp = ip_fparams(f.d, f.p, f.S, f.gamma, f.coef0, f.bias, _d(keep, f.sv), _d(keep, f.alpha), _kernel_code(f))
    sp = ip_space(f.d, _d(keep, wl.lat.M), _d(keep, wl.lat.Minv), _d(keep, wl.lat.o),
                  _d(keep, wl.dom.lo), _d(keep, wl.dom.hi))
    seeds = np.ascontiguousarray(wl.seeds, dtype=np.float64)
    sc = C.pointer(_scene_struct(scene, keep)) if scene is not None else None
    req = ip_request(C.pointer(fp), C.pointer(sp), seeds.ctypes.data_as(_dp), seeds.shape[0],
                     wl.k if coarse_k is None else coarse_k, precision, sc, budget, mem_bytes, flags)
    rid = C.c_uint64()
    _chk(None, _lib.ip_server_submit(server, C.byref(req), C.byref(rid)))
    return rid.value


def _take_result(rp):
    r = rp.contents
    out = {"status": r.status, "d": r.d, "stats": r.stats.as_dict(), "n_cells": r.n_cells,
           "n_free": r.n_free, "digest": (r.digest[0], r.digest[1]), "t_submit": r.t_submit,
           "t_start": r.t_start, "t_done": r.t_done, "error": r.error.decode(errors="replace"),
           "admitted_bytes": r.admitted_bytes, "n_probe_edges": r.n_probe_edges, "t_admit": r.t_admit}
    if r.free_pts and r.n_free > 0:
        out["free_pts"] = np.ctypeslib.as_array(r.free_pts, shape=(r.n_free * r.d,)).reshape(
            r.n_free, r.d).copy()
    if r.cells:
        out["cells"] = ip_cells_download(None, _vp(r.cells), r.d)
    _lib.ip_result_free(rp)
    return out


def ip_server_poll(server, rid):
    rp = _P(ip_result)()
    rc = _lib.ip_server_poll(server, rid, C.byref(rp))
    if rc == IP_EAGAIN:
        return None
    _chk(None, rc)
    return _take_result(rp)


def ip_server_wait(server, rid):
    rp = _P(ip_result)()
    _chk(None, _lib.ip_server_wait(server, rid, C.byref(rp)))
    return _take_result(rp)


def ip_server_destroy(server):
    _lib.ip_server_destroy(server)


def ip_server_clock(server) -> float:
    return _lib.ip_server_clock(server)
