"""Python access to the reference (oracle) implementation in oracle.c.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg load this module; the product library never does.

build() compiles oracle.c with gcc (-O2 -ffp-contract=off).  All arrays are
numpy float64 / int32 in C order.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "oracle.c")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_up = C.POINTER(C.c_uint32)


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-ffp-contract=off", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _F(C.Structure):
    _fields_ = [("d", C.c_int32), ("p", C.c_int32), ("S", C.c_int64),
                ("gamma", C.c_double), ("coef0", C.c_double), ("bias", C.c_double),
                ("sv", _dp), ("alpha", _dp), ("kernel", C.c_int32)]


class _Space(C.Structure):
    _fields_ = [("d", C.c_int32), ("M", _dp), ("Minv", _dp), ("o", _dp),
                ("lo", _dp), ("hi", _dp)]


class _Edges(C.Structure):
    _fields_ = [("n", C.c_int64), ("d", C.c_int32), ("v", _ip), ("mask", _up)]


class _Scene(C.Structure):
    _fields_ = [("n_joints", C.c_int32), ("joint_T", _dp), ("joint_axis", _ip),
                ("n_lsph", C.c_int32), ("lsph_link", _ip), ("lsph_c", _dp), ("lsph_r", _dp),
                ("n_lcap", C.c_int32), ("lcap_link", _ip), ("lcap_p0", _dp), ("lcap_p1", _dp),
                ("lcap_r", _dp),
                ("n_osph", C.c_int32), ("osph_c", _dp), ("osph_r", _dp),
                ("n_obox", C.c_int32), ("obox_T", _dp), ("obox_l", _dp),
                ("n_ocyl", C.c_int32), ("ocyl_T", _dp), ("ocyl_rh", _dp)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = C.CDLL(LIB)
        L.orc_exp.restype = C.c_double
        L.orc_exp.argtypes = [C.c_double]
        L.orc_f.restype = C.c_double
        L.orc_f.argtypes = [C.POINTER(_F), _dp]
        L.orc_f_batch.argtypes = [C.POINTER(_F), C.POINTER(_Space), C.c_int64, _ip, _dp]
        L.orc_f_grad.restype = C.c_double
        L.orc_f_grad.argtypes = [C.POINTER(_F), _dp, _dp]
        L.orc_seed_search.argtypes = [C.POINTER(_F), C.POINTER(_Space), C.c_int64, _dp, C.c_int32, _dp, _dp]
        L.orc_coords.argtypes = [C.POINTER(_Space), _ip, _dp]
        L.orc_locate.argtypes = [C.POINTER(_Space), C.c_int32, _dp, _ip, _ip]
        L.orc_cofaces2.restype = C.c_int64
        L.orc_cofaces2.argtypes = [C.c_int32, _ip, C.c_uint32, _ip]
        L.orc_ncofaces.restype = C.c_int64
        L.orc_ncofaces.argtypes = [C.c_int32, _ip, C.c_uint32, _ip]
        L.orc_canonical.restype = C.c_int32
        L.orc_canonical.argtypes = [C.c_int32, _ip, C.c_int32, _up, _ip, _up]
        for name in ("orc_trace_direct",):
            getattr(L, name).argtypes = [C.POINTER(_F), C.POINTER(_Space), C.c_int32, _dp,
                                         C.c_int64, C.POINTER(_Edges)]
        L.orc_trace_batch.argtypes = [C.POINTER(_F), C.POINTER(_Space), C.c_int32, _dp,
                                      C.c_int64, C.POINTER(_Edges), C.POINTER(C.c_int64)]
        L.orc_batch_sigma.argtypes = [C.POINTER(_F), C.POINTER(_Space), C.c_int32, _dp,
                                      C.c_int64, C.POINTER(C.c_int64), C.POINTER(_ip)]
        L.orc_brute.argtypes = [C.POINTER(_F), C.POINTER(_Space), C.POINTER(_Edges)]
        L.orc_template.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_int64), _ip,
                                   C.POINTER(C.c_int64), _ip, _up]
        L.orc_points.argtypes = [C.POINTER(_F), C.POINTER(_Space), C.c_int64, _ip, _up, _dp, _dp]
        L.orc_points_refined.argtypes = [C.POINTER(_F), C.POINTER(_Space), C.c_int64, _ip, _up, C.c_int32,
                                         _dp]
        L.orc_sincos.argtypes = [C.c_double, _dp, _dp]
        L.orc_sphere_sphere.argtypes = [_dp, C.c_double, _dp, C.c_double]
        L.orc_capsule_sphere.argtypes = [_dp, _dp, C.c_double, _dp, C.c_double]
        L.orc_sphere_box.argtypes = [_dp, C.c_double, _dp, _dp]
        L.orc_sphere_cylinder.argtypes = [_dp, C.c_double, _dp, C.c_double, C.c_double]
        L.orc_fk.argtypes = [C.POINTER(_Scene), _dp, _dp]
        L.orc_check.argtypes = [C.POINTER(_Scene), C.c_int64, _dp, C.POINTER(C.c_uint8)]
        L.orc_free.argtypes = [C.c_void_p]
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_ip)


class _Ctx:
    """Keeps numpy buffers alive while ctypes structs point into them."""

    def __init__(self, f=None, lat=None, dom=None):
        self.keep = []
        if f is not None:
            sv, psv = _d(f.sv)
            al, pal = _d(f.alpha)
            self.keep += [sv, al]
            self.f = _F(f.d, f.p, f.S, f.gamma, f.coef0, f.bias, psv, pal,
                        1 if getattr(f, "kernel", "poly") == "rbf" else 0)
        if lat is not None:
            M, pM = _d(lat.M)
            Mi, pMi = _d(lat.Minv)
            o, po = _d(lat.o)
            d = M.shape[0]
            if dom is None:
                lo, plo = _d(np.full(d, -np.inf))
                hi, phi = _d(np.full(d, np.inf))
            else:
                lo, plo = _d(dom.lo)
                hi, phi = _d(dom.hi)
            self.keep += [M, Mi, o, lo, hi]
            self.sp = _Space(d, pM, pMi, po, plo, phi)


def _take_edges(e: _Edges):
    n, d = e.n, e.d
    v = np.ctypeslib.as_array(e.v, shape=(max(n, 1) * d,))[: n * d].reshape(n, d).copy()
    m = np.ctypeslib.as_array(e.mask, shape=(max(n, 1),))[:n].copy()
    lib().orc_free(C.cast(e.v, C.c_void_p))
    lib().orc_free(C.cast(e.mask, C.c_void_p))
    return v, m


def coords(lat, v):
    c = _Ctx(lat=lat)
    v, pv = _i(np.atleast_2d(v))
    out = np.empty(v.shape, np.float64)
    for i in range(v.shape[0]):
        lib().orc_coords(C.byref(c.sp), v[i].ctypes.data_as(_ip), out[i].ctypes.data_as(_dp))
    return out


def feval(wl_f, lat, v):
    """Canonical FP64 f at lattice vertices v (n, d)."""
    c = _Ctx(wl_f, lat)
    v, pv = _i(np.atleast_2d(v))
    out = np.empty(v.shape[0], np.float64)
    lib().orc_f_batch(C.byref(c.f), C.byref(c.sp), v.shape[0], pv, out.ctypes.data_as(_dp))
    return out


def exp(t):
    return lib().orc_exp(float(t))


def f_at(wl_f, x):
    c = _Ctx(wl_f)
    x, px = _d(x)
    return lib().orc_f(C.byref(c.f), px)


def f_grad(wl_f, x):
    c = _Ctx(wl_f)
    x, px = _d(x)
    g = np.zeros(wl_f.d)
    v = lib().orc_f_grad(C.byref(c.f), px, g.ctypes.data_as(_dp))
    return v, g


def seed_search(wl, q0, iters):
    """Minimum-norm Newton steps towards f = 0 from the rows of q0."""
    c = _Ctx(wl.f, wl.lat, wl.dom)
    q0, pq0 = _d(np.atleast_2d(q0))
    q = np.zeros_like(q0)
    fq = np.zeros(q0.shape[0])
    _check(lib().orc_seed_search(C.byref(c.f), C.byref(c.sp), q0.shape[0], pq0, iters,
                                 q.ctypes.data_as(_dp), fq.ctypes.data_as(_dp)), "seed_search")
    return q, fq


def locate(lat, y, coarse_k=1):
    c = _Ctx(lat=lat)
    y, py = _d(y)
    d = y.shape[0]
    v = np.zeros(d, np.int32)
    w = np.zeros(d, np.int32)
    lib().orc_locate(C.byref(c.sp), coarse_k, py, v.ctypes.data_as(_ip), w.ctypes.data_as(_ip))
    return v, w


def cofaces2(d, v, mask):
    v, pv = _i(v)
    buf = np.zeros(3 * d * (2 << d), np.int32)
    n = lib().orc_cofaces2(d, pv, mask, buf.ctypes.data_as(_ip))
    return buf[: n * 3 * d].reshape(n, 3, d)


def ncofaces(d, v, mask):
    import math
    v, pv = _i(v)
    buf = np.zeros(2 * d * math.factorial(d + 1), np.int32)
    n = lib().orc_ncofaces(d, pv, mask, buf.ctypes.data_as(_ip))
    return buf[: n * 2 * d].reshape(n, 2 * d)


def canonical(d, v, parts):
    v, pv = _i(v)
    parts = np.ascontiguousarray(parts, np.uint32)
    vc = np.zeros(d, np.int32)
    pc = np.zeros(len(parts), np.uint32)
    lib().orc_canonical(d, pv, len(parts), parts.ctypes.data_as(_up),
                        vc.ctypes.data_as(_ip), pc.ctypes.data_as(_up))
    return vc, pc


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed: {rc}")


def trace_direct(wl, coarse_k=1):
    """Direct trace; returns (v (n,d) int32, mask (n,) uint32) sorted."""
    c = _Ctx(wl.f, wl.lat, wl.dom)
    s, ps = _d(wl.seeds)
    e = _Edges()
    _check(lib().orc_trace_direct(C.byref(c.f), C.byref(c.sp), coarse_k, ps,
                                  s.shape[0], C.byref(e)), "trace_direct")
    return _take_edges(e)


def trace_batch(wl, k=None):
    c = _Ctx(wl.f, wl.lat, wl.dom)
    s, ps = _d(wl.seeds)
    e = _Edges()
    ns = C.c_int64(0)
    _check(lib().orc_trace_batch(C.byref(c.f), C.byref(c.sp), wl.k if k is None else k,
                                 ps, s.shape[0], C.byref(e), C.byref(ns)), "trace_batch")
    v, m = _take_edges(e)
    return v, m, ns.value


def batch_sigma(wl, k=None):
    c = _Ctx(wl.f, wl.lat, wl.dom)
    s, ps = _d(wl.seeds)
    n = C.c_int64(0)
    out = _ip()
    _check(lib().orc_batch_sigma(C.byref(c.f), C.byref(c.sp), wl.k if k is None else k,
                                 ps, s.shape[0], C.byref(n), C.byref(out)), "batch_sigma")
    d = wl.f.d
    arr = np.ctypeslib.as_array(out, shape=(max(n.value, 1) * 2 * d,))[: n.value * 2 * d]
    arr = arr.reshape(n.value, 2 * d).copy()
    lib().orc_free(C.cast(out, C.c_void_p))
    return arr


def brute(wl):
    c = _Ctx(wl.f, wl.lat, wl.dom)
    e = _Edges()
    _check(lib().orc_brute(C.byref(c.f), C.byref(c.sp), C.byref(e)), "brute")
    return _take_edges(e)


def template(d, k):
    n_p = C.c_int64(0)
    n_e = C.c_int64(0)
    lib().orc_template(d, k, C.byref(n_p), None, C.byref(n_e), None, None)
    pts = np.zeros((n_p.value, d), np.int32)
    eu = np.zeros((n_e.value, d), np.int32)
    er = np.zeros(n_e.value, np.uint32)
    lib().orc_template(d, k, C.byref(n_p), pts.ctypes.data_as(_ip), C.byref(n_e),
                       eu.ctypes.data_as(_ip), er.ctypes.data_as(_up))
    return pts, eu, er


def points(wl, v, mask):
    c = _Ctx(wl.f, wl.lat, wl.dom)
    v, pv = _i(v)
    mask = np.ascontiguousarray(mask, np.uint32)
    n = v.shape[0]
    pts = np.zeros((n, wl.f.d), np.float64)
    t = np.zeros(n, np.float64)
    lib().orc_points(C.byref(c.f), C.byref(c.sp), n, pv, mask.ctypes.data_as(_up),
                     pts.ctypes.data_as(_dp), t.ctypes.data_as(_dp))
    return pts, t


def points_refined(wl, v, mask, iters):
    """Intersection points after `iters` false-position (Illinois) steps."""
    c = _Ctx(wl.f, wl.lat, wl.dom)
    v, pv = _i(v)
    mask = np.ascontiguousarray(mask, np.uint32)
    n = v.shape[0]
    pts = np.zeros((n, wl.f.d), np.float64)
    _check(lib().orc_points_refined(C.byref(c.f), C.byref(c.sp), n, pv, mask.ctypes.data_as(_up), iters,
                                    pts.ctypes.data_as(_dp)), "points_refined")
    return pts


def sincos(q):
    s = C.c_double()
    c = C.c_double()
    lib().orc_sincos(float(q), C.byref(s), C.byref(c))
    return s.value, c.value


def sphere_sphere(a, ra, b, rb):
    a, pa = _d(a)
    b, pb = _d(b)
    return lib().orc_sphere_sphere(pa, ra, pb, rb)


def capsule_sphere(p0, p1, rc, c, rs):
    p0, a = _d(p0)
    p1, b = _d(p1)
    c, pc = _d(c)
    return lib().orc_capsule_sphere(a, b, rc, pc, rs)


def sphere_box(c, r, T, l):
    c, pc = _d(c)
    T, pT = _d(T)
    l, pl = _d(l)
    return lib().orc_sphere_box(pc, r, pT, pl)


def sphere_cylinder(c, r, T, rc, h):
    c, pc = _d(c)
    T, pT = _d(T)
    return lib().orc_sphere_cylinder(pc, r, pT, rc, h)


class _SceneCtx:
    def __init__(self, sc):
        self.keep = []

        def D(a):
            a, p = _d(a)
            self.keep.append(a)
            return p

        def I(a):
            a, p = _i(a)
            self.keep.append(a)
            return p

        n = int(sc.joint_T.shape[0])
        self.s = _Scene(n, D(sc.joint_T), I(sc.joint_axis),
                        len(sc.lsph_r), I(sc.lsph_link), D(sc.lsph_c), D(sc.lsph_r),
                        len(sc.lcap_r), I(sc.lcap_link), D(sc.lcap_p0), D(sc.lcap_p1),
                        D(sc.lcap_r),
                        len(sc.osph_r), D(sc.osph_c), D(sc.osph_r),
                        len(sc.obox_l), D(sc.obox_T), D(sc.obox_l),
                        len(sc.ocyl_rh), D(sc.ocyl_T), D(sc.ocyl_rh))


def fk(sc, q):
    c = _SceneCtx(sc)
    q, pq = _d(q)
    n = sc.joint_T.shape[0]
    out = np.zeros((n, 12))
    lib().orc_fk(C.byref(c.s), pq, out.ctypes.data_as(_dp))
    return out


def check(sc, q):
    """Verdicts (uint8, 1 = collision) for configurations q (n, n_joints)."""
    c = _SceneCtx(sc)
    q, pq = _d(np.atleast_2d(q))
    out = np.zeros(q.shape[0], np.uint8)
    _check(lib().orc_check(C.byref(c.s), q.shape[0], pq,
                           out.ctypes.data_as(C.POINTER(C.c_uint8))), "check")
    return out
