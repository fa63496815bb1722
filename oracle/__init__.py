"""FP64 CPU oracle for the local Verlet buffer DEM step (ctypes over liborc.so).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may use it; the product path never does.  It shares no code
with the HIP library.  The C source (orc.c) cites the passages of the paper that
each function follows.
"""
import ctypes
import os

import numpy as np

from .build import LIB, build

SKIN_LOCAL, SKIN_UNIFORM, NO_BUFFER, FIXED_INTERVAL, NAIVE = 0, 1, 2, 3, 4


MAX_PLANES = 4
MAX_CYLINDERS = 2


class Params(ctypes.Structure):
    _fields_ = [
        ("skin_mode", ctypes.c_int32),
        ("cap_mode", ctypes.c_int32),
        ("ring", ctypes.c_int32),
        ("fixed_interval", ctypes.c_int32),
        ("check_superset", ctypes.c_int32),
        ("validity_uses_uncapped_skin", ctypes.c_int32),
        ("v_in_is_half_step", ctypes.c_int32),
        ("state_fp32", ctypes.c_int32),
        ("K", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("cell_size", ctypes.c_double),
        ("skin_uniform", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("kn", ctypes.c_double),
        ("gamma_n", ctypes.c_double),
        ("g", ctypes.c_double * 3),
        ("n_planes", ctypes.c_int32),
        ("pad2_", ctypes.c_int32),
        ("planes", (ctypes.c_double * 5) * MAX_PLANES),
        ("kt", ctypes.c_double),
        ("gamma_t", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("n_cylinders", ctypes.c_int32),
        ("pad3_", ctypes.c_int32),
        ("cylinders", (ctypes.c_double * 4) * MAX_CYLINDERS),
    ]


RECORD_DTYPE = np.dtype([
    ("step", np.int32), ("rebuilt", np.int32), ("list_pairs", np.int64),
    ("contacts", np.int64), ("violators", np.int64), ("missed", np.int64),
    ("max_excess", np.float64), ("kinetic_energy", np.float64),
])

_lib = None


class Springs(ctypes.Structure):
    """orc_springs: the tangential springs of the last step's contacts."""
    _fields_ = [("off", ctypes.c_void_p), ("j", ctypes.c_void_p), ("xi", ctypes.c_void_p),
                ("cap", ctypes.c_int64), ("n", ctypes.c_int64)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(
                os.path.join(os.path.dirname(LIB), "orc.c")):
            build()
        L = ctypes.CDLL(LIB)
        i64, i32, dp, ip = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p
        L.orc_broadphase_brute.restype = i64
        L.orc_broadphase_brute.argtypes = [i64, dp, dp, ctypes.c_double, ip, i64]
        L.orc_broadphase_linked_cell.restype = i64
        L.orc_broadphase_linked_cell.argtypes = [i64, dp, dp, ctypes.c_double, dp, dp,
                                                 ctypes.c_double, i32, ip, i64]
        L.orc_contacts_brute.restype = i64
        L.orc_contacts_brute.argtypes = [i64, dp, dp, ip, i64]
        L.orc_rebuild_radii.restype = ctypes.c_int
        L.orc_rebuild_radii.argtypes = [ctypes.POINTER(Params), i64, dp, dp, dp, dp]
        L.orc_forces.restype = ctypes.c_int
        L.orc_forces.argtypes = [ctypes.POINTER(Params), i64, dp, dp, dp, i64, ip, dp]
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_get_threads.restype = ctypes.c_int
        L.orc_get_threads.argtypes = []
        L.orc_run.restype = ctypes.c_int
        L.orc_run.argtypes = [ctypes.POINTER(Params), i64, dp, dp, dp, dp, i32, dp, dp, dp,
                              ip, i64, ctypes.POINTER(ctypes.c_int64)]
        L.orc_run_springs.restype = ctypes.c_int
        L.orc_run_springs.argtypes = [ctypes.POINTER(Params), i64, dp, dp, dp, dp, i32, dp, dp,
                                      dp, ip, i64, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(Springs)]
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """Threads the oracle's loops over particles use (results do not depend on it)."""
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def _d(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None and a.size else None


def make_params(p: dict) -> Params:
    """Build the oracle's parameter struct from a plain dict of the physical and
    method parameters (the keys are the field names above)."""
    q = Params()
    q.skin_mode = int(p.get("skin_mode", SKIN_LOCAL))
    q.cap_mode = int(p.get("cap_mode", 0))
    q.ring = int(p.get("ring", 0))
    q.fixed_interval = int(p.get("fixed_interval", 1))
    q.check_superset = int(p.get("check_superset", 0))
    q.validity_uses_uncapped_skin = int(p.get("validity_uses_uncapped_skin", 0))
    q.v_in_is_half_step = int(p.get("v_in_is_half_step", 0))
    q.state_fp32 = int(p.get("state_fp32", 0))
    for k in ("K", "dt", "cell_size", "skin_uniform", "eps", "kn", "gamma_n", "kt", "gamma_t", "mu"):
        setattr(q, k, float(p.get(k, 0.0)))
    for k in ("lo", "hi", "g"):
        v = p.get(k, (0.0, 0.0, 0.0))
        getattr(q, k)[:] = [float(t) for t in v]
    planes = p.get("planes", ())
    if len(planes) > MAX_PLANES:
        raise ValueError(f"at most {MAX_PLANES} planar walls")
    q.n_planes = len(planes)
    for w, pl in enumerate(planes):
        q.planes[w][:] = [float(t) for t in pl]
    cylinders = p.get("cylinders", ())
    if len(cylinders) > MAX_CYLINDERS:
        raise ValueError(f"at most {MAX_CYLINDERS} cylindrical walls")
    q.n_cylinders = len(cylinders)
    for w, cy in enumerate(cylinders):
        q.cylinders[w][:] = [float(t) for t in cy]
    return q


def _pairs_call(fn, n, *args, cap=None):
    if cap is None:
        cap = 1 << 16
    while True:
        out = np.empty((max(cap, 1), 2), dtype=np.int32)
        m = fn(n, *args, out.ctypes.data_as(ctypes.c_void_p), cap)
        if m < 0:
            raise MemoryError("oracle out of memory")
        if m <= cap:
            return out[:m].copy()
        cap = int(m)


def broadphase_brute(x, r, eps=0.0):
    x = _d(x, (-1, 3)); r = _d(r)
    return _pairs_call(lib().orc_broadphase_brute, len(r), _ptr(x), _ptr(r), float(eps))


def broadphase_linked_cell(x, r, eps, lo, hi, cell_edge_min, ring=1):
    x = _d(x, (-1, 3)); r = _d(r); lo = _d(lo); hi = _d(hi)
    return _pairs_call(lib().orc_broadphase_linked_cell, len(r), _ptr(x), _ptr(r), float(eps),
                       _ptr(lo), _ptr(hi), float(cell_edge_min), int(ring))


def contacts_brute(x, rc):
    x = _d(x, (-1, 3)); rc = _d(rc)
    return _pairs_call(lib().orc_contacts_brute, len(rc), _ptr(x), _ptr(rc))


def rebuild_radii(params: dict, v, rc):
    v = _d(v, (-1, 3)); rc = _d(rc)
    n = len(rc)
    rnl = np.zeros(n); se = np.zeros(n)
    q = make_params(params)
    rcode = lib().orc_rebuild_radii(ctypes.byref(q), n, _ptr(v), _ptr(rc), _ptr(rnl), _ptr(se))
    if rcode != 0:
        raise ValueError("R_C exceeds the cap")
    return rnl, se


def forces(params: dict, x, v, rc, contacts):
    x = _d(x, (-1, 3)); v = _d(v, (-1, 3)); rc = _d(rc)
    c = np.ascontiguousarray(contacts, dtype=np.int32).reshape(-1, 2)
    F = np.zeros_like(x)
    q = make_params(params)
    rcode = lib().orc_forces(ctypes.byref(q), len(rc), _ptr(x), _ptr(v), _ptr(rc), len(c),
                             _ptr(c), _ptr(F))
    if rcode != 0:
        raise MemoryError("oracle out of memory")
    return F


def run(params: dict, x, v, rc, invm, n_steps, want_list=False):
    """Run the time loop; returns (x^S, v^{S-1/2}, records, final list or None)."""
    x = _d(x, (-1, 3)); v = _d(v, (-1, 3)); rc = _d(rc); invm = _d(invm)
    n = len(rc)
    xo = np.zeros_like(x); vo = np.zeros_like(v)
    hist = np.zeros(max(n_steps, 1), dtype=RECORD_DTYPE)
    q = make_params(params)
    cap = 0
    nl = ctypes.c_int64(0)
    while True:
        lst = np.empty((max(cap, 1), 2), dtype=np.int32) if want_list else None
        rcode = lib().orc_run(ctypes.byref(q), n, _ptr(x), _ptr(v), _ptr(rc), _ptr(invm),
                              int(n_steps), _ptr(xo), _ptr(vo),
                              hist.ctypes.data_as(ctypes.c_void_p),
                              lst.ctypes.data_as(ctypes.c_void_p) if want_list else None,
                              cap, ctypes.byref(nl) if want_list else None)
        if rcode == -3 and want_list:
            cap = int(nl.value)
            continue
        if rcode == -1:
            raise ValueError("oracle: invalid parameters")
        if rcode == -2:
            raise MemoryError("oracle out of memory")
        break
    return xo, vo, hist[:n_steps], (lst[: nl.value].copy() if want_list else None)


def run_springs(params: dict, x, v, rc, invm, n_steps):
    """run() that also returns the springs of the last step's contacts:
    (x^S, v^{S-1/2}, records, (off, partner, spring)), where particle i's
    contacts are entries off[i] .. off[i+1]-1, partners ascending, and spring
    holds the pair's elongation as seen from i."""
    x = _d(x, (-1, 3)); v = _d(v, (-1, 3)); rc = _d(rc); invm = _d(invm)
    n = len(rc)
    xo = np.zeros_like(x); vo = np.zeros_like(v)
    hist = np.zeros(max(n_steps, 1), dtype=RECORD_DTYPE)
    q = make_params(params)
    off = np.zeros(n + 1, dtype=np.int64)
    cap = 0
    while True:
        j = np.zeros(max(cap, 1), dtype=np.int32)
        xi = np.zeros((max(cap, 1), 3))
        spr = Springs(off.ctypes.data, j.ctypes.data, xi.ctypes.data, cap, 0)
        rcode = lib().orc_run_springs(ctypes.byref(q), n, _ptr(x), _ptr(v), _ptr(rc), _ptr(invm),
                                      int(n_steps), _ptr(xo), _ptr(vo),
                                      hist.ctypes.data_as(ctypes.c_void_p), None, 0, None,
                                      ctypes.byref(spr))
        if rcode == -3:
            cap = int(spr.n)
            continue
        if rcode == -1:
            raise ValueError("oracle: invalid parameters")
        if rcode == -2:
            raise MemoryError("oracle out of memory")
        break
    return xo, vo, hist[:n_steps], (off.copy(), j[: spr.n].copy(), xi[: spr.n].copy())
