"""Local Verlet buffer DEM step on AMD Instinct MI355X: Python binding of libvbuf.so.

The functions below carry the names of the C ABI in include/vbuf.h and only
marshal arguments: every step of the method runs in the library's HIP kernels.
Device buffers are PyTorch tensors (their data_ptr()), the stream is PyTorch's
current stream.  A missing library is an error, never a fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvbuf.so")

VB_OK, VB_EINVAL, VB_ENOMEM, VB_EDEVICE, VB_ECAPACITY, VB_ENONFINITE = 0, -1, -2, -3, -4, -5
VB_SKIN_LOCAL, VB_SKIN_UNIFORM, VB_NO_BUFFER, VB_FIXED_INTERVAL = 0, 1, 2, 3


VB_MAX_PLANES = 4
VB_MAX_CYLINDERS = 2


class vb_params(ctypes.Structure):
    _fields_ = [
        ("skin_mode", ctypes.c_int32),
        ("cap_mode", ctypes.c_int32),
        ("K", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("cell_size", ctypes.c_double),
        ("skin_uniform", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("kn", ctypes.c_double),
        ("gamma_n", ctypes.c_double),
        ("gravity", ctypes.c_double * 3),
        ("max_neighbors", ctypes.c_int32),
        ("fixed_interval", ctypes.c_int32),
        ("reorder_interval", ctypes.c_int32),
        ("bin_capacity", ctypes.c_int32),
        ("n_planes", ctypes.c_int32),
        ("reserved_", ctypes.c_int32),
        ("planes", (ctypes.c_double * 5) * VB_MAX_PLANES),
        ("kt", ctypes.c_double),
        ("gamma_t", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("contact_capacity", ctypes.c_int32),
        ("reserved2_", ctypes.c_int32),
        ("n_cylinders", ctypes.c_int32),
        ("reserved3_", ctypes.c_int32),
        ("cylinders", (ctypes.c_double * 4) * VB_MAX_CYLINDERS),
    ]


STEP_RECORD_DTYPE = np.dtype([
    ("step", np.int32), ("rebuilt", np.int32), ("list_pairs", np.int64),
    ("contacts", np.int64), ("violators", np.int64), ("max_excess", np.float32),
    ("reserved", np.int32), ("kinetic_energy", np.float64),
])
assert STEP_RECORD_DTYPE.itemsize == 48

# name -> (restype, argtypes), in the order of include/vbuf.h
_P = ctypes.c_void_p
_SIGNATURES = {
    "vb_create": (ctypes.c_int32, [ctypes.POINTER(vb_params), ctypes.c_int64, _P,
                                   ctypes.POINTER(_P)]),
    "vb_batch_create": (ctypes.c_int32, [ctypes.POINTER(vb_params), ctypes.POINTER(ctypes.c_int64),
                                         ctypes.c_int32, _P, ctypes.POINTER(_P)]),
    "vb_set_state": (ctypes.c_int32, [_P, _P, _P, _P, _P, ctypes.c_int32]),
    "vb_run": (ctypes.c_int32, [_P, ctypes.c_int32, _P]),
    "vb_get_state": (ctypes.c_int32, [_P, _P, _P, ctypes.POINTER(ctypes.c_int32)]),
    "vb_get_pairs": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, _P, _P, ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_int64)]),
    "vb_get_verlet_state": (ctypes.c_int32, [_P, _P, ctypes.POINTER(ctypes.c_int32),
                                             ctypes.POINTER(ctypes.c_int64)]),
    "vb_set_verlet_state": (ctypes.c_int32, [_P, _P, ctypes.POINTER(ctypes.c_int32), ctypes.c_int64]),
    "vb_get_pairs_noalloc": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, _P, _P,
                                              ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "vb_get_history": (ctypes.c_int32, [_P, _P, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "vb_set_history": (ctypes.c_int32, [_P, _P, _P, ctypes.c_int32]),
    "vb_set_launch": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "vb_get_launch": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)]),
    "vb_tune": (ctypes.c_int32, [_P, ctypes.c_int32, _P]),
    "vb_force_rebuild": (ctypes.c_int32, [_P]),
    "vb_set_K": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_double]),
    "vb_set_timing": (ctypes.c_int32, [_P, ctypes.c_int32]),
    "vb_phase_times": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int64)]),
    "vb_get_info": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int64)]),
    "vb_last_error": (ctypes.c_char_p, [_P]),
    "vb_destroy": (None, [_P]),
}

_lib = None


class VbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libvbuf error {code}: {msg}")
        self.code = code


def lib():
    """The loaded library.  PyTorch is imported first so that the library binds
    to the HIP runtime PyTorch already loaded (one runtime per process)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (loads the HIP runtime the library must share)
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "python -m paper_2208_13770_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code, ctx=None):
    if code != VB_OK:
        msg = lib().vb_last_error(ctx)
        raise VbError(code, msg.decode() if msg else "")


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_params(p: dict) -> vb_params:
    """vb_params from a plain dict (the synthetic generator's parameter dicts)."""
    q = vb_params()
    q.skin_mode = int(p.get("skin_mode", VB_SKIN_LOCAL))
    q.cap_mode = int(p.get("cap_mode", 0))
    for k in ("K", "dt", "cell_size", "skin_uniform", "eps", "kn", "gamma_n", "kt", "gamma_t", "mu"):
        setattr(q, k, float(p.get(k, 0.0)))
    q.contact_capacity = int(p.get("contact_capacity", 0))
    q.lo[:] = [float(t) for t in p.get("lo", (0.0, 0.0, 0.0))]
    q.hi[:] = [float(t) for t in p.get("hi", (1.0, 1.0, 1.0))]
    q.gravity[:] = [float(t) for t in p.get("g", p.get("gravity", (0.0, 0.0, 0.0)))]
    q.max_neighbors = int(p.get("max_neighbors", 32))
    q.fixed_interval = int(p.get("fixed_interval", 1))
    q.reorder_interval = int(p.get("reorder_interval", 0))
    q.bin_capacity = int(p.get("bin_capacity", 0))
    planes = p.get("planes", ())
    if len(planes) > VB_MAX_PLANES:
        raise ValueError(f"at most {VB_MAX_PLANES} planar walls")
    q.n_planes = len(planes)
    for w, pl in enumerate(planes):
        q.planes[w][:] = [float(t) for t in pl]
    cylinders = p.get("cylinders", ())
    if len(cylinders) > VB_MAX_CYLINDERS:
        raise ValueError(f"at most {VB_MAX_CYLINDERS} cylindrical walls")
    q.n_cylinders = len(cylinders)
    for w, cy in enumerate(cylinders):
        q.cylinders[w][:] = [float(t) for t in cy]
    return q


def vb_create(params, n, stream=None):
    ctx = ctypes.c_void_p()
    q = params if isinstance(params, vb_params) else make_params(params)
    _check(lib().vb_create(ctypes.byref(q), int(n), stream if stream is not None else _stream(),
                           ctypes.byref(ctx)))
    return ctx


def vb_batch_create(params_list, n_list, stream=None):
    arr = (vb_params * len(params_list))(
        *[p if isinstance(p, vb_params) else make_params(p) for p in params_list])
    ns = (ctypes.c_int64 * len(n_list))(*[int(n) for n in n_list])
    ctx = ctypes.c_void_p()
    _check(lib().vb_batch_create(arr, ns, len(params_list),
                                 stream if stream is not None else _stream(), ctypes.byref(ctx)))
    return ctx


def _device_ptrs(*specs):
    """Addresses of the tensors in specs, (name, tensor, dtype, shape) each, after
    checking that every one is a contiguous tensor of its dtype and shape on the
    GPU: the library writes or reads exactly that many elements there, so a wrong
    buffer is refused here, before any device access.  A shape may be a callable
    (evaluated once the checks that need no context have passed).  Layouts are
    checked for every tensor before the device of any."""
    import torch
    for name, t, dtype, _ in specs:
        if not isinstance(t, torch.Tensor):
            raise ValueError(f"{name} must be a torch tensor, not {type(t).__name__}")
        if t.dtype != dtype:
            raise ValueError(f"{name} must be {dtype}, not {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
    for name, t, _, shape in specs:
        want = tuple(shape() if callable(shape) else shape)
        if tuple(t.shape) != want:
            raise ValueError(f"{name} must have shape {list(want)}, not {list(t.shape)}")
    for name, t, _, _ in specs:
        if not t.is_cuda:
            raise ValueError(f"{name} must be a GPU tensor")
    return [t.data_ptr() for _, t, _, _ in specs]


def _n_total(ctx):
    return vb_get_info(ctx)["n_total"]


def vb_set_state(ctx, x, v, rc, invm, v_is_half_step=False):
    """x, v: float64 [N,3] device tensors; rc, invm: float32 [N] device tensors."""
    import torch
    n = lambda: (_n_total(ctx),)  # noqa: E731
    px, pv, pr, pm = _device_ptrs(("x", x, torch.float64, lambda: n() + (3,)),
                                  ("v", v, torch.float64, lambda: n() + (3,)),
                                  ("rc", rc, torch.float32, n), ("invm", invm, torch.float32, n))
    _check(lib().vb_set_state(ctx, px, pv, pr, pm, int(bool(v_is_half_step))), ctx)


def vb_run(ctx, n_steps, want_history=True):
    """Advance n_steps; returns the [n_sys, n_steps] step records (or None)."""
    n_sys = vb_get_info(ctx)["n_sys"] if want_history else 0
    hist = np.zeros((n_sys, max(n_steps, 0)), dtype=STEP_RECORD_DTYPE) if want_history else None
    ptr = hist.ctypes.data_as(ctypes.c_void_p) if want_history and n_steps > 0 else None
    _check(lib().vb_run(ctx, int(n_steps), ptr), ctx)
    return hist


def vb_get_state(ctx, x=None, v=None):
    """Fills x, v (float64 [N,3] device tensors, either may be None); returns True
    when v holds the half-step velocity."""
    import torch
    shape = lambda: (_n_total(ctx), 3)  # noqa: E731
    specs = [(name, t, torch.float64, shape) for name, t in (("x", x), ("v", v)) if t is not None]
    ptrs = iter(_device_ptrs(*specs))
    px = next(ptrs) if x is not None else None
    pv = next(ptrs) if v is not None else None
    half = ctypes.c_int32(0)
    _check(lib().vb_get_state(ctx, px, pv, ctypes.byref(half)), ctx)
    return bool(half.value)


VB_NOALLOC_MAX_N = 4194304


def vb_get_pairs(ctx, sys, which, pairs=None, delta=None, noalloc=False):
    """Fills pairs (int32 [cap,2]) and delta (float64 [cap]) device tensors; returns
    the total count.  Call with pairs=None to get the count only.  noalloc=True
    calls vb_get_pairs_noalloc, which takes its scratch from the library's fixed
    array instead of the context's buffers."""
    import torch
    n = ctypes.c_int64(0)
    cap = 0
    pp = pd = None
    if pairs is not None:
        if not isinstance(pairs, torch.Tensor) or pairs.dim() != 2:
            raise ValueError("pairs must be a [cap, 2] tensor")
        cap = int(pairs.shape[0])
        specs = [("pairs", pairs, torch.int32, (cap, 2))]
        if delta is not None:
            specs.append(("delta", delta, torch.float64, (cap,)))
        ptrs = _device_ptrs(*specs)
        pp, pd = ptrs[0], (ptrs[1] if delta is not None else None)
    elif delta is not None:
        raise ValueError("delta needs pairs")
    fn = lib().vb_get_pairs_noalloc if noalloc else lib().vb_get_pairs
    _check(fn(ctx, int(sys), int(which), pp, pd, cap, ctypes.byref(n)), ctx)
    return int(n.value)


def vb_get_history(ctx, partner=None, spring=None):
    """Fills partner (int32 [N, cap]) and spring (float64 [N, cap, 3]) device
    tensors with the friction history; returns the largest contact count.  Call
    with partner=None to get the count only."""
    cap, pp, ps = _history_ptrs(ctx, partner, spring)
    need = ctypes.c_int32(0)
    code = lib().vb_get_history(ctx, pp, ps, cap, ctypes.byref(need))
    if code == VB_ECAPACITY and partner is None:
        return int(need.value)
    _check(code, ctx)
    return int(need.value)


def vb_get_verlet_state(ctx, x0r):
    """Fills x0r (float32 [N,4] device tensor: x0 and R_NL of the last broad
    phase, original order); returns (pending flags per system, step counter)."""
    import torch
    (p,) = _device_ptrs(("x0r", x0r, torch.float32, lambda: (_n_total(ctx), 4)))
    n_sys = vb_get_info(ctx)["n_sys"]
    pend = (ctypes.c_int32 * n_sys)()
    step = ctypes.c_int64(0)
    _check(lib().vb_get_verlet_state(ctx, p, pend, ctypes.byref(step)), ctx)
    return [int(t) for t in pend], int(step.value)


def vb_set_verlet_state(ctx, x0r, pending, step):
    """Loads a Verlet state (the values of vb_get_verlet_state) right after
    vb_set_state."""
    import torch
    (p,) = _device_ptrs(("x0r", x0r, torch.float32, lambda: (_n_total(ctx), 4)))
    n_sys = vb_get_info(ctx)["n_sys"]
    if len(pending) != n_sys:
        raise ValueError(f"pending must have one flag per system ({n_sys})")
    pend = (ctypes.c_int32 * n_sys)(*[int(t) for t in pending])
    _check(lib().vb_set_verlet_state(ctx, p, pend, int(step)), ctx)


def _history_ptrs(ctx, partner, spring):
    """(cap, partner address, spring address) of a friction history: partner int32
    [N, cap], spring float64 [N, cap, 3] (both None: cap 0)."""
    import torch
    if partner is None and spring is None:
        return 0, None, None
    if partner is None or spring is None:
        raise ValueError("partner and spring go together")
    if not isinstance(partner, torch.Tensor) or partner.dim() != 2:
        raise ValueError("partner must be an [N, cap] tensor")
    cap = int(partner.shape[1])
    n = lambda: (_n_total(ctx), cap)  # noqa: E731
    pp, ps = _device_ptrs(("partner", partner, torch.int32, n),
                          ("spring", spring, torch.float64, lambda: n() + (3,)))
    return cap, pp, ps


def vb_set_history(ctx, partner, spring):
    """Loads a friction history (the tensors of vb_get_history) right after
    vb_set_state."""
    cap, pp, ps = _history_ptrs(ctx, partner, spring)
    _check(lib().vb_set_history(ctx, pp, ps, cap), ctx)


def vb_set_launch(ctx, unroll=8, xcd_order=2, pairs_threads=384):
    """Launch shape of the context (results do not depend on it)."""
    _check(lib().vb_set_launch(ctx, int(unroll), int(xcd_order), int(pairs_threads)), ctx)


def vb_get_launch(ctx):
    u, x, p = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib().vb_get_launch(ctx, ctypes.byref(u), ctypes.byref(x), ctypes.byref(p)), ctx)
    return {"unroll": u.value, "xcd_order": x.value, "pairs_threads": p.value}


def vb_tune(ctx, n_steps, want_history=True):
    """vb_run that chooses the launch shape by measurement while it runs; returns
    the [n_sys, n_steps] step records (or None)."""
    n_sys = vb_get_info(ctx)["n_sys"] if want_history else 0
    hist = np.zeros((n_sys, max(n_steps, 0)), dtype=STEP_RECORD_DTYPE) if want_history else None
    ptr = hist.ctypes.data_as(ctypes.c_void_p) if want_history and n_steps > 0 else None
    _check(lib().vb_tune(ctx, int(n_steps), ptr), ctx)
    return hist


def vb_force_rebuild(ctx):
    _check(lib().vb_force_rebuild(ctx), ctx)


def vb_set_K(ctx, K, sys=-1):
    """Skin factor K for system sys (all when sys < 0), from the next broad phase."""
    _check(lib().vb_set_K(ctx, int(sys), float(K)), ctx)


def vb_set_timing(ctx, on):
    _check(lib().vb_set_timing(ctx, int(bool(on))), ctx)


def vb_phase_times(ctx):
    a, b = ctypes.c_double(0), ctypes.c_double(0)
    c, d = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().vb_phase_times(ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                ctypes.byref(d)), ctx)
    return {"ms_rebuild": a.value, "ms_step": b.value, "steps": c.value,
            "rebuild_steps": d.value}


def vb_get_info(ctx):
    n, s, w, st = ctypes.c_int64(0), ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int64(0)
    _check(lib().vb_get_info(ctx, ctypes.byref(n), ctypes.byref(s), ctypes.byref(w),
                             ctypes.byref(st)), ctx)
    return {"n_total": n.value, "n_sys": s.value, "row_width": w.value, "step": st.value}


def vb_last_error(ctx=None):
    m = lib().vb_last_error(ctx)
    return m.decode() if m else ""


def vb_destroy(ctx):
    if ctx is not None:
        lib().vb_destroy(ctx)


def state_tensors(systems, device="cuda"):
    """Concatenate synthetic systems into the device tensors vb_set_state takes:
    x, v float64 [N,3]; rc, invm float32 [N]."""
    import torch
    pos = np.concatenate([s.pos_r for s in systems], axis=0)
    vel = np.concatenate([s.vel_m for s in systems], axis=0)
    x = torch.from_numpy(pos[:, :3].astype(np.float64)).to(device)
    v = torch.from_numpy(vel[:, :3].astype(np.float64)).to(device)
    rc = torch.from_numpy(np.ascontiguousarray(pos[:, 3])).to(device)
    invm = torch.from_numpy(np.ascontiguousarray(vel[:, 3])).to(device)
    return x, v, rc, invm
