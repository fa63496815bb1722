"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
function include/vbuf.h declares, and the binding's struct layouts equal the C
compiler's."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

import paper_2208_13770_amd as vb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vbuf.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vb_[A-Za-z_]+)\s*\(", src)))


def test_header_declares_the_abi():
    names = declared_functions()
    assert "vb_create" in names and "vb_run" in names and len(names) == 21


@pytest.mark.skipif(not os.path.exists(vb.LIB_PATH), reason="libvbuf.so not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(vb.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert set(declared_functions()) == set(vb._SIGNATURES)


def test_struct_layouts_match_c():
    prog = r'''
#include <stddef.h>
#include <stdio.h>
#include "vbuf.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(vb_params), offsetof(vb_params, K),
         offsetof(vb_params, lo), offsetof(vb_params, gravity),
         offsetof(vb_params, max_neighbors), offsetof(vb_params, fixed_interval),
         offsetof(vb_params, bin_capacity), offsetof(vb_params, n_planes),
         offsetof(vb_params, planes), offsetof(vb_params, mu),
         offsetof(vb_params, contact_capacity), offsetof(vb_params, n_cylinders),
         offsetof(vb_params, cylinders));
  printf("%zu %zu %zu %zu\n", sizeof(vb_step_record), offsetof(vb_step_record, list_pairs),
         offsetof(vb_step_record, max_excess), offsetof(vb_step_record, kinetic_energy));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write(prog)
        subprocess.run(["gcc", "-std=c99", "-I" + os.path.dirname(HEADER), c, "-o", exe],
                       check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    P = vb.vb_params
    want = [ctypes.sizeof(P), P.K.offset, P.lo.offset, P.gravity.offset,
            P.max_neighbors.offset, P.fixed_interval.offset, P.bin_capacity.offset,
            P.n_planes.offset, P.planes.offset, P.mu.offset, P.contact_capacity.offset,
            P.n_cylinders.offset, P.cylinders.offset]
    assert [int(t) for t in out[:13]] == want
    R = vb.STEP_RECORD_DTYPE
    want_r = [R.itemsize, R.fields["list_pairs"][1], R.fields["max_excess"][1],
              R.fields["kinetic_energy"][1]]
    assert [int(t) for t in out[13:]] == want_r


def test_params_from_generator_dict():
    import synth
    s = synth.lattice_system(4, 4, 4, 1, 1, 0.1, 0)
    q = vb.make_params(s.params)
    assert q.K == 200.0 and q.max_neighbors == 32 and q.hi[2] == s.params["hi"][2]
    assert q.cell_size == s.params["cell_size"]


@pytest.mark.skipif(not os.path.exists(vb.LIB_PATH), reason="libvbuf.so not built")
@pytest.mark.parametrize("eps", [0.0, 1.8e-6, float("nan")])
def test_create_refuses_a_margin_below_the_fp32_floor(eps):
    """R10: the FP32 broad phase returns a superset of the exact list only with a
    positive margin of at least 16 FP32 ulps of the largest coordinate
    (2^-19 = 1.907e-6 for a unit box).  The parameters are checked before any
    device call, so this runs without a GPU."""
    import synth
    s = synth.lattice_system(4, 4, 4, 1, 1, 0.1, 0)
    assert s.params["hi"][0] == 1.0 and s.params["eps"] >= 2.0 ** -19
    with pytest.raises(vb.VbError) as e:
        vb.vb_create(dict(s.params, eps=eps), s.n, stream=ctypes.c_void_p(0))
    assert e.value.code == vb.VB_EINVAL and "eps" in str(e.value)


@pytest.mark.skipif(not os.path.exists(vb.LIB_PATH), reason="libvbuf.so not built")
def test_create_refuses_a_system_beyond_2_29_particles():
    """One system holds at most 2^29 - 256 particles (the step kernel addresses
    its 8-byte position codes with 32-bit byte offsets); the count is checked
    before any device call, so this runs without a GPU."""
    import synth
    s = synth.lattice_system(4, 4, 4, 1, 1, 0.1, 0)
    with pytest.raises(vb.VbError) as e:
        vb.vb_create(s.params, 2 ** 29 - 255, stream=ctypes.c_void_p(0))
    assert e.value.code == vb.VB_EINVAL and "too large" in str(e.value)


def _bad_params():
    """(case, mutation of a valid vb_params, expected words of the message).
    Every rejection that vb_create makes before touching the device."""
    def setf(name, value):
        return lambda q: setattr(q, name, value)

    def seta(name, i, value):
        return lambda q: getattr(q, name).__setitem__(i, value)

    def plane(values):
        def f(q):
            q.n_planes = 1
            q.planes[0][:] = values
        return f

    def cyl(values):
        def f(q):
            q.n_cylinders = 1
            q.cylinders[0][:] = values
        return f

    def fixed_zero(q):
        q.skin_mode = vb.VB_FIXED_INTERVAL
        q.fixed_interval = 0

    inf, nan = float("inf"), float("nan")
    return [
        ("skin_mode", setf("skin_mode", 4), "skin_mode"),
        ("cap_mode", setf("cap_mode", 2), "cap_mode"),
        ("dt zero", setf("dt", 0.0), "dt"),
        ("dt negative", setf("dt", -1e-5), "dt"),
        ("dt infinite", setf("dt", inf), "dt"),
        ("dt nan", setf("dt", nan), "dt"),
        ("cell_size zero", setf("cell_size", 0.0), "cell_size"),
        ("cell_size nan", setf("cell_size", nan), "cell_size"),
        ("K negative", setf("K", -1.0), "K must"),
        ("K infinite", setf("K", inf), "K must"),
        ("K nan", setf("K", nan), "K must"),
        ("skin_uniform negative", setf("skin_uniform", -0.1), "skin_uniform"),
        ("kn negative", setf("kn", -1.0), "kn and gamma_n"),
        ("gamma_n nan", setf("gamma_n", nan), "kn and gamma_n"),
        ("box empty", seta("hi", 0, 0.0), "lo < hi"),
        ("box inverted", seta("lo", 2, 2.0), "lo < hi"),
        ("box infinite", seta("hi", 1, inf), "lo < hi"),
        ("gravity nan", seta("gravity", 2, nan), "gravity"),
        ("max_neighbors zero", setf("max_neighbors", 0), "max_neighbors"),
        ("max_neighbors above the row limit", setf("max_neighbors", 129), "max_neighbors"),
        ("fixed interval zero", fixed_zero, "fixed_interval"),
        ("reorder_interval negative", setf("reorder_interval", -1), "reorder_interval"),
        ("bin_capacity negative", setf("bin_capacity", -1), "bin_capacity"),
        ("bin_capacity above the limit", setf("bin_capacity", 257), "bin_capacity"),
        ("kt negative", setf("kt", -1.0), "kt, gamma_t and mu"),
        ("mu nan", setf("mu", nan), "kt, gamma_t and mu"),
        ("contact_capacity above the limit", setf("contact_capacity", 65), "contact_capacity"),
        ("n_planes above the limit", setf("n_planes", vb.VB_MAX_PLANES + 1), "n_planes"),
        ("n_planes negative", setf("n_planes", -1), "n_planes"),
        ("plane normal not unit", plane([0.0, 0.0, 2.0, 0.1, 0.0]), "unit length"),
        ("plane nan", plane([0.0, 0.0, 1.0, nan, 0.0]), "plane values"),
        ("plane height +inf", plane([0.0, 0.0, 1.0, 0.1, inf]), "plane values"),
        ("n_cylinders above the limit", setf("n_cylinders", vb.VB_MAX_CYLINDERS + 1), "n_cylinders"),
        ("cylinder radius zero", cyl([0.5, 0.5, 0.0, 0.0]), "radii"),
        ("cylinder nan", cyl([nan, 0.5, 0.4, 0.0]), "cylinder values"),
    ]


@pytest.mark.skipif(not os.path.exists(vb.LIB_PATH), reason="libvbuf.so not built")
@pytest.mark.parametrize("case,mutate,words", _bad_params(), ids=[c[0] for c in _bad_params()])
def test_create_refuses_invalid_parameters(case, mutate, words):
    """Each parameter check of vb_create and vb_batch_create returns VB_EINVAL
    with a message that names the parameter, before any device call (so this
    runs without a GPU) and without leaving a context behind."""
    import synth
    s = synth.lattice_system(4, 4, 4, 1, 1, 0.1, 0)
    q = vb.make_params(s.params)
    mutate(q)
    with pytest.raises(vb.VbError) as e:
        vb.vb_create(q, s.n, stream=ctypes.c_void_p(0))
    assert e.value.code == vb.VB_EINVAL and words in str(e.value), str(e.value)
    # in a batch the message names the system
    good = vb.make_params(s.params)
    with pytest.raises(vb.VbError) as e:
        vb.vb_batch_create([good, q], [s.n, s.n], stream=ctypes.c_void_p(0))
    assert e.value.code == vb.VB_EINVAL and "system 1" in str(e.value) and words in str(e.value)


@pytest.mark.skipif(not os.path.exists(vb.LIB_PATH), reason="libvbuf.so not built")
def test_create_refuses_negative_counts_and_batch_sizes():
    import synth
    s = synth.lattice_system(4, 4, 4, 1, 1, 0.1, 0)
    with pytest.raises(vb.VbError) as e:
        vb.vb_create(s.params, -1, stream=ctypes.c_void_p(0))
    assert e.value.code == vb.VB_EINVAL and "n < 0" in str(e.value)
    with pytest.raises(vb.VbError) as e:
        vb.vb_batch_create([], [], stream=ctypes.c_void_p(0))
    assert e.value.code == vb.VB_EINVAL and "n_sys" in str(e.value)


@pytest.mark.skipif(not os.path.exists(vb.LIB_PATH), reason="libvbuf.so not built")
def test_every_context_call_refuses_a_null_context():
    """Every call that takes a context returns VB_EINVAL for a NULL one, with
    vb_last_error(NULL) saying so; vb_destroy(NULL) does nothing; the create
    calls refuse a NULL output handle.  No device call is made."""
    L = vb.lib()
    skip = {"vb_create", "vb_batch_create", "vb_last_error", "vb_destroy"}
    called = []
    for name, (res, args) in vb._SIGNATURES.items():
        if name in skip:
            continue
        vals = []
        for t in args:
            if t is ctypes.c_double:
                vals.append(0.0)
            elif t in (ctypes.c_int32, ctypes.c_int64):
                vals.append(0)
            else:
                vals.append(None)
        assert getattr(L, name)(*vals) == vb.VB_EINVAL, name
        assert L.vb_last_error(None) == b"ctx is NULL", name
        called.append(name)
    assert len(called) == 17
    L.vb_destroy(None)
    import synth
    s = synth.lattice_system(4, 4, 4, 1, 1, 0.1, 0)
    q = vb.make_params(s.params)
    assert L.vb_create(ctypes.byref(q), s.n, None, None) == vb.VB_EINVAL
    assert L.vb_last_error(None) == b"out is NULL"
    n = (ctypes.c_int64 * 1)(s.n)
    assert L.vb_batch_create(ctypes.byref(q), n, 1, None, None) == vb.VB_EINVAL
    assert L.vb_last_error(None) == b"out is NULL"
