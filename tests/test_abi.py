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
