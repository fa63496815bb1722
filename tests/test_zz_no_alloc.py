"""The allocation-free pair export, vb_get_pairs_noalloc, through the C ABI: the
same pairs and overlaps as vb_get_pairs, which uses the context's own scratch.
Two calls in a row, the second with a smaller input (the fixed scratch keeps the
first call's contents), in separate contexts and within one batch; a system
larger than the fixed scratch is refused."""
import numpy as np
import pytest

import paper_2208_13770_amd as vb
import synth
from tests._gpu import GpuSession, say

pytestmark = pytest.mark.gpu


def export(ctx, sys, which, noalloc):
    import torch
    n = vb.vb_get_pairs(ctx, sys, which, noalloc=noalloc)
    p = torch.full((max(n, 1), 2), -7, dtype=torch.int32, device="cuda")
    d = torch.full((max(n, 1),), float("nan"), dtype=torch.float64, device="cuda")
    m = vb.vb_get_pairs(ctx, sys, which, p, d, noalloc=noalloc)
    assert m == n
    return n, p[:n].cpu().numpy(), d[:n].cpu().numpy()


def same(a, b, what):
    assert a[0] == b[0], (what, a[0], b[0])
    assert np.array_equal(a[1], b[1]), what
    assert np.array_equal(a[2], b[2]), what
    assert not np.isnan(a[2]).any(), what


def test_noalloc_export_equals_the_context_export():
    big = synth.config_systems("M1", seed=21)[0]
    small = synth.lattice_system(10, 9, 7, 2, 1, 0.2, seed=22)
    assert small.n < big.n
    for s in (big, small):  # the second call has the smaller input
        say(f"allocation-free export: N={s.n}")
        with GpuSession([s]) as g:
            g.run(40)
            for which in (0, 1):
                got = export(g.ctx, 0, which, True)
                ref = export(g.ctx, 0, which, False)
                same(ref, got, f"N={s.n} which={which}")
                assert got[0] > 0
    with GpuSession([big, small]) as g:  # one batch: system 0, then the smaller system 1
        g.run(25)
        for sys in (0, 1):
            same(export(g.ctx, sys, 0, False), export(g.ctx, sys, 0, True), f"batch system {sys}")


def test_noalloc_export_at_and_beyond_its_limit():
    at = synth.config_systems("M2", seed=0)[0]
    assert at.n == vb.VB_NOALLOC_MAX_N
    say(f"allocation-free export at the limit: N={at.n}")
    with GpuSession([at]) as g:
        g.run(3)
        same(export(g.ctx, 0, 1, False), export(g.ctx, 0, 1, True), "M2")
    over = synth.lattice_system(257, 256, 64, 0, 0, 0.0, seed=1)
    assert over.n > vb.VB_NOALLOC_MAX_N
    with GpuSession([over]) as g:
        with pytest.raises(vb.VbError) as e:
            vb.vb_get_pairs(g.ctx, 0, 0, noalloc=True)
        assert e.value.code == vb.VB_EINVAL and "allocation-free" in str(e.value)
