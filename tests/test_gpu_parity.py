"""Parity of the HIP path (through the C ABI) with the FP64 oracle, on the GPU.

Bar (stated once, used everywhere): after a run, positions within 1e-5 box units
and velocities within 1e-5 v_max of the oracle, element by element.  The HIP path
keeps positions and velocities in FP64 and evaluates the contact law and the
integration in the oracle's order with every operation rounded (no contraction,
the contact normal by division, correctly rounded square root and division), so
positions and velocities come out bit for bit equal to the oracle's, which
every comparison below also asserts; the kinetic energy differs only by its
summation order (rtol 1e-9).  Contact sets, contact counts and the reproduced
closed-form rebuild cadences are compared exactly.  The broad phase and the
validity test run in FP32 with the eps margin, so the Verlet list and the
rebuild schedule may differ from the oracle's only at near-ties of those FP32
tests; such differences are checked to be near-ties, and the results (which by
the theorem of Sec. 4.2 do not depend on the list) are still compared bit for
bit.
"""
import numpy as np
import pytest

import oracle
import paper_2208_13770_amd as vb
import synth
from tests._gpu import GpuSession, gpu_trajectory, host_arrays, say

pytestmark = pytest.mark.gpu

TOL_X = 1e-5      # box units
TOL_V = 1e-5      # units of v_max


def oracle_run(systems_or_one, steps, **overrides):
    s = systems_or_one
    x, v, rc, invm = host_arrays([s])
    return oracle.run(dict(s.params, **overrides), x, v, rc, invm, steps)


def assert_close(sys_, xg, vg, xo, vo, what):
    ex = np.abs(xg - xo).max() if len(xo) else 0.0
    ev = np.abs(vg - vo).max() / sys_.meta.get("v_max", 1.0) if len(vo) else 0.0
    nd = int((xg != xo).sum() + (vg != vo).sum())
    say(f"  {what}: max|dx| = {ex:.3e} box units, max|dv| = {ev:.3e} v_max, "
        f"{nd} of {xo.size + vo.size} values differ from the oracle's")
    assert ex <= TOL_X and ev <= TOL_V, (what, ex, ev)
    assert nd == 0, (what, "not bit for bit", nd)
    return ex, ev


RECORD_EXACT = ("step", "rebuilt", "list_pairs", "contacts", "violators", "max_excess")


def assert_same_records(ha, hb, what):
    """Two runs' step records agree: every field exactly, the kinetic energy up to
    the order of its sum over tiles (which follows the storage order)."""
    for f in RECORD_EXACT:
        assert np.array_equal(ha[f], hb[f]), (what, f)
    assert np.allclose(ha["kinetic_energy"], hb["kinetic_energy"], rtol=1e-12, atol=0), what


def check_schedule(hg, ho, what):
    """Rebuild schedules agree up to the first difference, which must be a
    near-tie of the validity test (the oracle's max excess there is ~0)."""
    rg, ro = hg["rebuilt"].astype(bool), ho["rebuilt"].astype(bool)
    diff = np.nonzero(rg != ro)[0]
    say(f"  {what}: {int(rg.sum())} broad phases (oracle {int(ro.sum())}), "
        f"first difference at {diff[0] if len(diff) else None}")
    if len(diff):
        n = diff[0]
        assert n > 0 and abs(ho["max_excess"][n - 1]) < 1e-6, (n, ho["max_excess"][n - 1])


# --------------------------------------------------------------------- M1

@pytest.mark.parametrize("seed", [0, 1])
def test_m1_parity_with_oracle(seed):
    """The small workload (16,384 particles, 200 steps, K = 200): GPU vs oracle."""
    s = synth.config_systems("M1", seed=seed)[0]
    say(f"M1 seed {seed}: N={s.n}, 200 steps")
    with GpuSession([s]) as g:
        hg = g.run(200)
        xg, vg, _ = g.state()
        n_list = vb.vb_get_pairs(g.ctx, 0, 0)
    assert hg[0]["list_pairs"][-1] == n_list  # the record counts the list in use
    xo, vo, ho, _ = oracle_run(s, 200)
    assert_close(s, xg, vg, xo, vo, "M1")
    assert np.array_equal(hg[0]["contacts"], ho["contacts"])
    assert ho["contacts"].max() > 100
    assert np.allclose(hg[0]["kinetic_energy"], ho["kinetic_energy"], rtol=1e-9, atol=0)
    check_schedule(hg[0], ho, "M1")
    assert hg[0]["rebuilt"][0] == 1


def test_k_invariance_bitwise():
    """Theorem of Sec. 4.2 on the GPU: the local buffer (K = 200, K = 10), the
    uniform skin and the broad phase at every step give bit-identical results."""
    s = synth.config_systems("M1", seed=3)[0]
    ref = None
    for name, ov in (("no buffer", {"skin_mode": 2}), ("K=200", {}), ("K=10", {"K": 10.0}),
                     ("uniform", {"skin_mode": 1}), ("K=5000", {"K": 5000.0})):
        say(f"K-invariance: {name}")
        x, v, h = gpu_trajectory([s], 150, **ov)
        if ref is None:
            ref = (x, v, h)
            assert h[0]["rebuilt"].all()
            continue
        assert np.array_equal(x, ref[0]) and np.array_equal(v, ref[1]), name
        assert np.array_equal(h[0]["contacts"], ref[2][0]["contacts"]), name
        if name == "K=200":
            assert h[0]["rebuilt"].sum() < 20


def test_run_to_run_determinism():
    s = synth.config_systems("M1", seed=4)[0]
    say("determinism: two identical runs")
    a = gpu_trajectory([s], 120)
    b = gpu_trajectory([s], 120)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])


# --------------------------------------------------------------------- lists

def test_verlet_list_matches_oracle_broad_phase():
    """The first broad phase (Alg. 1 on Eq. bounding_sphere spheres with the local
    skin) vs the oracle's: every pair the oracle includes with margin > 1e-6 is in
    the GPU list, and every GPU pair lies within 1e-6 of the inclusion bound."""
    s = synth.config_systems("M1", seed=5)[0]
    x, v, rc, invm = host_arrays([s])
    with GpuSession([s]) as g:
        say("list at step 0")
        g.pairs(0, 1)  # runs the step-0 broad phase
        gl, _ = g.pairs(0, 0)
    rnl, _ = oracle.rebuild_radii(s.params, v, rc)
    eps = s.params["eps"]
    ol = oracle.broadphase_brute(x, rnl + 1e-6, eps)  # oracle pairs, widened by the tolerance

    def margin(p):
        d = np.linalg.norm(x[p[:, 0]] - x[p[:, 1]], axis=1)
        return rnl[p[:, 0]] + rnl[p[:, 1]] + eps - d

    gset = set(map(tuple, gl.tolist()))
    sure = ol[margin(ol) > 1e-6]
    missing = [t for t in map(tuple, sure.tolist()) if t not in gset]
    assert not missing, missing[:5]
    assert (margin(gl) > -1e-6).all()
    assert np.all(gl[:, 0] < gl[:, 1])
    assert np.array_equal(gl, gl[np.lexsort((gl[:, 1], gl[:, 0]))])
    say(f"  GPU list {len(gl)} pairs, oracle {len(sure)} sure pairs")


def test_contacts_equal_brute_force_after_run():
    """After 150 steps, the contact set the GPU reports (narrow phase on its list,
    Eq. delta) equals brute force over all pairs at the GPU's own positions."""
    s = synth.config_systems("M1", seed=6)[0]
    _, _, rc, _ = host_arrays([s])
    with GpuSession([s]) as g:
        say("contacts after 150 steps")
        g.run(150)
        xg, _, _ = g.state()
        gc, gd = g.pairs(0, 1)
    oc = oracle.contacts_brute(xg, rc)
    assert len(oc) > 100
    assert np.array_equal(gc, oc)
    d = rc[oc[:, 0]] + rc[oc[:, 1]] - np.linalg.norm(xg[oc[:, 0]] - xg[oc[:, 1]], axis=1)
    assert np.abs(gd - d).max() < 1e-15


def test_pair_export_into_a_short_buffer():
    """vb_get_pairs reports the full count and writes the first cap pairs of the
    canonical (sorted) list when the buffer is shorter; NULL buffers give the
    count alone."""
    import torch
    import paper_2208_13770_amd as vb
    s = synth.config_systems("M1", seed=6)[0]
    with GpuSession([s]) as g:
        g.run(40)
        full, fd = g.pairs(0, 0)
        n = len(full)
        assert n > 100 and vb.vb_get_pairs(g.ctx, 0, 0) == n
        cap = n // 3
        p = torch.full((cap, 2), -7, dtype=torch.int32, device="cuda")
        d = torch.zeros(cap, dtype=torch.float64, device="cuda")
        assert vb.vb_get_pairs(g.ctx, 0, 0, p, d) == n
        assert np.array_equal(p.cpu().numpy(), full[:cap])
        assert np.array_equal(d.cpu().numpy(), fd[:cap])
        assert (full[:, 0] < full[:, 1]).all()
        assert (np.diff(full[:, 0] * (s.n + 1) + full[:, 1]) > 0).all()


# --------------------------------------------------------------------- cadence

@pytest.mark.parametrize("K", [0, 7, 50])
def test_free_flight_cadence_on_gpu(K):
    """Sec. 4.1: in free flight every particle violates Eq. update after exactly
    K+1 drifts; the GPU's FP32 test reproduces the cadence exactly (dyadic data)."""
    s = synth.free_flight_system(4, [2.0 ** -4, 2.0 ** -5, 2.0 ** -6], seed=K, K=float(K))
    say(f"free flight K={K}")
    _, _, h = gpu_trajectory([s], 300)
    expect = np.zeros(300, dtype=np.int32)
    expect[:: K + 1] = 1
    assert np.array_equal(h[0]["rebuilt"], expect)
    assert h[0]["contacts"].sum() == 0


def test_capped_cadence_and_literal_cap_on_gpu():
    """Eq. skin_formulus_mincell: capped skins set the period (769 steps here), in
    both cap readings (half cell with one ring, full cell with two rings)."""
    s = synth.free_flight_system(3, [2.0 ** -4, 2.0 ** -6], seed=1, K=5000.0)
    for cap_mode, period in ((0, 769), (1, 1793)):
        say(f"capped cadence, cap mode {cap_mode}")
        _, _, h = gpu_trajectory([s], 1800, cap_mode=cap_mode)
        expect = np.zeros(1800, dtype=np.int32)
        expect[::period] = 1
        assert np.array_equal(h[0]["rebuilt"], expect)


def test_literal_cap_parity():
    s = synth.lattice_system(10, 9, 7, 3, 2, 0.2, 21)
    say("cap mode 1 parity")
    xg, vg, hg = gpu_trajectory([s], 150, cap_mode=1)
    xo, vo, ho, _ = oracle_run(s, 150, cap_mode=1)
    assert_close(s, xg, vg, xo, vo, "cap mode 1")
    assert np.array_equal(hg[0]["contacts"], ho["contacts"])


# --------------------------------------------------------------------- shapes

def test_ragged_and_empty_systems_in_one_batch():
    """A batch of systems with 0, 1, 2, 255, 256, 257 and 315 particles: each
    matches its own oracle run (ragged tiles, empty system, lone particle)."""
    shapes = [(0, 1, 1), (1, 1, 1), (2, 1, 1), (15, 17, 1), (16, 16, 1), (257, 1, 1), (7, 9, 5)]
    systems = []
    for i, (a, b, c) in enumerate(shapes):
        if a * b * c == 0:
            s = synth.lattice_system(1, 1, 1, 0, 0, 0.0, 100 + i)
            s.pos_r = s.pos_r[:0].copy()
            s.vel_m = s.vel_m[:0].copy()
        else:
            s = synth.lattice_system(a, b, c, 1, 1, 0.3, 100 + i)
        systems.append(s)
    say("ragged batch", [s.n for s in systems])
    with GpuSession(systems) as g:
        h = g.run(80)
        xg, vg, _ = g.state()
    off = 0
    for k, s in enumerate(systems):
        xo, vo, ho, _ = oracle_run(s, 80)
        sl = slice(off, off + s.n)
        assert_close(s, xg[sl], vg[sl], xo, vo, f"system {k} (N={s.n})")
        assert np.array_equal(h[k]["contacts"], ho["contacts"])
        off += s.n


def test_batch_equals_single_runs_bitwise():
    systems = [synth.lattice_system(*d, 2, 1, 0.2, 200 + i)
               for i, d in enumerate([(12, 10, 6), (5, 30, 4), (20, 20, 3)])]
    say("batch vs singles")
    xb, vb_, hb = gpu_trajectory(systems, 100)
    off = 0
    for k, s in enumerate(systems):
        x1, v1, h1 = gpu_trajectory([s], 100)
        sl = slice(off, off + s.n)
        assert np.array_equal(xb[sl], x1) and np.array_equal(vb_[sl], v1)
        assert np.array_equal(hb[k]["rebuilt"], h1[0]["rebuilt"])
        off += s.n


def test_row_overflow_is_regrown():
    """Rows narrower than the list: the call grows them and reruns; results are
    bit-identical to wide rows (theorem of Sec. 4.2)."""
    s = synth.config_systems("M1", seed=7)[0]
    say("row overflow")
    xw, vw, hw = gpu_trajectory([s], 100, max_neighbors=64)
    with GpuSession([s], {"max_neighbors": 2}) as g:
        hn = g.run(100)
        xn, vn, _ = g.state()
        assert g.info()["row_width"] > 2
    assert np.array_equal(xw, xn) and np.array_equal(vw, vn)
    # the run again starts from a snapshot whose rows are rebuilt from its x0 and
    # R_NL: the schedule of broad phases is that of a run that never overflowed
    assert_same_records(hw[0], hn[0], "row overflow")


def test_overflow_stops_a_long_call_early():
    """A 1,100-step call whose rows overflow at once stops launching after its
    first blocks of steps, grows the rows and runs again from its start: the
    state is bit-identical to wide rows, and the records and timing cover every
    step of the call (contacts and kinetic energy equal those of the wide run)."""
    import paper_2208_13770_amd as vb
    s = synth.config_systems("M1", seed=5)[0]
    say("overflow in a long call")
    n = 1100
    xw, vw, hw = gpu_trajectory([s], n, max_neighbors=64)
    with GpuSession([s], {"max_neighbors": 2}) as g:
        vb.vb_set_timing(g.ctx, 1)
        h = g.run(n)
        pt = vb.vb_phase_times(g.ctx)
        xn, vn, _ = g.state()
        assert g.info()["row_width"] > 2 and g.info()["step"] == n
    assert np.array_equal(xw, xn) and np.array_equal(vw, vn)
    assert len(h[0]) == n and h[0]["step"].tolist() == list(range(n))
    assert_same_records(hw[0], h[0], "long call")
    assert np.array_equal(h[0]["kinetic_energy"], hw[0]["kinetic_energy"])
    assert pt["steps"] == n and pt["rebuild_steps"] == int(h[0]["rebuilt"].sum())


def test_checkpoint_resume_bitwise():
    """Resume from (x^n, v^{n-1/2}) in a new context continues bit-identically."""
    import torch
    import paper_2208_13770_amd as vb
    s = synth.config_systems("M1", seed=8)[0]
    say("checkpoint/resume")
    xa, va, _ = gpu_trajectory([s], 200)
    with GpuSession([s]) as g:
        g.run(120)
        x1, v1, half = g.state()
        assert half
    with GpuSession([s]) as g:
        vb.vb_set_state(g.ctx, torch.from_numpy(x1).cuda(), torch.from_numpy(v1).cuda(), g.rc,
                        g.invm, v_is_half_step=True)
        g.run(80)
        xb, vb2, _ = g.state()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb2)


@pytest.mark.parametrize("case,n1,n2", [("M1", 120, 80), ("M1 friction", 120, 80),
                                        ("hopper", 900, 400)])
def test_verlet_state_checkpoint_resumes_the_schedule(case, n1, n2):
    """Sec. 4.2: besides positions and velocities the method carries, from one
    step to the next, the reference positions x0 and extended radii R_NL of the
    last broad phase and whether the validity test failed (Eq. update, Def.
    autoverlet).  n1 + n2 steps equal n1 steps, a checkpoint (state, Verlet state
    and, under friction, the contact history) and n2 steps in a new context: positions
    and velocities bit for bit, and every record field, the broad-phase schedule
    included (the kinetic energy up to its summation order)."""
    import torch
    import paper_2208_13770_amd as vb
    if case == "hopper":
        s = synth.hopper_system(3654, 5)
        ov = {}
    else:
        s = synth.config_systems("M1", seed=12)[0]
        ov = _frictional(s) if case == "M1 friction" else {}
    say(f"Verlet-state checkpoint: {case}, N={s.n}")
    with GpuSession([s], ov) as g:
        ha = g.run(n1 + n2)
        xa, va, _ = g.state()
    x0r = torch.empty((s.n, 4), dtype=torch.float32, device="cuda")
    with GpuSession([s], ov) as g:
        h1 = g.run(n1)
        x1, v1, half = g.state()
        pending, step = vb.vb_get_verlet_state(g.ctx, x0r)
        assert half and step == n1
        if ov:
            need = vb.vb_get_history(g.ctx)
            partner = torch.empty((s.n, need), dtype=torch.int32, device="cuda")
            spring = torch.empty((s.n, need, 3), dtype=torch.float64, device="cuda")
            vb.vb_get_history(g.ctx, partner, spring)
    with GpuSession([s], ov) as g:
        vb.vb_set_state(g.ctx, torch.from_numpy(x1).cuda(), torch.from_numpy(v1).cuda(), g.rc,
                        g.invm, v_is_half_step=True)
        vb.vb_set_verlet_state(g.ctx, x0r, pending, step)
        if ov:
            vb.vb_set_history(g.ctx, partner, spring)
        h2 = g.run(n2)
        xb, vb2, _ = g.state()
        assert g.info()["step"] == n1 + n2
    say(f"  pending at the checkpoint {pending}, broad phases after it "
        f"{int(ha[0]['rebuilt'][n1:].sum())}, contacts after it {int(ha[0]['contacts'][n1:].sum())}")
    assert np.array_equal(xa, xb) and np.array_equal(va, vb2)
    assert_same_records(ha[0][:n1], h1[0], case)
    assert_same_records(ha[0][n1:], h2[0], case)
    assert h2[0]["rebuilt"][0] == pending[0] and ha[0]["rebuilt"][n1:].sum() >= 1
    assert ha[0]["contacts"][n1:].sum() > 0


def test_verlet_state_input_is_checked():
    import torch
    import paper_2208_13770_amd as vb
    s = synth.config_systems("M1", scale=0.5, seed=2)[0]
    x0r = torch.empty((s.n, 4), dtype=torch.float32, device="cuda")
    with GpuSession([s]) as g:
        with pytest.raises(vb.VbError) as e:  # no list before the first step
            vb.vb_get_verlet_state(g.ctx, x0r)
        assert e.value.code == vb.VB_EINVAL
        g.run(30)
        pending, step = vb.vb_get_verlet_state(g.ctx, x0r)
        with pytest.raises(vb.VbError) as e:  # only right after vb_set_state
            vb.vb_set_verlet_state(g.ctx, x0r, pending, step)
        assert e.value.code == vb.VB_EINVAL
        good = x0r.clone()
        for name, bad, code in (
                ("R_NL below R_C", lambda t: t[:, 3].mul_(0.5), vb.VB_EINVAL),
                ("R_NL beyond the cap", lambda t: t[:, 3].fill_(s.params["cell_size"]), vb.VB_EINVAL),
                ("NaN", lambda t: t[7, 1].fill_(float("nan")), vb.VB_ENONFINITE)):
            t = good.clone()
            bad(t)
            vb.vb_set_state(g.ctx, g.x, g.v, g.rc, g.invm)
            with pytest.raises(vb.VbError) as e:
                vb.vb_set_verlet_state(g.ctx, t, pending, step)
            assert e.value.code == code, name
        vb.vb_set_state(g.ctx, g.x, g.v, g.rc, g.invm)
        for bad_pending, bad_step in (([2], step), (pending, -1)):
            with pytest.raises(vb.VbError) as e:
                vb.vb_set_verlet_state(g.ctx, good, bad_pending, bad_step)
            assert e.value.code == vb.VB_EINVAL
        vb.vb_set_verlet_state(g.ctx, good, pending, step)
        g.run(5)


def test_overflow_late_in_a_call_runs_again_from_a_snapshot():
    """A lattice in free fall: every skin grows with the speed (Eq.
    skin_formulus1), so each broad phase lists more neighbours, and rows of 8
    overflow only some 300 steps into a 560-step call, after the call's
    snapshot at step 257.  The call grows the rows and runs again from that
    snapshot; state and records equal those of wide rows bit for bit, and both
    equal the oracle."""
    s = synth.lattice_system(16, 16, 8, 0, 0, 0.0, seed=3)
    a, dt = s.meta["a"], s.params["dt"]
    s.params["g"] = (0.0, 0.0, float(np.float32(-3.25e-6 * a / dt ** 2)))
    n = 560
    say("late overflow in one call")
    with GpuSession([s], {"max_neighbors": 32}) as g:
        hw = g.run(n)
        xw, vw, _ = g.state()
    with GpuSession([s], {"max_neighbors": 8}) as g:
        hn = g.run(n)
        xn, vn, _ = g.state()
        assert g.info()["row_width"] > 8
    rows = 2 * hw[0]["list_pairs"] / s.n
    first_wide = int(np.argmax(rows > 6.0))
    say(f"  mean row length reaches 6+ at step {first_wide}; broad phases {int(hw[0]['rebuilt'].sum())}")
    assert first_wide > 257
    assert np.array_equal(xw, xn) and np.array_equal(vw, vn)
    assert_same_records(hw[0], hn[0], "late overflow")
    xo, vo, ho, _ = oracle_run(s, n)
    assert_close(s, xn, vn, xo, vo, "free fall")


# --------------------------------------------------------------------- errors

def test_error_paths():
    import torch
    import paper_2208_13770_amd as vb
    s = synth.lattice_system(4, 4, 4, 1, 1, 0.1, 0)
    say("error paths")
    with pytest.raises(vb.VbError) as e:
        vb.vb_create(dict(s.params, dt=-1.0), s.n)
    assert e.value.code == vb.VB_EINVAL
    with pytest.raises(vb.VbError) as e:
        vb.vb_create(dict(s.params, max_neighbors=1000), s.n)
    assert e.value.code == vb.VB_EINVAL
    ctx = vb.vb_create(s.params, s.n)
    try:
        with pytest.raises(vb.VbError) as e:
            vb.vb_run(ctx, 5)
        assert e.value.code == vb.VB_EINVAL
        x, v, rc, invm = vb.state_tensors([s])
        xb = x.clone()
        xb[3, 1] = float("nan")
        with pytest.raises(vb.VbError) as e:
            vb.vb_set_state(ctx, xb, v, rc, invm)
        assert e.value.code == vb.VB_ENONFINITE
        rb = rc.clone()
        rb[0] = float(s.params["cell_size"])
        with pytest.raises(vb.VbError) as e:
            vb.vb_set_state(ctx, x, v, rb, invm)
        assert e.value.code == vb.VB_EINVAL
        vb.vb_set_state(ctx, x, v, rc, invm)
        h = vb.vb_run(ctx, 3)
        assert h.shape == (1, 3)
        with pytest.raises(vb.VbError):
            vb.vb_get_pairs(ctx, 1, 0)
    finally:
        vb.vb_destroy(ctx)
    torch.cuda.synchronize()


def test_diverged_state_is_reported():
    """A state that leaves the finite numbers during a call (here a velocity whose
    kinetic energy overflows) is reported as VB_ENONFINITE; the context then needs
    a new state, after which it runs as a fresh one does (bitwise)."""
    import torch
    import paper_2208_13770_amd as vb
    s = synth.lattice_system(4, 4, 4, 1, 1, 0.1, 0)
    say("diverged state: 100 steps with |v| = 1e160 for one particle")
    x, v, rc, invm = vb.state_tensors([s])
    vbad = v.clone()
    vbad[5, 0] = 1e160
    ctx = vb.vb_create(s.params, s.n)
    try:
        vb.vb_set_state(ctx, x, vbad, rc, invm)
        with pytest.raises(vb.VbError) as e:
            vb.vb_run(ctx, 100)
        assert e.value.code == vb.VB_ENONFINITE
        assert "step 0" in str(e.value)
        with pytest.raises(vb.VbError) as e:
            vb.vb_run(ctx, 1)
        assert e.value.code == vb.VB_EINVAL
        vb.vb_set_state(ctx, x, v, rc, invm)
        vb.vb_run(ctx, 100)
        xa, va = torch.empty_like(x), torch.empty_like(v)
        vb.vb_get_state(ctx, xa, va)
    finally:
        vb.vb_destroy(ctx)
    xb, vb2, _ = gpu_trajectory([s], 100)
    assert np.array_equal(xa.cpu().numpy(), xb) and np.array_equal(va.cpu().numpy(), vb2)


def test_bin_overflow_is_regrown():
    """Cell bins smaller than the cells' occupancy: the call grows them and reruns;
    results are bit-identical."""
    s = synth.config_systems("M1", seed=9)[0]
    say("bin overflow")
    xw, vw, hw = gpu_trajectory([s], 60)
    xn, vn, hn = gpu_trajectory([s], 60, bin_capacity=1)
    assert np.array_equal(xw, xn) and np.array_equal(vw, vn)
    assert_same_records(hw[0], hn[0], "bin overflow")


def test_periodic_storage_sort_changes_nothing():
    """Re-sorting the particle storage by cell every few steps (for locality) moves
    every slot; results stay bit-identical (sums run in original index order),
    and since x0 and R_NL move with their particles and the rows are rebuilt from
    them, the schedule of broad phases and every record are unchanged too."""
    s = synth.config_systems("M1", seed=10)[0]
    say("periodic storage sort")
    xa, va, ha = gpu_trajectory([s], 150)
    xb, vb_, hb = gpu_trajectory([s], 150, reorder_interval=7)
    assert np.array_equal(xa, xb) and np.array_equal(va, vb_)
    assert_same_records(ha[0], hb[0], "storage sort")
    assert 1 < ha[0]["rebuilt"].sum() < 150 // 7


def test_k_sweep_rows_identical_to_no_buffer(tmp_path):
    """The K experiment on M1: every K and the uniform skin reproduce the run
    without buffer bit for bit, K = 0 rebuilds at (nearly) every step, larger K
    rebuilds less, and the summary row names an optimum."""
    import json
    from paper_2208_13770_amd import sweep
    out = tmp_path / "sweep.json"
    say("K sweep on M1, 150 steps")
    sweep.main(["--workload", "M1", "--steps", "150", "--repeats", "2", "--out", str(out)])
    res = json.loads(out.read_text())
    rows = {r["case"]: r for r in res["rows"]}
    k_opt = res["summary"]["k_opt"]
    assert rows[f"K={k_opt:g}"]["overhead_to_opt_pct"] == 0.0
    assert all(r["overhead_to_opt_pct"] >= 0.0 for r in res["rows"] if r["K"] is not None)
    assert rows["K=200"]["runs"] == 2
    for name, r in rows.items():
        if not name.startswith("fixed"):
            assert r["identical_to_no_buffer"], name
    assert rows["no buffer"]["executed_pct"] == 100.0
    assert rows["K=0"]["executed_pct"] > 90.0
    assert rows["K=5000"]["broad_phases"] < rows["K=10"]["broad_phases"]
    assert res["summary"]["k_opt"] in sweep.K_SWEEP
    assert rows["auto (tuned K)"]["identical_to_no_buffer"]


def test_changing_K_mid_run_changes_nothing():
    """vb_set_K between vb_run calls (what the tuner does): bit-identical to the
    broad phase at every step (Sec. 4.2); invalid K values are refused."""
    import paper_2208_13770_amd as vb
    s = synth.config_systems("M1", seed=5)[0]
    say("K changed between calls: 200 -> 10 -> 5000 -> 0 -> 100")
    xr, vr, hr = gpu_trajectory([s], 160, skin_mode=2)
    with GpuSession([s]) as g:
        for K, n in ((200.0, 40), (10.0, 30), (5000.0, 40), (0.0, 20), (100.0, 30)):
            vb.vb_set_K(g.ctx, K)
            g.run(n)
        x, v, _ = g.state()
        for bad in (-1.0, float("nan"), float("inf")):
            with pytest.raises(vb.VbError):
                vb.vb_set_K(g.ctx, bad)
        with pytest.raises(vb.VbError):
            vb.vb_set_K(g.ctx, 1.0, sys=3)
    assert np.array_equal(x, xr) and np.array_equal(v, vr)


@pytest.mark.parametrize("name,scale,steps", [("H125", 0.3, 2500), ("INCLINE", 0.15, 2500)])
def test_gravity_plane_workloads_parity(name, scale, steps):
    """Gravity, polydisperse radii and planar walls (hopper sides with an outlet,
    tilted gravity on a floor): GPU vs oracle, element by element."""
    s = synth.config_systems(name, scale=scale)[0]
    say(f"{name} at scale {scale}: N={s.n}, {steps} steps, {len(s.params['planes'])} planes")
    xg, vg, hg = gpu_trajectory([s], steps)
    xo, vo, ho, _ = oracle_run(s, steps)
    assert_close(s, xg, vg, xo, vo, name)
    assert np.array_equal(hg[0]["contacts"], ho["contacts"])
    assert ho["contacts"].max() > 20
    check_schedule(hg[0], ho, name)


def test_silo_cylinder_parity(scale=0.3, steps=2500):
    """The silo stand-in (a vertical cylinder wall open below its lower edge,
    polydisperse radii, gravity) at reduced size against the oracle, element by
    element, while its grains discharge through the ring under the wall."""
    s = synth.config_systems("SILO", scale=scale)[0]
    say(f"SILO at scale {scale}: N={s.n}, {steps} steps, cylinder {s.params['cylinders'][0]}")
    xg, vg, hg = gpu_trajectory([s], steps)
    xo, vo, ho, _ = oracle_run(s, steps)
    assert_close(s, xg, vg, xo, vo, "SILO")
    assert np.array_equal(hg[0]["contacts"], ho["contacts"])
    assert ho["contacts"].max() > 20
    check_schedule(hg[0], ho, "SILO")


def test_silo_cylinder_k_invariance_bitwise():
    s = synth.config_systems("SILO", scale=0.3)[0]
    say(f"silo K-invariance: N={s.n}")
    ref = gpu_trajectory([s], 300, skin_mode=2)
    for ov in ({}, {"K": 20.0}, {"K": 2000.0}):
        x, v, h = gpu_trajectory([s], 300, **ov)
        assert np.array_equal(x, ref[0]) and np.array_equal(v, ref[1]), ov


def test_cylinder_parameters_are_checked():
    import paper_2208_13770_amd as vb
    s = synth.silo_system(500, 3)
    for cyl in ([(0.5, 0.5, 0.0, 0.0)], [(0.5, float("nan"), 0.3, 0.0)], [(0.5, 0.5, -0.2, 0.0)]):
        with pytest.raises(vb.VbError) as e:
            vb.vb_create(dict(s.params, cylinders=cyl), s.n)
        assert e.value.code == vb.VB_EINVAL
    with pytest.raises(ValueError):
        vb.make_params(dict(s.params, cylinders=[(0.5, 0.5, 0.3, 0.0)] * 3))


def test_gravity_plane_k_invariance_bitwise():
    s = synth.config_systems("H125", scale=0.35)[0]
    say(f"hopper K-invariance: N={s.n}")
    ref = gpu_trajectory([s], 300, skin_mode=2)
    for ov in ({}, {"K": 20.0}, {"K": 2000.0}):
        x, v, h = gpu_trajectory([s], 300, **ov)
        assert np.array_equal(x, ref[0]) and np.array_equal(v, ref[1]), ov
        assert np.array_equal(h[0]["contacts"], ref[2][0]["contacts"])


def test_plane_parameters_are_checked():
    import paper_2208_13770_amd as vb
    s = synth.config_systems("M1", scale=0.25)[0]
    for planes in ([(0.0, 0.0, 2.0, 0.0, 0.0)], [(float("nan"), 0.0, 1.0, 0.0, 0.0)],
                   [(0.0, 0.0, 1.0, 0.0, 0.0)] * 5):
        with pytest.raises((vb.VbError, ValueError)):
            vb.vb_create(dict(s.params, planes=planes), s.n)


# ---------------------------------------------------------------- friction
def _frictional(s, mu=0.4):
    return {"kt": 0.5 * s.params["kn"], "gamma_t": 0.5 * s.params["gamma_n"], "mu": mu}


@pytest.mark.parametrize("name,scale,steps", [("M1", 1.0, 200), ("H125", 0.3, 1200)])
def test_friction_parity_with_oracle(name, scale, steps):
    """Tangential spring-dashpot with Coulomb limit and per-contact history: GPU vs
    oracle, element by element (a collisional flow; a hopper under gravity)."""
    s = synth.config_systems(name, seed=1, scale=scale)[0]
    fr = _frictional(s)
    say(f"friction on {name}: N={s.n}, {steps} steps, {fr}")
    xg, vg, hg = gpu_trajectory([s], steps, **fr)
    xo, vo, ho, _ = oracle_run(s, steps, **fr)
    assert_close(s, xg, vg, xo, vo, name + " with friction")
    assert np.array_equal(hg[0]["contacts"], ho["contacts"])
    assert ho["contacts"].max() > 20
    # friction changes the trajectory
    xf, _, _ = gpu_trajectory([s], steps)
    assert not np.array_equal(xf, xg)


def test_friction_k_invariance_sorts_and_history_regrow_bitwise():
    """The springs belong to the contacts, not to the Verlet list: K = 200, K = 20
    and the broad phase at every step give the same bits; so do periodic storage
    re-sorts (the history moves with its particle) and a history table that
    starts with room for one contact and is grown by vb_run."""
    s = synth.config_systems("M1", seed=6)[0]
    fr = _frictional(s, mu=0.3)
    ref = gpu_trajectory([s], 180, skin_mode=2, **fr)
    for name, ov in (("K=200", {}), ("K=20", {"K": 20.0}), ("re-sort every 25", {"reorder_interval": 25}),
                     ("capacity 1", {"contact_capacity": 1})):
        say(f"friction, {name}")
        x, v, h = gpu_trajectory([s], 180, **dict(fr, **ov))
        assert np.array_equal(x, ref[0]) and np.array_equal(v, ref[1]), name
        assert np.array_equal(h[0]["contacts"], ref[2][0]["contacts"]), name


def test_friction_parameters_are_checked():
    import paper_2208_13770_amd as vb
    s = synth.config_systems("M1", scale=0.25)[0]
    for bad in ({"mu": -0.1}, {"kt": float("nan"), "mu": 0.3}, {"contact_capacity": 65}):
        with pytest.raises(vb.VbError):
            vb.vb_create(dict(s.params, **bad), s.n)


# ---------------------------------------------------------------- degenerate cases
def test_particles_at_rest_on_gpu():
    """v = 0 (Eq. skin_formulus1 gives skin 0): one broad phase at step 0, none
    after, nothing moves, and the list is exactly the pairs within
    R_C,i + R_C,j + eps (brute force); exactly touching spheres (delta = 0, the
    spacing of this lattice without jitter) feel no force."""
    s = synth.lattice_system(16, 12, 8, 0, 0, 0.0, seed=9)
    h = 2.0 ** -5                                     # dyadic spacing: distances are exact
    idx = np.round(s.pos_r[:, :3] / s.meta["a"]) - 1.0
    s.pos_r[:, :3] = (idx + 1.0) * h
    s.pos_r[:, 3] = 0.5 * h                           # neighbours exactly touching
    x, v, rc, invm = host_arrays([s])
    with GpuSession([s]) as g:
        hist = g.run(60)
        xo, vo, _ = g.state()
        lst, _ = g.pairs(0, 0)
        con, _ = g.pairs(0, 1)
    say(f"at rest: {hist[0]['rebuilt'].sum()} broad phases, list {len(lst)}, contacts {len(con)}")
    assert hist[0]["rebuilt"].tolist() == [1] + [0] * 59
    assert np.array_equal(xo, x.astype(np.float32).astype(np.float64)) and not vo.any()
    assert len(con) == 0 and hist[0]["contacts"].max() == 0
    ref = oracle.broadphase_brute(xo, rc, s.params["eps"])
    assert np.array_equal(lst, ref)


def _face_system():
    """Particles placed exactly on cell faces, edges, corners and centres
    (dyadic coordinates on a grid of 16 cells per axis)."""
    rng = np.random.default_rng(11)
    edge = 2.0 ** -4                      # 16 cells per axis: L_C (1 + 2^-10) + 2 eps <= 1/16
    L_C = (edge - 4.5e-6) / (1 + 2.0 ** -10)
    n = 3000
    x = rng.integers(2, 30, size=(n, 3)) * (edge / 2)   # cell faces, edges, corners, centres
    x = np.unique(x, axis=0)[:1500]
    n = len(x)
    R = np.full(n, 2.0 ** -6)             # grid neighbours exactly touch
    v = rng.normal(0, 1e-3, size=(n, 3))
    p = {"skin_mode": 0, "cap_mode": 0, "K": 50.0, "dt": 2.0 ** -10, "cell_size": L_C,
         "skin_uniform": 0.0, "eps": 2e-6, "lo": (0, 0, 0), "hi": (1, 1, 1), "kn": 1e3,
         "gamma_n": 0.0, "g": (0, 0, 0), "max_neighbors": 64}

    class Sys:  # the minimal system object GpuSession needs
        pass
    s = Sys()
    s.pos_r = np.concatenate([x, R[:, None]], axis=1).astype(np.float32)
    s.vel_m = np.concatenate([v, np.ones((n, 1))], axis=1).astype(np.float32)
    s.params = p
    s.n = n
    s.meta = {"v_max": 1e-3}
    return s


def test_cell_face_placements_broad_phase():
    """Particles placed exactly on cell faces and corners (dyadic coordinates on
    the cell grid): the GPU list contains every pair the oracle's brute-force
    broad phase finds with a margin, and nothing beyond the eps band."""
    s = _face_system()
    p = s.params
    xh, vh, rc, invm = host_arrays([s])
    with GpuSession([s]) as g:
        g.pairs(0, 1)
        gl, _ = g.pairs(0, 0)
    rnl, _ = oracle.rebuild_radii(p, vh, rc)
    eps = p["eps"]
    ol = oracle.broadphase_brute(xh, rnl + 1e-6, eps)

    def margin(q):
        d = np.linalg.norm(xh[q[:, 0]] - xh[q[:, 1]], axis=1)
        return rnl[q[:, 0]] + rnl[q[:, 1]] + eps - d
    gset = set(map(tuple, gl.tolist()))
    sure = ol[margin(ol) > 1e-6]
    assert len(sure) > 100
    assert not [t for t in map(tuple, sure.tolist()) if t not in gset]
    assert (margin(gl) > -1e-6).all()


def _windows_case(case):
    """(systems, overrides, steps) of the pair-window comparison below."""
    if case in ("M1", "M1_256", "M1_512"):
        return synth.config_systems("M1", seed=3), {}, 200
    if case in ("literal_cap_256", "literal_cap_512"):
        return [synth.lattice_system(10, 9, 7, 3, 2, 0.2, 21)], {"cap_mode": 1}, 150
    if case == "literal_cap":
        return [synth.lattice_system(10, 9, 7, 3, 2, 0.2, 21)], {"cap_mode": 1}, 150
    if case in ("H125", "SILO"):
        return synth.config_systems(case, scale=0.3), {}, 300
    if case == "faces":
        return [_face_system()], {}, 100
    if case == "big_cells":
        # a twentieth of the particles moved next to others, so that some cells
        # hold 9 to 11 (staged in two passes), and 70 into one cell (staged
        # without windows: its brick tests whole rows); rows of ~80 entries
        s = synth.lattice_system(20, 20, 16, 4, 2, 0.1, seed=9)
        rng = np.random.default_rng(6)
        idx = rng.choice(s.n, size=s.n // 20 + 70, replace=False)
        to = rng.choice(s.n, size=len(idx) - 70, replace=False)
        L = s.params["cell_size"]
        a = L / 1.7
        s.pos_r[idx[70:], :3] = (s.pos_r[to, :3] + rng.uniform(-0.3, 0.3, size=(len(to), 3)) * a
                                 ).astype(np.float32)
        s.pos_r[idx[:70], :3] = ((np.array([5, 6, 4]) + rng.uniform(0.05, 0.95, size=(70, 3))) * L
                                 ).astype(np.float32)
        return [s], {}, 1  # one step: vb_run grows the bins and rows first
    if case == "outside":
        # a tenth of the particles moved out of the box across each face, so that
        # they are binned into border cells they do not lie in (no steps run)
        s = synth.lattice_system(20, 18, 16, 4, 2, 0.2, 8)
        rng = np.random.default_rng(4)
        lo, hi = np.asarray(s.params["lo"], float), np.asarray(s.params["hi"], float)
        idx = rng.choice(s.n, size=s.n // 10, replace=False)
        ax = rng.integers(0, 3, size=len(idx))
        side = rng.integers(0, 2, size=len(idx))
        d = rng.uniform(0.0, 2.0 * s.params["cell_size"], size=len(idx))
        s.pos_r[idx, ax] = np.where(side == 0, lo[ax] - d, hi[ax] + d).astype(np.float32)
        return [s], {}, 0
    raise ValueError(case)


@pytest.mark.parametrize("case", ["M1", "literal_cap", "H125", "SILO", "faces", "big_cells",
                                  "outside", "M1_256", "M1_512", "literal_cap_256",
                                  "literal_cap_512"])
def test_pair_windows_leave_the_lists_unchanged(case):
    """The pair search tests, in each row of cells, only the x sub-bins within
    reach of the particle.  Against the search over whole rows (windows off
    through the environment) the Verlet list is the same pair for pair at the
    first broad phase and at the end, and the run is bit-identical with the same
    records: lattice, two-ring (literal cap), hopper and silo systems, particles
    on cell faces (on sub-bin bounds too), cells of 9 to 11 particles and one
    of 70, and particles outside the box, binned into border cells they do not
    lie in; the lattice and two-ring cases also with 256 and 512 threads per
    pair-search workgroup."""
    import os
    systems, ov, steps = _windows_case(case)
    out = {}
    for win in ("0", "1"):
        os.environ["VBUF_PAIR_WINDOWS"] = win
        try:
            with GpuSession(systems, ov) as g:
                if case.endswith(("_256", "_512")):  # other pair-search workgroup sizes
                    vb.vb_set_launch(g.ctx, 8, 2, int(case[-3:]))
                if case == "big_cells":  # the bins and rows overflow at first
                    hist = g.run(steps)
                    first, _ = g.pairs(0, 0)
                else:
                    g.pairs(0, 1)
                    first, _ = g.pairs(0, 0)
                    hist = g.run(steps) if steps else None
                last, _ = g.pairs(0, 0)
                x, v, _ = g.state()
        finally:
            del os.environ["VBUF_PAIR_WINDOWS"]
        out[win] = (first, last, x, v, hist)
        say(f"  {case}, windows {win}: {len(first)} pairs at the first broad phase, "
            f"{len(last)} at step {steps}")
    (f0, l0, x0, v0, h0), (f1, l1, x1, v1, h1) = out["0"], out["1"]
    assert len(f0) > 0
    assert np.array_equal(f0, f1) and np.array_equal(l0, l1)
    assert np.array_equal(x0, x1) and np.array_equal(v0, v1)
    if steps:
        assert_same_records(h0[0], h1[0], case)


@pytest.mark.parametrize("radii", ["polydisperse", "monodisperse", "tiny"])
def test_contact_pretest_at_near_touching_distances(radii):
    """Pairs placed a hair inside or outside touching distance (relative gaps
    from 1e-9 to 1e-4), some of them with centres off the grid of the coded
    positions that the step kernel's pre-test reads (beyond two cells outside
    the box, and one pair across that grid's edge): the contacts the step
    kernel finds equal a brute-force count at every step and the oracle's.
    With "tiny" radii (about 1e-5 box units) a pair's reach is only some six
    steps of that grid, so the pre-test's rounding margin dominates."""
    rng = np.random.default_rng({"polydisperse": 21, "monodisperse": 22, "tiny": 23}[radii])
    L_C = 0.02
    sites = np.stack(np.meshgrid(*[np.arange(0.05, 0.96, 0.05)] * 3, indexing="ij"), -1).reshape(-1, 3)
    sites = sites[rng.permutation(len(sites))[:2400]]
    off = np.array([[-0.1, 0.5, 0.5], [0.5, -0.12, 0.3], [0.4, 0.6, 1.1], [1.15, 1.15, 1.15],
                    [-0.04, 0.3, 0.3]])        # the last straddles the grid edge at lo - 2 cells
    centres = np.concatenate([sites, off], axis=0)
    m = len(centres)
    if radii == "polydisperse":
        R = rng.uniform(0.004, 0.008, size=(m, 2))
    elif radii == "tiny":
        R = rng.uniform(4e-6, 8e-6, size=(m, 2))
    else:
        R = np.full((m, 2), 0.006)
    u = rng.normal(size=(m, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    u[-1] = (1.0, 0.0, 0.0)
    rel = rng.choice([1e-9, 1e-7, 1e-5, 1e-4], size=m) * rng.choice([-1.0, 1.0], size=m)
    d = (R[:, 0] + R[:, 1]) * (1.0 + rel)
    x = np.concatenate([centres - 0.5 * d[:, None] * u, centres + 0.5 * d[:, None] * u])
    rc = np.concatenate([R[:, 0], R[:, 1]])
    n = len(rc)
    v = rng.normal(0, 1e-3, size=(n, 3))
    p = {"skin_mode": 0, "cap_mode": 0, "K": 50.0, "dt": 2.0 ** -12, "cell_size": L_C,
         "skin_uniform": 0.0, "eps": 2e-6, "lo": (0, 0, 0), "hi": (1, 1, 1), "kn": 1e3,
         "gamma_n": 0.0, "g": (0, 0, 0), "max_neighbors": 32}

    class Sys:  # the minimal system object GpuSession needs
        pass
    s = Sys()
    s.pos_r = np.concatenate([x, rc[:, None]], axis=1).astype(np.float32)
    s.vel_m = np.concatenate([v, np.ones((n, 1))], axis=1).astype(np.float32)
    s.params = p
    s.n = n
    s.meta = {"v_max": 1e-3}
    xh, vh, rch, invm = host_arrays([s])
    brute0 = len(oracle.contacts_brute(xh, rch))
    say(f"pre-test at near-touching distances ({radii}): {n} particles, {brute0} contacts at step 0")
    assert 0.3 * m < brute0 < 0.7 * m
    steps = 6
    with GpuSession([s]) as g:
        h = g.run(steps)[0]
        xg, vg, _ = g.state()
    xo, vo, ho, _ = oracle_run(s, steps)
    assert h["contacts"][0] == brute0
    assert np.array_equal(h["contacts"], ho["contacts"])
    assert_close(s, xg, vg, xo, vo, "near-touching pairs")
    x1, _, _, _ = oracle_run(s, steps - 1)
    assert h["contacts"][-1] == len(oracle.contacts_brute(x1, rch))


def test_k_zero_parity():
    """K = 0: every particle that moves violates at once, the broad phase runs at
    (nearly) every step, and the results still match the oracle."""
    s = synth.config_systems("M1", seed=8, scale=0.6)[0]
    xg, vg, hg = gpu_trajectory([s], 120, K=0.0)
    xo, vo, ho, _ = oracle_run(s, 120, K=0.0)
    assert_close(s, xg, vg, xo, vo, "K=0")
    assert hg[0]["rebuilt"].mean() > 0.9


def test_pair_search_beyond_lds_capacity():
    """Cells four lattice spacings wide hold ~64 particles each, so a brick's
    neighbourhood (6^3 cells) holds ~14,000: far more than the pair search stages
    in LDS, which then reads the bins directly.  Results and contacts still match
    the oracle, and the bins (16 at first) are grown on the way."""
    s = synth.lattice_system(24, 24, 24, 6, 3, 0.1, seed=12, K=5.0, cell_factor=4.0)
    say(f"large cells: N={s.n}, cell {s.params['cell_size']:.4f}")
    xg, vg, hg = gpu_trajectory([s], 120)
    xo, vo, ho, _ = oracle_run(s, 120)
    assert_close(s, xg, vg, xo, vo, "large cells")
    assert np.array_equal(hg[0]["contacts"], ho["contacts"])
    assert ho["contacts"].max() > 50


def test_long_rows_sorted_like_short_ones():
    """Rows of 33 to 43 entries (cells of about 2.1 lattice spacings, K = 5000, so
    every moving particle's sphere reaches the cap): the pair search sorts such
    rows with its longest register network and in LDS.  The rows must really be
    that long, and K = 5000 must still equal the broad phase at every step bit
    for bit (Sec. 4.2), which holds only if every row is in canonical order."""
    s = synth.lattice_system(18, 18, 18, 3, 2, 0.2, 5, cell_factor=2.2, K=5000.0,
                             max_neighbors=64)
    say(f"long rows: N={s.n}, 120 steps, K=5000 vs no buffer")
    with GpuSession([s]) as g:
        g.run(1)
        pairs, _ = g.pairs(0, 0)
    deg = np.bincount(pairs.ravel(), minlength=s.n)
    say(f"  longest row {int(deg.max())}, rows over 32: {int((deg > 32).sum())}")
    assert deg.max() > 32 and (deg > 32).sum() > 1000
    xa, va, ha = gpu_trajectory([s], 120)
    xb, vb_, hb = gpu_trajectory([s], 120, skin_mode=2)
    assert np.array_equal(xa, xb) and np.array_equal(va, vb_)
    assert np.array_equal(ha[0]["contacts"], hb[0]["contacts"])
    assert ha[0]["rebuilt"].sum() < hb[0]["rebuilt"].sum()
    xo, vo, ho, _ = oracle_run(s, 120)
    assert_close(s, xa, va, xo, vo, "long rows")
    assert np.array_equal(ha[0]["contacts"], ho["contacts"])


@pytest.mark.parametrize("name,scale,friction", [("M1", 1.0, False), ("H125", 0.3, True)])
def test_graph_replay_equals_eager_launches(name, scale, friction):
    """Blocks of 64 steps replayed as one captured HIP graph against the same
    steps launched one by one (VBUF_GRAPHS=0 at create): five calls of 70 steps,
    each mixing eager steps with a replayed block, with the host reading the
    state between calls.  State and step records agree bit for bit after every
    call."""
    import os
    s = synth.config_systems(name, seed=2, scale=scale)[0]
    ov = _frictional(s) if friction else {}
    say(f"graph replay vs eager launches: {name} N={s.n}, friction {friction}")
    os.environ["VBUF_GRAPHS"] = "0"
    try:
        eager = GpuSession([s], ov)
    finally:
        del os.environ["VBUF_GRAPHS"]
    graph = GpuSession([s], ov)
    try:
        for call in range(5):
            he, hg = eager.run(70), graph.run(70)
            xe, ve, _ = eager.state()
            xg, vg, _ = graph.state()
            assert np.array_equal(xe, xg) and np.array_equal(ve, vg), call
            assert np.array_equal(he, hg), call
        assert hg[0]["rebuilt"].sum() < 70
    finally:
        eager.close()
        graph.close()


def test_checkpoint_resume_with_friction_history_bitwise():
    """A frictional run checkpointed with its state and its friction history
    (vb_get_history) and resumed in a new context (vb_set_history) continues
    bit-identically; resumed without the history, every spring starts at zero
    and the run departs from the uninterrupted one."""
    import torch
    import paper_2208_13770_amd as vb
    s = synth.config_systems("M1", seed=8)[0]
    fr = _frictional(s)
    say(f"checkpoint/resume with friction: N={s.n}")
    xa, va, _ = gpu_trajectory([s], 200, **fr)
    with GpuSession([s], fr) as g:
        g.run(120)
        x1, v1, half = g.state()
        assert half
        need = vb.vb_get_history(g.ctx)
        assert need > 0
        partner = torch.empty((s.n, need + 1), dtype=torch.int32, device="cuda")
        spring = torch.empty((s.n, need + 1, 3), dtype=torch.float64, device="cuda")
        assert vb.vb_get_history(g.ctx, partner, spring) == need
        small = torch.empty((s.n, need - 1), dtype=torch.int32, device="cuda")
        small3 = torch.empty((s.n, need - 1, 3), dtype=torch.float64, device="cuda")
        with pytest.raises(vb.VbError) as e:
            vb.vb_get_history(g.ctx, small, small3)
        assert e.value.code == vb.VB_ECAPACITY
    p = partner.cpu().numpy()
    assert (p[:, -1] == -1).all() and (p >= -1).all()
    say(f"  {int((p >= 0).sum())} contacts carried, at most {need} per particle")
    xt, vt = torch.from_numpy(x1).cuda(), torch.from_numpy(v1).cuda()
    with GpuSession([s], fr) as g:
        vb.vb_set_state(g.ctx, xt, vt, g.rc, g.invm, v_is_half_step=True)
        g.pairs(0, 1)  # runs the storage sort first: the history follows the particles
        vb.vb_set_history(g.ctx, partner, spring)
        g.run(80)
        xb, vb2, _ = g.state()
        with pytest.raises(vb.VbError) as e:  # only right after vb_set_state
            vb.vb_set_history(g.ctx, partner, spring)
        assert e.value.code == vb.VB_EINVAL
    assert np.array_equal(xa, xb) and np.array_equal(va, vb2)
    with GpuSession([s], fr) as g:
        vb.vb_set_state(g.ctx, xt, vt, g.rc, g.invm, v_is_half_step=True)
        g.run(80)
        xc, _, _ = g.state()
    assert not np.array_equal(xa, xc)


def test_friction_history_equals_the_oracle_springs():
    """The springs the step kernel carries from step to step are the oracle's, bit
    for bit: after 150 frictional steps on M1, every particle's contacts
    (vb_get_history: partners in ascending original index) and the elongation
    vector of each equal the oracle's exported springs."""
    import torch
    import paper_2208_13770_amd as vb
    s = synth.config_systems("M1", seed=1)[0]
    fr = _frictional(s)
    steps = 150
    say(f"friction history against the oracle's springs: N={s.n}, {steps} steps")
    x, v, rc, invm = host_arrays([s])
    xo, vo, ho, (off, j, xi) = oracle.run_springs(dict(s.params, **fr), x, v, rc, invm, steps)
    with GpuSession([s], fr) as g:
        g.run(steps)
        xg, vg, _ = g.state()
        need = vb.vb_get_history(g.ctx)
        partner = torch.empty((s.n, need), dtype=torch.int32, device="cuda")
        spring = torch.empty((s.n, need, 3), dtype=torch.float64, device="cuda")
        assert vb.vb_get_history(g.ctx, partner, spring) == need
    assert_close(s, xg, vg, xo, vo, "M1 with friction")
    cnt = np.diff(off)
    assert need == cnt.max() and len(j) > 20
    po = np.full((s.n, need), -1, dtype=np.int32)
    so = np.zeros((s.n, need, 3))
    row = np.repeat(np.arange(s.n), cnt)
    col = np.arange(len(j)) - np.repeat(off[:-1], cnt)
    po[row, col] = j
    so[row, col] = xi
    pg, sg = partner.cpu().numpy(), spring.cpu().numpy()
    assert np.array_equal(pg, po)
    used = po >= 0
    nd = int((sg[used] != so[used]).sum())
    say(f"  {len(j)} springs, {nd} components differ from the oracle's")
    assert nd == 0


def test_history_input_is_checked():
    import torch
    import paper_2208_13770_amd as vb
    s = synth.config_systems("H125", seed=3, scale=0.3)[0]
    fr = _frictional(s)
    say("history input checks")
    partner = torch.full((s.n, 3), -1, dtype=torch.int32, device="cuda")
    spring = torch.zeros((s.n, 3, 3), dtype=torch.float64, device="cuda")
    with GpuSession([s]) as g:  # no friction
        with pytest.raises(vb.VbError):
            vb.vb_set_history(g.ctx, partner, spring)
    with GpuSession([s], fr) as g:
        vb.vb_set_history(g.ctx, partner, spring)  # an empty history is fine
        for bad in ([5, 5], [7, 3], [0, s.n], [1, -1, 2]):
            q = partner.clone()
            q[0, :len(bad)] = torch.tensor(bad, dtype=torch.int32)
            if bad == [1, -1, 2]:
                vb.vb_set_history(g.ctx, q, spring)  # entries after -1 are ignored
                continue
            with pytest.raises(vb.VbError) as e:
                vb.vb_set_history(g.ctx, q, spring)
            assert e.value.code == vb.VB_EINVAL, bad
        q = partner.clone()
        q[1, 0] = 0
        sp = spring.clone()
        sp[1, 0, 2] = float("nan")
        with pytest.raises(vb.VbError) as e:
            vb.vb_set_history(g.ctx, q, sp)
        assert e.value.code == vb.VB_ENONFINITE
        q = partner.clone()
        q[0, 0] = 0  # the particle itself
        with pytest.raises(vb.VbError) as e:
            vb.vb_set_history(g.ctx, q, spring)
        assert e.value.code == vb.VB_EINVAL


@pytest.mark.parametrize("seed", range(6))
def test_random_mixes_against_oracle(seed):
    """Seeded random mixes of the options in one uneven batch: lattice, hopper and
    incline systems, mono- or polydisperse, K in {0, 10, 200, 5000} (at most 10
    with the literal cap, whose spheres reach L_C), both cap modes, local or
    uniform skin, friction on or off, narrow rows and bins that must grow.  Every system against the oracle (the 1e-5 bars, contact counts
    exact at every step), and the batch against the broad phase at every step,
    bit for bit (Sec. 4.2)."""
    _random_mix(1000 + seed, 3)


@pytest.mark.parametrize("seed", [2, 11, 15])  # draws that mix silos with other kinds
def test_random_mixes_with_silos_against_oracle(seed):
    """The same with cylindrical silos among the kinds, so that cylinders meet
    friction, the uniform skin, growing rows and bins, and systems without
    walls in one batch (the walls' instance of the step kernel serves them
    all)."""
    _random_mix(2000 + seed, 4)


def _random_mix(rng_seed, n_kinds):
    import torch
    import paper_2208_13770_amd as vb
    rng = np.random.default_rng(rng_seed)
    systems, params = [], []
    for _ in range(int(rng.integers(1, 4))):
        kind, sd = int(rng.integers(0, n_kinds)), int(rng.integers(0, 1 << 30))
        K = float(rng.choice([0.0, 10.0, 200.0, 5000.0]))
        if kind == 0:
            dims = [int(rng.integers(4, 15)) for _ in range(3)]
            cap = int(rng.integers(0, 2))
            if cap == 1:  # spheres up to L_C: rows past the 128-entry limit at large K
                K = min(K, 10.0)
            s = synth.lattice_system(*dims, int(rng.integers(0, 4)), int(rng.integers(0, 3)),
                                     float(rng.uniform(0.02, 0.3)), sd,
                                     polydisperse=bool(rng.integers(0, 2)), K=K, cap_mode=cap)
        elif kind == 1:
            s = synth.hopper_system(int(rng.integers(400, 2500)), sd, K=K)
        elif kind == 2:
            s = synth.incline_system(int(rng.integers(400, 2500)), sd, K=K)
        else:
            s = synth.silo_system(int(rng.integers(400, 2500)), sd, K=K)
        p = dict(s.params, max_neighbors=int(rng.choice([4, 16, 32])),
                 bin_capacity=int(rng.choice([2, 8, 16])))
        if rng.random() < 0.3:
            p["skin_mode"] = vb.VB_SKIN_UNIFORM
            p["skin_uniform"] = float(0.1 * s.meta["a"])
        if rng.random() < 0.4:
            p.update(_frictional(s))
        systems.append(s)
        params.append(p)
    steps = 600
    say(f"random mix {rng_seed}: " + ", ".join(
        f"{s.meta.get('kind', 'lattice')} N={s.n} K={p['K']:g} cap={p.get('cap_mode', 0)} "
        f"skin={p.get('skin_mode', 0)} mu={p.get('mu', 0.0):g}" for s, p in zip(systems, params)))
    x, v, rc, invm = vb.state_tensors(systems)

    def run(plist):
        ctx = vb.vb_batch_create(plist, [s.n for s in systems])
        try:
            vb.vb_set_state(ctx, x, v, rc, invm)
            h = vb.vb_run(ctx, steps)
            xo, vo = torch.empty_like(x), torch.empty_like(v)
            vb.vb_get_state(ctx, xo, vo)
        finally:
            vb.vb_destroy(ctx)
        return xo.cpu().numpy(), vo.cpu().numpy(), h

    xg, vg, hg = run(params)
    off = np.cumsum([0] + [s.n for s in systems])
    for b, (s, p) in enumerate(zip(systems, params)):
        sl = slice(int(off[b]), int(off[b + 1]))
        X, Vv, R, M = host_arrays([s])
        xo, vo, ho, _ = oracle.run(p, X, Vv, R, M, steps)
        assert_close(s, xg[sl], vg[sl], xo, vo, f"system {b}")
        assert np.array_equal(hg[b]["contacts"], ho["contacts"]), b
    xn, vn, hn = run([dict(p, skin_mode=vb.VB_NO_BUFFER) for p in params])
    assert np.array_equal(xg, xn) and np.array_equal(vg, vn)
    assert np.array_equal(hg["contacts"], hn["contacts"])


def test_forced_rebuild_timing_and_info():
    """vb_force_rebuild runs a broad phase at the next step and changes no result
    (Sec. 4.2); vb_set_timing / vb_phase_times count exactly the timed steps and
    the steps with a broad phase; vb_get_info reports sizes and the step counter;
    vb_last_error gives the message of a failed call."""
    import paper_2208_13770_amd as vb
    s = synth.config_systems("M1", seed=11)[0]
    say("forced rebuild, timing, info")
    xr, vr, hr = gpu_trajectory([s], 61)
    with GpuSession([s]) as g:
        h1 = g.run(30)
        vb.vb_force_rebuild(g.ctx)
        h2 = g.run(1)
        assert h2[0]["rebuilt"][0] == 1
        vb.vb_set_timing(g.ctx, 1)
        h3 = g.run(30)
        pt = vb.vb_phase_times(g.ctx)
        assert pt["steps"] == 30 and pt["ms_step"] > 0.0 and pt["ms_rebuild"] > 0.0
        assert pt["rebuild_steps"] == int(h3[0]["rebuilt"].sum())
        info = g.info()
        assert info["n_total"] == s.n and info["n_sys"] == 1 and info["step"] == 61
        assert info["row_width"] >= s.params.get("max_neighbors", 32)
        x, v, _ = g.state()
        with pytest.raises(vb.VbError):
            vb.vb_set_K(g.ctx, 5, 100.0)  # no system 5
        assert "sys" in vb.vb_last_error(g.ctx)
    assert np.array_equal(x, xr) and np.array_equal(v, vr)
    contacts = np.concatenate([h1[0]["contacts"], h2[0]["contacts"], h3[0]["contacts"]])
    assert np.array_equal(contacts, hr[0]["contacts"])


def test_fixed_interval_schedule_on_gpu():
    """The fixed-update practice the automatic scheme replaces (Sec. 1, Sec. 2):
    with VB_FIXED_INTERVAL the broad phase runs exactly every F steps whatever
    the particles do, and with a skin too small for the flow it misses contacts.
    At the first step where the contact count departs from the exact run it is
    lower: a stale list can miss a contact, never make one."""
    import paper_2208_13770_amd as vb
    s = synth.config_systems("M1", seed=12)[0]
    F = 25
    say(f"fixed interval {F} on M1")
    ov = {"skin_mode": vb.VB_FIXED_INTERVAL, "fixed_interval": F,
          "skin_uniform": float(1e-3 * s.meta["a"])}
    _, _, hf = gpu_trajectory([s], 150, **ov)
    _, _, he = gpu_trajectory([s], 150, skin_mode=vb.VB_NO_BUFFER)
    steps = np.arange(150)
    assert np.array_equal(hf[0]["rebuilt"].astype(bool), steps % F == 0)
    cf, ce = hf[0]["contacts"], he[0]["contacts"]
    diff = np.nonzero(cf != ce)[0]
    say(f"  first departure at step {diff[0] if len(diff) else None}")
    assert len(diff) > 0
    assert cf[diff[0]] < ce[diff[0]]
    assert diff[0] % F != 0


def test_context_without_particles():
    """A context of one empty system loads, runs and reports without launching
    work: records of zeros, an empty pair list."""
    import torch
    import paper_2208_13770_amd as vb
    s = synth.lattice_system(2, 2, 2, 0, 0, 0.0, 5)
    say("empty context")
    ctx = vb.vb_create(s.params, 0)
    try:
        e3 = torch.empty((0, 3), dtype=torch.float64, device="cuda")
        e1 = torch.empty((0,), dtype=torch.float32, device="cuda")
        vb.vb_set_state(ctx, e3, e3, e1, e1)
        h = vb.vb_run(ctx, 10)
        assert h.shape == (1, 10)
        assert (h["contacts"] == 0).all() and (h["list_pairs"] == 0).all()
        assert vb.vb_get_pairs(ctx, 0, 0) == 0 and vb.vb_get_pairs(ctx, 0, 1) == 0
        vb.vb_get_state(ctx, e3, e3)
        assert vb.vb_get_info(ctx)["n_total"] == 0
    finally:
        vb.vb_destroy(ctx)


@pytest.mark.parametrize("env", [{"VBUF_STEP_UNROLL": "1"}, {"VBUF_STEP_UNROLL": "2"},
                                 {"VBUF_STEP_UNROLL": "4"}, {"VBUF_XCD_REMAP": "1"}])
def test_tuning_variants_against_oracle(env):
    """The step kernel's other instantiations (1, 2 or 4 gathers in flight per
    thread) and the XCD tile order, chosen at create through the environment:
    each matches the oracle and is K-invariant bit for bit (with and without
    friction)."""
    import os
    s = synth.config_systems("M1", seed=13)[0]
    fr = _frictional(s)
    say(f"tuning variant {env}")
    os.environ.update(env)
    try:
        xg, vg, hg = gpu_trajectory([s], 120)
        xn, vn, _ = gpu_trajectory([s], 120, skin_mode=2)
        xf, vf, hf = gpu_trajectory([s], 120, **fr)
        xfn, vfn, _ = gpu_trajectory([s], 120, skin_mode=2, **fr)
    finally:
        for k in env:
            del os.environ[k]
    xo, vo, ho, _ = oracle_run(s, 120)
    assert_close(s, xg, vg, xo, vo, "variant")
    assert np.array_equal(hg[0]["contacts"], ho["contacts"])
    assert np.array_equal(xg, xn) and np.array_equal(vg, vn)
    xo, vo, ho, _ = oracle_run(s, 120, **fr)
    assert_close(s, xf, vf, xo, vo, "variant with friction")
    assert np.array_equal(hf[0]["contacts"], ho["contacts"])
    assert np.array_equal(xf, xfn) and np.array_equal(vf, vfn)


def test_launch_shapes_give_identical_bits():
    """Every launch shape (vb_set_launch: 1, 2, 4 or 8 partner gathers in flight,
    tile order 0, 1 or 2, 256, 384 or 512 pair-search threads) gives the
    same positions, velocities and records, bit for bit: with the local buffer,
    with friction, and with a broad phase at every step (every pair-search shape
    at work every step)."""
    import paper_2208_13770_amd as vb
    s = synth.config_systems("M1", seed=13)[0]
    for name, ov in (("K=200", {}), ("friction", _frictional(s)), ("no buffer", {"skin_mode": 2})):
        ref = None
        for unroll in (8, 4, 2, 1):
            for xcd in (0, 1, 2):
                for pt in (256, 384, 512):
                    with GpuSession([s], ov) as g:
                        vb.vb_set_launch(g.ctx, unroll, xcd, pt)
                        assert vb.vb_get_launch(g.ctx) == {"unroll": unroll, "xcd_order": xcd,
                                                           "pairs_threads": pt}
                        h = g.run(120)
                        x, v, _ = g.state()
                    if ref is None:
                        ref = (x, v, h)
                        continue
                    what = f"{name} unroll={unroll} xcd={xcd} threads={pt}"
                    assert np.array_equal(x, ref[0]) and np.array_equal(v, ref[1]), what
                    assert np.array_equal(h, ref[2]), what
        say(f"  {name}: 36 launch shapes, identical")
    with GpuSession([s]) as g:
        for bad in ((3, 0, 384), (8, 3, 384), (8, -1, 384), (8, 0, 300)):
            with pytest.raises(vb.VbError) as e:
                vb.vb_set_launch(g.ctx, *bad)
            assert e.value.code == vb.VB_EINVAL


def test_tile_orders_on_a_system_of_several_tile_groups():
    """The tile orders permute whole groups of 8 runs of 32 tiles (order 2) or
    split the tiles in eight (order 1); on a system of 320 tiles (one whole group
    of 256 and a shorter last group) every order gives the same bits."""
    import paper_2208_13770_amd as vb
    s = synth.lattice_system(64, 64, 20, 16, 8, 0.1, 21)
    assert s.n == 81920
    ref = None
    for xcd in (0, 1, 2):
        with GpuSession([s]) as g:
            vb.vb_set_launch(g.ctx, 8, xcd, 384)
            h = g.run(100)
            x, v, _ = g.state()
        if ref is None:
            ref = (x, v, h)
            continue
        assert np.array_equal(x, ref[0]) and np.array_equal(v, ref[1]), xcd
        assert np.array_equal(h, ref[2]), xcd
    assert ref[2]["contacts"][0].sum() > 0


def test_default_launch_shape_follows_batch_size():
    """A new context of a kind no tuner has seen starts from 4 gathers in flight,
    8 for a batch with friction of 2^20 particles and more, tile order 2 and 384
    pair-search threads."""
    import paper_2208_13770_amd as vb
    small = synth.lattice_system(24, 24, 16, 2, 1, 0.1, 22)
    large = synth.lattice_system(128, 128, 64, 8, 4, 0.1, 23)
    assert small.n < 2 ** 20 <= large.n
    for s, ov, unroll in ((small, {}, 4), (small, _frictional(small), 4), (large, {}, 4),
                          (large, _frictional(large), 8)):
        ctx = vb.vb_batch_create([dict(s.params, **ov)], [s.n])
        try:
            assert vb.vb_get_launch(ctx) == {"unroll": unroll, "xcd_order": 2, "pairs_threads": 384}
        finally:
            vb.vb_destroy(ctx)


def test_tuner_runs_the_same_steps_and_remembers_its_choice():
    """vb_tune advances the state exactly as vb_run does (its forced broad phases
    change no result) while it times every launch shape, and a later context of
    the same kind starts from the shape it chose."""
    import paper_2208_13770_amd as vb
    s = synth.config_systems("M1", seed=14)[0]
    xa, va, ha = gpu_trajectory([s], 240)
    with GpuSession([s]) as g:
        with pytest.raises(vb.VbError) as e:
            vb.vb_tune(g.ctx, 10)
        assert e.value.code == vb.VB_EINVAL
        h = vb.vb_tune(g.ctx, 240)
        x, v, _ = g.state()
        chosen = vb.vb_get_launch(g.ctx)
    say(f"  tuned shape {chosen}; broad phases {int(h[0]['rebuilt'].sum())} "
        f"(plain run {int(ha[0]['rebuilt'].sum())})")
    assert np.array_equal(x, xa) and np.array_equal(v, va)
    assert np.array_equal(h[0]["contacts"], ha[0]["contacts"])
    assert h[0]["step"].tolist() == list(range(240))
    assert h[0]["rebuilt"].sum() >= ha[0]["rebuilt"].sum()
    with GpuSession([s]) as g:
        assert vb.vb_get_launch(g.ctx) == chosen
