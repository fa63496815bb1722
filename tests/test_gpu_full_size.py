"""Parity at the benchmark's full size, in the launch configuration bench.py times.

The workload is M2: 256x256x64 = 4,194,304 particles, K = 200, default launch
parameters, for the 500 steps bench.py times. The oracle runs the whole system
(it is O(N) per step with linked cells, on the host's cores), so every particle
is compared, not just a sample. The tolerance is that
of the small-size tests: positions within 1e-5 box units and velocities within
1e-5 v_max, element by element; positions and velocities are also asserted
equal to the oracle's bit for bit (the GPU evaluates the FP64 contact law and
integration in the oracle's order, every operation rounded). Contact counts are
compared exactly at every step. The theorem of Sec. 4.2 (method == broad phase
every step) is checked bitwise at full size.
"""
import numpy as np
import pytest

import oracle
import paper_2208_13770_amd as vb
import synth
from tests._gpu import GpuSession, gpu_trajectory, host_arrays, say

pytestmark = pytest.mark.gpu

TOL_X = 1e-5
TOL_V = 1e-5
STEPS = 500          # the steps bench.py times on M2
STEPS_FRICTION = 200


@pytest.fixture(scope="module")
def m2():
    return synth.config_systems("M2", seed=0)[0]


def test_m2_full_size_parity_with_oracle(m2):
    s = m2
    say(f"M2 full size: N={s.n}, {STEPS} steps, GPU then oracle")
    with GpuSession([s]) as g:
        hg = g.run(STEPS)
        xg, vg, _ = g.state()
        n_list = vb.vb_get_pairs(g.ctx, 0, 0)
    # the record's list_pairs (bench.py's byte count uses it) is the list in use
    say(f"  list pairs: record {int(hg[0]['list_pairs'][-1])}, exported list {n_list}")
    assert hg[0]["list_pairs"][-1] == n_list
    x, v, rc, invm = host_arrays([s])
    xo, vo, ho, _ = oracle.run(s.params, x, v, rc, invm, STEPS)
    ex = np.abs(xg - xo).max()
    ev = np.abs(vg - vo).max() / s.meta["v_max"]
    say(f"  max|dx| = {ex:.3e} box units, max|dv| = {ev:.3e} v_max; "
        f"contacts at the last step {int(ho['contacts'][-1])}, "
        f"broad phases GPU {int(hg[0]['rebuilt'].sum())} oracle {int(ho['rebuilt'].sum())}")
    assert ex <= TOL_X and ev <= TOL_V
    assert np.array_equal(xg, xo) and np.array_equal(vg, vo)
    assert np.array_equal(hg[0]["contacts"], ho["contacts"])
    assert ho["contacts"][-1] > 10000
    assert np.allclose(hg[0]["kinetic_energy"], ho["kinetic_energy"], rtol=1e-9, atol=0)


def test_m2_full_size_friction_parity_with_oracle(m2):
    """M2 with the tangential friction bench.py --friction 0.4 times (kt = kn/2,
    gamma_t = gamma_n/2, mu = 0.4), 200 steps, every particle against the
    oracle, bit for bit, with its contact count at every step."""
    s = m2
    fr = {"kt": 0.5 * s.params["kn"], "gamma_t": 0.5 * s.params["gamma_n"], "mu": 0.4}
    say(f"M2 with friction: N={s.n}, {STEPS_FRICTION} steps, GPU then oracle")
    xg, vg, hg = gpu_trajectory([s], STEPS_FRICTION, **fr)
    x, v, rc, invm = host_arrays([s])
    xo, vo, ho, _ = oracle.run(dict(s.params, **fr), x, v, rc, invm, STEPS_FRICTION)
    ex = np.abs(xg - xo).max()
    ev = np.abs(vg - vo).max() / s.meta["v_max"]
    say(f"  max|dx| = {ex:.3e}, max|dv| = {ev:.3e} v_max, contacts at the last step "
        f"{int(ho['contacts'][-1])}")
    assert ex <= TOL_X and ev <= TOL_V
    assert np.array_equal(xg, xo) and np.array_equal(vg, vo)
    assert np.array_equal(hg[0]["contacts"], ho["contacts"])
    assert ho["contacts"][-1] > 10000


def test_m2_full_size_k_invariance_bitwise(m2):
    """K = 200 against the broad phase at every step: identical bits (Sec. 4.2)."""
    s = m2
    steps = 60
    say(f"M2 full size: K=200 vs no buffer, {steps} steps")
    xa, va, ha = gpu_trajectory([s], steps)
    xb, vb_, hb = gpu_trajectory([s], steps, skin_mode=2)
    say(f"  broad phases: K=200 {int(ha[0]['rebuilt'].sum())}, no buffer {int(hb[0]['rebuilt'].sum())}")
    assert hb[0]["rebuilt"].all() and ha[0]["rebuilt"].sum() < steps
    assert np.array_equal(xa, xb) and np.array_equal(va, vb_)
    assert np.array_equal(ha[0]["contacts"], hb[0]["contacts"])


def _oracle_system(s, steps):
    x, v, rc, invm = host_arrays([s])
    return oracle.run(s.params, x, v, rc, invm, steps)


def _slices(systems):
    off = np.cumsum([0] + [s.n for s in systems])
    return [slice(int(off[i]), int(off[i + 1])) for i in range(len(systems))]


def test_m3_batch_parity_with_oracle():
    """The 64 uneven systems (19.9M particles) as one batch against the oracle,
    system by system, every particle."""
    systems = synth.config_systems("M3", seed=0, workers=8)
    steps = 30
    say(f"M3: {len(systems)} systems, N={sum(s.n for s in systems)}, {steps} steps")
    xg, vg, hg = gpu_trajectory(systems, steps)
    worst_x = worst_v = 0.0
    for i, (s, sl) in enumerate(zip(systems, _slices(systems))):
        xo, vo, ho, _ = _oracle_system(s, steps)
        worst_x = max(worst_x, np.abs(xg[sl] - xo).max())
        worst_v = max(worst_v, np.abs(vg[sl] - vo).max() / s.meta["v_max"])
        assert np.array_equal(xg[sl], xo) and np.array_equal(vg[sl], vo), i
        assert np.array_equal(hg[i]["contacts"], ho["contacts"]), i
    say(f"  max|dx| = {worst_x:.3e} box units, max|dv| = {worst_v:.3e} v_max over all systems")
    assert worst_x <= TOL_X and worst_v <= TOL_V
    assert hg["contacts"][:, -1].sum() > 0


def test_m5_every_system_bitwise_with_oracle():
    """The largest workload, 16 systems of 512x512x64 (268M particles) in one
    batch, in the launch configuration bench.py times, for 50 steps: every system
    against the oracle, which runs them in parallel processes on the host.  Each
    compares the SHA-256 of the FP64 positions and velocities (bit-for-bit
    equality of all 268M particles) and the contact count of every step."""
    import hashlib
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor

    from synth.systems import _lattice_args
    from tests._gpu import oracle_digest
    args = _lattice_args("M5", 0, 1.0)
    systems = synth.config_systems("M5", seed=0, workers=16)
    steps = 50
    say(f"M5: {len(systems)} systems, N={sum(s.n for s in systems)}, {steps} steps on the GPU")
    xg, vg, hg = gpu_trajectory(systems, steps)
    sl = _slices(systems)
    gpu = [(hashlib.sha256(np.ascontiguousarray(xg[sl[i]]).tobytes()).hexdigest(),
            hashlib.sha256(np.ascontiguousarray(vg[sl[i]]).tobytes()).hexdigest())
           for i in range(len(systems))]
    del xg, vg, systems
    say("  oracle on every system, 16 processes")
    # spawned workers: this process has initialised the GPU, the workers use none
    with ProcessPoolExecutor(max_workers=16, mp_context=multiprocessing.get_context("spawn")) as ex:
        ref = list(ex.map(oracle_digest, args, [steps] * len(args)))
    for i, (hx, hv, con, reb) in enumerate(ref):
        say(f"  system {i}: positions {'equal' if hx == gpu[i][0] else 'DIFFER'}, velocities "
            f"{'equal' if hv == gpu[i][1] else 'DIFFER'}, contacts at the end {int(con[-1])}")
        assert (hx, hv) == gpu[i], i
        assert np.array_equal(hg[i]["contacts"], con), i
    assert hg["rebuilt"][:, 0].all()


@pytest.mark.parametrize("name,steps", [("H125", 200), ("INCLINE", 150), ("SILO", 200)])
def test_paper_size_gravity_workloads_parity(name, steps):
    """The hopper stand-in at the paper's smallest size (125k particles), the
    inclined-plane stand-in (250k) and the cylindrical silo stand-in (126k),
    every particle against the oracle."""
    s = synth.config_systems(name, seed=0)[0]
    say(f"{name}: N={s.n}, {steps} steps")
    xg, vg, hg = gpu_trajectory([s], steps)
    xo, vo, ho, _ = _oracle_system(s, steps)
    ex = np.abs(xg - xo).max()
    ev = np.abs(vg - vo).max() / s.meta["v_max"]
    say(f"  max|dx| = {ex:.3e}, max|dv| = {ev:.3e} v_max, contacts at the end {int(ho['contacts'][-1])}")
    assert ex <= TOL_X and ev <= TOL_V
    assert np.array_equal(xg, xo) and np.array_equal(vg, vo)
    assert np.array_equal(hg[0]["contacts"], ho["contacts"])
