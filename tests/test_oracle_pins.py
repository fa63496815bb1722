"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage or the closed form it pins.  None of them compares
the oracle with itself by retyping its formulas: they use the theorem of Sec. 4.2
(results identical to the broad phase at every step), brute force, closed-form
cadences, exact dyadic kinematics, textbook spring-dashpot solutions,
conservation laws, symmetry, and the numbers printed in Tab. summary.
Labels R1 to R13 name the readings of the paper listed in the header of
oracle/orc.c.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import synth
from paper_2208_13770_amd import report

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def arrays(sys_):
    x = sys_.pos_r[:, :3].astype(np.float64)
    v = sys_.vel_m[:, :3].astype(np.float64)
    rc = sys_.pos_r[:, 3].astype(np.float64)
    invm = sys_.vel_m[:, 3].astype(np.float64)
    return x, v, rc, invm


def colliding(seed=0, poly=False):
    """A small, strongly stirred system with many collisions and wall contacts."""
    return synth.lattice_system(8, 8, 6, 3, 2, 0.3, seed, polydisperse=poly)


# ---------------------------------------------------------------- exactness, list superset
@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("mode,K,cap", [
    (0, 0.0, 0), (0, 10.0, 0), (0, 200.0, 0), (0, 5000.0, 0),
    (0, 200.0, 1), (0, 5000.0, 1), (1, 0.0, 0), (1, 0.0, 1), (2, 0.0, 0),
])
def test_exactness_vs_naive(orc, seed, mode, K, cap):
    """Sec. 1 and Sec. 4 (theorem of Sec. 4.2): the automatic Verlet update gives
    results identical to detecting contacts among all pairs at every step, for
    any K, either cap reading, local or uniform skin; and the list is a superset
    of the contact set at every step (Def. verletlist)."""
    s = colliding(seed, poly=(seed == 1))
    x, v, rc, invm = arrays(s)
    p = dict(s.params)
    p.update(skin_mode=mode, K=K, cap_mode=cap, check_superset=1)
    steps = 300
    xn, vn, hn, _ = orc.run(dict(p, skin_mode=orc.NAIVE), x, v, rc, invm, steps)
    xm, vm, hm, _ = orc.run(p, x, v, rc, invm, steps)
    assert hn["contacts"].sum() > 100, "the workload must collide"
    assert np.array_equal(xm, xn) and np.array_equal(vm, vn)
    assert np.array_equal(hm["contacts"], hn["contacts"])
    assert np.array_equal(hm["kinetic_energy"], hn["kinetic_energy"])
    assert hm["missed"].sum() == 0
    if mode == 2:
        assert hm["rebuilt"].all()
    elif mode == 0 and K > 0:
        assert hm["rebuilt"].sum() < steps // 2


def test_k_zero_rebuilds_whenever_anything_moves(orc):
    """Eq. skin_formulus1 with K = 0 gives skin 0, so any motion violates Eq. update."""
    s = colliding(3)
    x, v, rc, invm = arrays(s)
    p = dict(s.params, K=0.0)
    _, _, h, _ = orc.run(p, x, v, rc, invm, 50)
    assert h["rebuilt"].all()


# ---------------------------------------------------------------- Alg. 1 completeness
def _cell_edge_min(L_C, eps):
    return L_C * (1.0 + 1e-9) + eps


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("eps", [0.0, 1e-3])
def test_linked_cell_equals_brute_force(orc, seed, eps):
    """Alg. 1 (Sec. 3.2) finds exactly the pairs whose spheres intersect, when the
    cells are not smaller than the bounding spheres (Sec. 3.2).  Positions are
    snapped to cell faces and corners half the time."""
    rng = np.random.default_rng(seed)
    n = 400
    L_C = 0.1
    lo, hi = np.zeros(3), np.array([1.0, 0.7, 0.45])
    x = rng.uniform(lo, hi, size=(n, 3))
    edge = (hi - lo) / np.maximum(1, np.floor((hi - lo) / _cell_edge_min(L_C, eps)))
    snap = rng.random(n) < 0.5
    x[snap] = np.round(x[snap] / edge * 2) * edge / 2
    r = rng.uniform(0.2, 0.5, size=n) * L_C
    bf = orc.broadphase_brute(x, r, eps)
    lc = orc.broadphase_linked_cell(x, r, eps, lo, hi, _cell_edge_min(L_C, eps), ring=1)
    assert len(bf) > 50
    assert np.array_equal(bf, lc)


def test_linked_cell_exhaustive_two_particles(orc):
    """Alg. 1 on every placement of two particles over a grid of points on cell
    faces, edges and corners of a 3x3x3-cell box, radii summing to the cell edge."""
    L_C = 0.25
    lo, hi = np.zeros(3), np.full(3, 0.75)
    pts = np.array([[i, j, k] for i in range(7) for j in range(7) for k in range(7)],
                   dtype=np.float64) * (0.75 / 6.0)
    edge_min = _cell_edge_min(L_C, 0.0)
    bad = 0
    for a in range(0, len(pts), 7):
        x = np.concatenate([pts[a:a + 1], pts], axis=0)
        r = np.full(len(x), L_C / 2)
        bf = orc.broadphase_brute(x, r, 0.0)
        lc = orc.broadphase_linked_cell(x, r, 0.0, lo, hi, edge_min, ring=1)
        bf0 = bf[bf[:, 0] == 0]
        lc0 = lc[lc[:, 0] == 0]
        bad += int(not np.array_equal(bf0, lc0))
    assert bad == 0


def test_linked_cell_small_n_enumerated(orc):
    """Alg. 1 vs brute force for every N <= 8 over many random draws, including
    coincident particles and particles outside the box (clamped to border cells)."""
    rng = np.random.default_rng(7)
    lo, hi = np.zeros(3), np.ones(3)
    for n in range(0, 9):
        for _ in range(150):
            x = rng.uniform(-0.1, 1.1, size=(n, 3))
            if n >= 2 and rng.random() < 0.2:
                x[1] = x[0]
            r = rng.uniform(0.01, 0.15, size=n)
            bf = orc.broadphase_brute(x, r, 1e-6)
            lc = orc.broadphase_linked_cell(x, r, 1e-6, lo, hi, _cell_edge_min(0.3, 1e-6), 1)
            assert np.array_equal(bf.reshape(-1, 2), lc.reshape(-1, 2))


def test_literal_cap_needs_two_rings(orc):
    """Reading of Eq. skin_formulus_mincell: with R_NL <= L_C taken literally, two
    spheres can reach 2 L_C and a one-ring search of Alg. 1 misses pairs two
    cells apart; a two-ring search finds them all."""
    rng = np.random.default_rng(3)
    L_C = 0.1
    lo, hi = np.zeros(3), np.ones(3)
    x = rng.uniform(0, 1, size=(300, 3))
    r = np.full(300, L_C)  # capped at the literal bound
    bf = orc.broadphase_brute(x, r, 0.0)
    one = orc.broadphase_linked_cell(x, r, 0.0, lo, hi, _cell_edge_min(L_C, 0.0), ring=1)
    two = orc.broadphase_linked_cell(x, r, 0.0, lo, hi, _cell_edge_min(L_C, 0.0), ring=2)
    assert len(one) < len(bf)
    assert np.array_equal(two, bf)


# ---------------------------------------------------------------- closed-form cadences
@pytest.mark.parametrize("K", [0, 1, 7, 50, 200])
def test_free_flight_cadence(orc, K):
    """Sec. 4.1 and Sec. 5.1: K is the number of skipped steps; with skin_p = K|v_p|dt
    and a straight-line displacement (Sec. 2) every particle in free flight
    violates Eq. update exactly after K+1 drifts, whatever its speed, so a broad
    phase runs at steps 0, K+1, 2(K+1), ... .  All values are dyadic, so this
    holds exactly."""
    s = synth.free_flight_system(4, [2.0 ** -4, 2.0 ** -5, 2.0 ** -6], seed=K, K=float(K))
    x, v, rc, invm = arrays(s)
    steps = 700
    _, _, h, _ = orc.run(s.params, x, v, rc, invm, steps)
    expect = np.zeros(steps, dtype=np.int32)
    expect[:: K + 1] = 1
    assert np.array_equal(h["rebuilt"], expect)
    assert h["contacts"].sum() == 0
    frac = report.executed_fraction(int(h["rebuilt"].sum()), steps)
    assert abs(frac - 100.0 * len(range(0, steps, K + 1)) / steps) < 1e-12


def test_capped_skin_cadence(orc):
    """Eq. skin_formulus_mincell with R4: a capped particle violates when its
    displacement exceeds cap - R_C, i.e. after floor((cap-R_C)/(v dt)) + 1 drifts
    (the fastest particle sets the global period)."""
    s = synth.free_flight_system(3, [2.0 ** -4, 2.0 ** -6], seed=1, K=5000.0)
    x, v, rc, invm = arrays(s)
    cap = s.params["cell_size"] / 2
    period = int(np.floor((cap - rc[0]) / (2.0 ** -4 * s.params["dt"]))) + 1
    assert period == 769
    steps = 2000
    _, _, h, _ = orc.run(s.params, x, v, rc, invm, steps)
    expect = np.zeros(steps, dtype=np.int32)
    expect[::period] = 1
    assert np.array_equal(h["rebuilt"], expect)


def test_cap_plateau(orc):
    """Sec. 5.4: once every skin reaches the cell-size cap, results and rebuild
    schedule no longer depend on K (K = 5000 vs 50000)."""
    s = colliding(5)
    x, v, rc, invm = arrays(s)
    p = dict(s.params)
    h = []
    for K in (5000.0, 50000.0):
        h.append(orc.run(dict(p, K=K), x, v, rc, invm, 200, want_list=True))
    assert np.array_equal(h[0][2], h[1][2])
    assert np.array_equal(h[0][3], h[1][3])


def test_particles_at_rest(orc):
    """Eq. skin_formulus1 with v = 0: the skin is 0, nothing moves, no broad phase
    after step 0, and the list holds exactly the pairs within R_C,i + R_C,j + eps."""
    s = synth.lattice_system(6, 6, 4, 0, 0, 0.0, 9)
    x, v, rc, invm = arrays(s)
    assert not v.any()
    xo, vo, h, lst = orc.run(s.params, x, v, rc, invm, 40, want_list=True)
    assert h["rebuilt"].tolist() == [1] + [0] * 39
    assert np.array_equal(xo, x) and not vo.any()
    assert np.array_equal(lst, orc.broadphase_brute(x, rc, s.params["eps"]))


# ---------------------------------------------------------------- P4c gravity
def test_constant_gravity_exact(orc):
    """Velocity Verlet (Sec. 3.1, Sec. 5.1) is exact for constant acceleration:
    x_n = x_0 + n dt v_0 + n^2 dt^2 g / 2.  Dyadic data make it exact in FP64."""
    dt = 2.0 ** -10
    g = np.array([0.0, -2.0 ** -2, 2.0 ** -3])
    x0 = np.array([[0.5, 0.5, 0.5]])
    v0 = np.array([[2.0 ** -5, 2.0 ** -4, -2.0 ** -6]])
    p = {"skin_mode": 0, "K": 200.0, "dt": dt, "cell_size": 2.0 ** -3, "eps": 0.0,
         "lo": (0, 0, 0), "hi": (1, 1, 1), "kn": 1.0, "gamma_n": 0.0, "g": tuple(g)}
    for n in (1, 2, 3, 17, 300):
        xo, vo, _, _ = orc.run(p, x0, v0, np.array([2.0 ** -6]), np.array([1.0]), n)
        assert np.array_equal(xo[0], x0[0] + n * dt * v0[0] + 0.5 * n * n * dt * dt * g)
        assert np.array_equal(vo[0], v0[0] + (n - 0.5) * dt * g)


# ---------------------------------------------------------------- the step record
def _exact(frac):
    """float of a Fraction that FP64 holds exactly (the closed forms below are
    chosen so that it does)."""
    f = float(frac)
    assert Fraction(f) == frac
    return f


def test_kinetic_energy_record_is_exact_under_gravity(orc):
    """The record of step n holds sum_p m_p |v^n_p|^2 / 2 with the full-step
    velocity v^n of velocity Verlet (Sec. 3.1, Sec. 5.1).  Under constant gravity
    and without contacts, v^n = v^0 + n dt g exactly; with dyadic data every term
    and every partial sum is exact, so the record equals the closed form bit for
    bit.  Masses 2, 1/2 and 1 make a missing factor 1/2 or the half-step velocity
    v^{n+1/2} visible."""
    dt = Fraction(1, 2 ** 10)
    g = (Fraction(0), Fraction(-1, 4), Fraction(1, 8))
    x0 = np.array([[0.5, 0.5, 0.5], [0.25, 0.75, 0.5], [0.75, 0.25, 0.5]])
    v0 = [(Fraction(1, 32), Fraction(1, 16), Fraction(-1, 64)),
          (Fraction(-3, 64), Fraction(0), Fraction(5, 128)),
          (Fraction(0), Fraction(-7, 256), Fraction(1, 16))]
    invm = [Fraction(1, 2), Fraction(2), Fraction(1)]
    p = {"skin_mode": 0, "K": 200.0, "dt": float(dt), "cell_size": 2.0 ** -3, "eps": 0.0,
         "lo": (0, 0, 0), "hi": (1, 1, 1), "kn": 1.0, "gamma_n": 0.0,
         "g": tuple(float(t) for t in g)}
    steps = 300
    _, _, h, _ = orc.run(p, x0, np.array([[float(c) for c in v] for v in v0]),
                         np.full(3, 2.0 ** -6), np.array([float(m) for m in invm]), steps)
    assert h["contacts"].sum() == 0
    for n in range(steps):
        ke = sum(Fraction(1, 2) / m * sum((v[a] + n * dt * g[a]) ** 2 for a in range(3))
                 for v, m in zip(v0, invm))
        assert h["kinetic_energy"][n] == _exact(ke), n


@pytest.mark.parametrize("K", [3, 50, 200])
def test_max_excess_record_in_free_flight(orc, K):
    """Eq. update in free flight: after the broad phase at step r the list holds the
    skins K |v_p| dt (Eq. skin_formulus1, uncapped here), and after step n particle p
    is (n + 1 - r) |v_p| dt from x0 (a straight line, Sec. 2).  The record's
    max_excess is therefore max_p (n + 1 - r - K) |v_p| dt: taken by the fastest
    particle once the skins are exceeded and by the slowest before.  The violator
    count is every particle exactly when n + 1 - r > K.  Dyadic data: exact."""
    speeds = [2.0 ** -4, 2.0 ** -5, 2.0 ** -6]
    s = synth.free_flight_system(4, speeds, seed=K + 11, K=float(K))
    x, v, rc, invm = arrays(s)
    moving = np.abs(v).max(axis=1)
    vmin, vmax = Fraction(moving.min()), Fraction(moving.max())
    assert vmin < vmax
    dt = Fraction(s.params["dt"])
    steps = 3 * (K + 1) + 7
    _, _, h, _ = orc.run(s.params, x, v, rc, invm, steps)
    r = 0
    for n in range(steps):
        if h["rebuilt"][n]:
            r = n
        k = n + 1 - r - K
        expect = k * (vmax if k >= 0 else vmin) * dt
        assert h["max_excess"][n] == _exact(expect), n
        assert h["violators"][n] == (len(moving) if k > 0 else 0), n


def test_list_pairs_record_counts_the_lattice_bonds(orc):
    """A lattice at rest with spacing exactly 2 R_C: every nearest-neighbour pair
    touches (delta = 0: no contact, Eq. delta) and lies within R_NL,i + R_NL,j of
    Alg. 1 (skin 0 at rest, Eq. skin_formulus1), diagonal pairs do not.  The record's
    list_pairs is then the closed-form number of lattice bonds at every step, its
    contact count 0, and the list returned is that many pairs."""
    nx, ny, nz = 5, 4, 3
    R = 2.0 ** -6
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    x = (np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1) + 8.0) * 2 * R
    n = len(x)
    p = {"skin_mode": 0, "K": 200.0, "dt": 2.0 ** -10, "cell_size": 2.0 ** -3, "eps": 2e-6,
         "lo": (0, 0, 0), "hi": (1, 1, 1), "kn": 1.0, "gamma_n": 0.0, "g": (0, 0, 0)}
    bonds = (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)
    _, _, h, lst = orc.run(p, x, np.zeros((n, 3)), np.full(n, R), np.ones(n), 20, want_list=True)
    assert (h["list_pairs"] == bonds).all()
    assert (h["contacts"] == 0).all()
    assert len(lst) == bonds


def test_list_pairs_record_is_the_list_in_use(orc):
    """The record of the last step counts the pairs of the list that step used,
    which is the list orc_run returns (Def. verletlist); at every step it holds
    at least the contacts (superset, Sec. 4.2)."""
    s = colliding(8)
    x, v, rc, invm = arrays(s)
    _, _, h, lst = orc.run(dict(s.params, check_superset=1), x, v, rc, invm, 150, want_list=True)
    assert h["list_pairs"][-1] == len(lst)
    assert (h["list_pairs"] >= h["contacts"]).all() and h["missed"].sum() == 0
    # the count changes only at a broad phase
    changed = np.nonzero(np.diff(h["list_pairs"]))[0] + 1
    assert h["rebuilt"][changed].all()


# ---------------------------------------------------------------- gravity stand-ins (Sec. 5.2)
def test_gravity_stand_in_static_overlap_is_one_percent():
    """The gravity of the hopper and incline stand-ins comes from their column
    depth: a column of `depth` particles of the heaviest mass resting on one
    contact of stiffness kn compresses it by depth m g / kn (the closed form of
    a linear spring under a static load, Sec. 5.1's linear spring-dashpot), and
    that is at most 1 % of the smallest R_C."""
    for s in (synth.hopper_system(2000, 5), synth.config_systems("H125")[0],
              synth.config_systems("H500")[0], synth.config_systems("INCLINE")[0],
              synth.silo_system(2000, 5), synth.config_systems("SILO")[0]):
        g = np.linalg.norm(s.params["g"])
        if s.meta["kind"] == "incline":
            g *= np.cos(np.radians(s.meta["theta_deg"]))  # the load along the floor normal
        m_max = 1.0 / s.vel_m[:, 3].min()
        overlap = s.meta["depth"] * m_max * g / s.params["kn"]
        assert overlap <= 0.01 * s.pos_r[:, 3].min() * (1 + 1e-6), (s.meta["kind"], s.n)


def test_stack_at_the_stand_in_gravity_rests_at_its_static_overlaps(orc):
    """A vertical stack of `depth` particles of the reduced hopper's smallest
    radius and heaviest mass, placed at the static overlaps of a linear spring
    under gravity (the contact below particle k carries the weight of the
    particles from k up), stays at rest over 2,000 steps, and its lowest contact
    (against the floor) is compressed by at most 1 % of R_C."""
    h = synth.hopper_system(2000, 5)
    D, R, m = h.meta["depth"], float(h.pos_r[:, 3].min()), float(1.0 / h.vel_m[:, 3].min())
    g, kn = -h.params["g"][2], h.params["kn"]
    z = np.empty(D)
    z[0] = R - D * m * g / kn
    for k in range(1, D):
        z[k] = z[k - 1] + 2 * R - (D - k) * m * g / kn
    x = np.stack([np.full(D, 0.5), np.full(D, 0.5), z], axis=1)
    p = dict(h.params, planes=[])
    p["hi"] = (1.0, 1.0, float(z[-1] + 2.0))
    xo, vo, hist, _ = orc.run(p, x, np.zeros((D, 3)), np.full(D, R), np.full(D, 1.0 / m), 2000)
    assert np.abs(xo - x).max() < 1e-12 and np.abs(vo).max() < 1e-9
    assert (hist["contacts"] == D - 1).all()
    assert R - xo[0, 2] <= 0.01 * R * (1 + 1e-6)


def test_hopper_stand_in_over_the_paper_run_length(orc):
    """The reduced hopper over 5,000 steps, the paper's shortest run (Sec. 5.1):
    no collapse under gravity.  Sampled every 250 steps, every overlap (pairs,
    box faces and hopper walls) stays below 8 % of the smallest R_C (impacts at
    the speeds gravity reaches; the static load alone gives 1 %), no cell of
    edge L_C holds more than 16 particles, and particles leave through the
    outlet into the collection bin."""
    s = synth.hopper_system(2000, 5)
    x, v, rc, invm = arrays(s)
    lo, hi, L = np.array(s.params["lo"]), np.array(s.params["hi"]), s.params["cell_size"]
    z_outlet = s.params["planes"][0][4]
    worst, fullest = 0.0, 0
    for c in range(20):
        x, v, h, _ = orc.run(dict(s.params, v_in_is_half_step=int(c > 0)), x, v, rc, invm, 250)
        pr = orc.contacts_brute(x, rc)
        if len(pr):
            worst = max(worst, (rc[pr[:, 0]] + rc[pr[:, 1]]
                                - np.linalg.norm(x[pr[:, 0]] - x[pr[:, 1]], axis=1)).max())
        worst = max(worst, np.maximum(rc[:, None] - (x - lo), rc[:, None] - (hi - x)).max())
        for pl in s.params["planes"]:
            above = x[:, 2] > pl[4]
            worst = max(worst, (rc[above] - (x[above] @ np.array(pl[:3]) - pl[3])).max())
        fullest = max(fullest, np.unique(np.floor((x - lo) / L).astype(int), axis=0,
                                         return_counts=True)[1].max())
    assert worst < 0.08 * rc.min(), worst / rc.min()
    assert fullest <= 16
    assert (x[:, 2] < z_outlet).sum() > 10


# ---------------------------------------------------------------- precision of the state
@pytest.mark.parametrize("seed", [0, 1])
def test_fp32_state_misses_the_parity_bar(orc, seed):
    """Why positions and velocities are kept in FP64: the paper fixes no
    precision, and the parity bar of this build is 1e-5 box units in position and
    1e-5 v_max in velocity after the run.  Storing the state in FP32 between
    steps (the FP32 record layout of a 16-byte position and a 16-byte velocity),
    even with every step computed in FP64, puts M1's velocities some 4e-3 v_max
    away from the FP64 run after its 200 steps, 400 times the bar: a contact
    overlap is a few 1e-5 box units, so an FP32 position (one ulp is 6e-8 near
    0.5) moves each contact force by about a thousandth.  The positions drift by
    some 5e-8 per step (the rounding of x + dt v) and leave the bar soon after
    step 200; the contact counts part by then too."""
    s = synth.config_systems("M1", seed=seed)[0]
    x, v, rc, invm = arrays(s)
    a = orc.run(s.params, x, v, rc, invm, 200)
    b = orc.run(dict(s.params, state_fp32=1), x, v, rc, invm, 200)
    ev = np.abs(a[1] - b[1]).max() / s.meta["v_max"]
    ex = np.abs(a[0] - b[0]).max()
    assert ev > 100 * 1e-5, ev
    assert 1e-6 < ex < 1e-5, ex
    a = orc.run(s.params, x, v, rc, invm, 300)
    b = orc.run(dict(s.params, state_fp32=1), x, v, rc, invm, 300)
    assert np.abs(a[0] - b[0]).max() > 1e-5
    assert not np.array_equal(a[2]["contacts"], b[2]["contacts"])


# ---------------------------------------------------------------- fixed interval, capped skin (R4)
def _two_body(v_b, gap, p_extra):
    """Particle A at rest, particle B approaching it along x."""
    R = 2.0 ** -6
    x = np.array([[0.5, 0.5, 0.5], [0.5 + 2 * R + gap, 0.5, 0.5]])
    v = np.array([[0.0, 0.0, 0.0], [-v_b, 0.0, 0.0]])
    p = {"skin_mode": 0, "K": 200.0, "dt": 2.0 ** -10, "cell_size": 2.0 ** -3, "eps": 0.0,
         "lo": (0, 0, 0), "hi": (1, 1, 1), "kn": 1e3, "gamma_n": 0.0, "g": (0, 0, 0),
         "check_superset": 1}
    p.update(p_extra)
    return x, v, np.full(2, R), np.ones(2), p


def test_fixed_interval_misses_contacts(orc):
    """Sec. 1 and Sec. 4.2: a list rebuilt at a fixed interval with a skin sized for
    typical speeds misses the contact of a fast particle; the automatic update of
    Def. autoverlet misses none."""
    x, v, rc, invm, p = _two_body(2.0 ** -2, 2.0 ** -6, {})
    fixed = dict(p, skin_mode=orc.FIXED_INTERVAL, fixed_interval=200, skin_uniform=2.0 ** -9)
    _, _, hf, _ = orc.run(fixed, x, v, rc, invm, 180)
    _, _, ha, _ = orc.run(p, x, v, rc, invm, 180)
    _, _, hn, _ = orc.run(dict(p, skin_mode=orc.NAIVE), x, v, rc, invm, 180)
    assert hn["contacts"].sum() > 0
    assert hf["missed"].sum() > 0
    assert ha["missed"].sum() == 0
    assert np.array_equal(ha["contacts"], hn["contacts"])


def test_fixed_interval_rebuilds_on_its_schedule_and_is_exact_with_a_safe_skin(orc):
    """The conventional scheme the paper compares with (Sec. 1): the list is
    rebuilt at step 0 and every I steps, whatever happens in between; with a
    skin no particle outruns in I steps it misses no contact and gives results
    identical to the contacts of all pairs at every step."""
    s = colliding(0)
    x, v, rc, invm = arrays(s)
    p = dict(s.params, check_superset=1)
    steps, I = 300, 5
    fixed = dict(p, skin_mode=orc.FIXED_INTERVAL, fixed_interval=I, skin_uniform=float(rc.max()))
    xf, vf, hf, _ = orc.run(fixed, x, v, rc, invm, steps)
    xn, vn, hn, _ = orc.run(dict(p, skin_mode=orc.NAIVE), x, v, rc, invm, steps)
    assert hn["contacts"].sum() > 100
    assert np.array_equal(hf["rebuilt"] != 0, np.arange(steps) % I == 0)
    assert hf["missed"].sum() == 0
    assert np.array_equal(xf, xn) and np.array_equal(vf, vn)


def test_uncapped_skin_in_validity_test_breaks_theorem(orc):
    """R4: Eq. update must use the skin left after the cap of Eq.
    skin_formulus_mincell.  Testing the displacement against the uncapped K|v|dt
    (a planted mistake) keeps a stale list and misses a contact."""
    x, v, rc, invm, p = _two_body(2.0 ** -2, 0.09, {"K": 5000.0})
    _, _, ok, _ = orc.run(p, x, v, rc, invm, 400)
    _, _, bad, _ = orc.run(dict(p, validity_uses_uncapped_skin=1), x, v, rc, invm, 400)
    assert ok["missed"].sum() == 0 and ok["contacts"].sum() > 0
    assert bad["missed"].sum() > 0


# ---------------------------------------------------------------- contact law
def test_touching_spheres_exert_no_force(orc):
    """Eq. delta: the particles collide only if the overlap is positive; exactly
    touching spheres (delta = 0) are not in contact and feel no force."""
    R = 2.0 ** -4
    x = np.array([[0.5, 0.5, 0.5], [0.5 + 2 * R, 0.5, 0.5], [0.5, 0.5 + 2 * R - 2.0 ** -20, 0.5]])
    rc = np.full(3, R)
    assert orc.contacts_brute(x, rc).tolist() == [[0, 2]]
    p = {"kn": 1.0, "gamma_n": 0.0, "lo": (0, 0, 0), "hi": (1, 1, 1)}
    F = orc.forces(p, x, np.zeros_like(x), rc, np.zeros((0, 2), np.int32))
    assert not F.any()


def _head_on(orc, kn, gamma, dt, m_b=1.0, wall=False):
    R = 0.05
    if wall:
        x = np.array([[0.3, 0.5, R + 1e-3]])
        v = np.array([[0.0, 0.0, -1.0]])
        rc, invm = np.array([R]), np.array([1.0 / m_b])
    else:
        x = np.array([[0.4, 0.5, 0.5], [0.4 + 2 * R + 1e-3, 0.5, 0.5]])
        v = np.array([[0.5, 0.0, 0.0], [-0.5, 0.0, 0.0]])
        rc, invm = np.full(2, R), np.array([1.0, 1.0 / m_b])
    p = {"skin_mode": 0, "K": 200.0, "dt": dt, "cell_size": 0.25, "eps": 0.0,
         "lo": (0, 0, 0), "hi": (1, 1, 1), "kn": kn, "gamma_n": gamma, "g": (0, 0, 0)}
    steps = 8000
    _, vo, h, _ = orc.run(p, x, v, rc, invm, steps)
    return vo, h


@pytest.mark.parametrize("gamma", [0.0, 5.0, 20.0])
def test_spring_dashpot_restitution_and_duration(orc, gamma):
    """Textbook solution of the normal linear spring-dashpot (the model of Sec. 5.1;
    the paper gives no constants): m_eff d'' + gamma d' + kn d = 0 gives contact
    time pi/omega_d and restitution exp(-gamma pi / (2 m_eff omega_d)), with
    omega_d = sqrt(kn/m_eff - (gamma/(2 m_eff))^2).  Pair and wall cases."""
    kn = 1e4
    for wall, m_eff in ((False, 0.5), (True, 1.0)):
        w0 = np.sqrt(kn / m_eff)
        wd = np.sqrt(w0 ** 2 - (gamma / (2 * m_eff)) ** 2)
        e = np.exp(-gamma * np.pi / (2 * m_eff * wd))
        dt = (np.pi / wd) / 2000
        vo, h = _head_on(orc, kn, gamma, dt, wall=wall)
        if wall:
            v_out = vo[0, 2]
            in_contact = None
        else:
            v_out = vo[1, 0] - vo[0, 0]
            in_contact = int(h["contacts"].sum())
        assert abs(v_out - e * 1.0) < 2e-3 * e, (wall, v_out, e)
        if in_contact is not None:
            assert abs(in_contact * dt - np.pi / wd) <= 2 * dt


def test_energy_bounded_without_damping(orc):
    """With gamma = 0 the contact force is conservative and velocity Verlet keeps
    the total energy (kinetic + kn delta^2/2 per contact) within O(dt^2) of its
    initial value over many collisions."""
    s = colliding(11)
    x, v, rc, invm = arrays(s)
    p = dict(s.params, gamma_n=0.0)
    _, _, h, _ = orc.run(p, x, v, rc, invm, 400)
    ke = h["kinetic_energy"]
    assert h["contacts"].sum() > 500
    # kinetic energy dips while springs are loaded but returns; never grows
    assert ke.max() <= ke[0] * (1 + 1e-3)
    assert ke[-1] > 0.9 * ke[0]


# ---------------------------------------------------------------- invariants
def test_momentum_and_angular_momentum_conserved(orc):
    """Pair forces are equal and opposite and central, so without walls or gravity
    the linear and angular momentum of the full-step velocities are conserved."""
    rng = np.random.default_rng(2)
    g = np.arange(5)
    X = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3) * 0.02 + 0.45
    X += rng.uniform(-1e-3, 1e-3, X.shape)
    V = rng.normal(0, 0.05, X.shape)
    rc = rng.uniform(0.009, 0.0105, len(X))
    m = rng.uniform(0.5, 2.0, len(X))
    p = {"skin_mode": 0, "K": 50.0, "dt": 1e-4, "cell_size": 0.03, "eps": 0.0,
         "lo": (0, 0, 0), "hi": (1, 1, 1), "kn": 1e4, "gamma_n": 3.0, "g": (0, 0, 0)}
    x1, vh, h, _ = orc.run(p, X, V, rc, 1 / m, 300)
    assert h["contacts"].sum() > 1000
    # forces at the final state give the full-step velocity
    C = orc.contacts_brute(x1, rc)
    F = orc.forces(p, x1, vh, rc, C)
    vfull = vh + 0.5 * p["dt"] * F / m[:, None]
    P0, P1 = (m[:, None] * V).sum(0), (m[:, None] * vfull).sum(0)
    assert np.abs(P1 - P0).max() < 1e-12
    # angular momentum about the origin, with x^S and the kick of F^S
    L0 = np.cross(X, m[:, None] * V).sum(0)
    L1 = np.cross(x1, m[:, None] * vfull).sum(0)
    assert np.abs(L1 - L0).max() < 1e-6 * np.abs(L0).max() + 1e-12


def test_permutation_invariance(orc):
    """Relabelling the particles relabels the result (same physics, sums in a
    different order): catches index mix-ups between i and j."""
    s = colliding(4, poly=True)
    x, v, rc, invm = arrays(s)
    perm = np.random.default_rng(0).permutation(len(rc))
    a = orc.run(s.params, x, v, rc, invm, 150)
    b = orc.run(s.params, x[perm], v[perm], rc[perm], invm[perm], 150)
    assert np.abs(a[0][perm] - b[0]).max() < 1e-12
    assert np.abs(a[1][perm] - b[1]).max() < 1e-10
    assert np.array_equal(a[2]["contacts"], b[2]["contacts"])


def test_walls_push_inward(orc):
    """Each wall is a plane boundary whose overlap is R_C minus the distance of the
    centre to the plane; the force points into the box on all six faces."""
    R = 0.1
    x = np.array([[0.05, 0.5, 0.5], [0.95, 0.5, 0.5], [0.5, 0.05, 0.5],
                  [0.5, 0.95, 0.5], [0.5, 0.5, 0.05], [0.5, 0.5, 0.95]])
    p = {"kn": 2.0, "gamma_n": 0.0, "lo": (0, 0, 0), "hi": (1, 1, 1)}
    F = orc.forces(p, x, np.zeros_like(x), np.full(6, R), np.zeros((0, 2), np.int32))
    expect = np.zeros((6, 3))
    for k in range(6):
        expect[k, k // 2] = (1 if k % 2 == 0 else -1) * 2.0 * 0.05
    assert np.allclose(F, expect, rtol=0, atol=1e-15)


# ---------------------------------------------------------------- Tab. summary formulas
def test_summary_table_formulas():
    """Eq. impr and the overhead column reproduce Tab. summary (Sec. 5.4).  The
    printed improvements differ from the recomputed ones by up to 0.021 (Avalanche,
    the table's own rounding), hence 0.025; the overhead divides by the default-K
    time (dividing by the optimum time misses Powder leveling by 0.047)."""
    with open(os.path.join(GOLDEN, "tab_summary.json")) as f:
        tab = json.load(f)
    for name, t0, _k, t_opt, i_opt, t_def, i_def, ovh in tab["rows"]:
        assert abs(report.improvement(t0, t_opt) - i_opt) <= 0.025, name
        assert abs(report.improvement(t0, t_def) - i_def) <= 0.025, name
        assert abs(report.overhead_to_optimum(t_def, t_opt) - ovh) <= 0.01, name


def test_resume_from_half_step_state(orc):
    """A run split in two (the second part resumed from x^n and the half-step
    velocity v^{n-1/2}) equals the uninterrupted run; the resumed method run starts
    with a broad phase (R7), which by the theorem of Sec. 4.2 changes nothing."""
    s = colliding(6)
    x, v, rc, invm = arrays(s)
    for mode in (orc.NAIVE, orc.SKIN_LOCAL):
        p = dict(s.params, skin_mode=mode)
        xa, va, _, _ = orc.run(p, x, v, rc, invm, 200)
        x1, v1, _, _ = orc.run(p, x, v, rc, invm, 120)
        xb, vb, _, _ = orc.run(dict(p, v_in_is_half_step=1), x1, v1, rc, invm, 80)
        assert np.array_equal(xa, xb) and np.array_equal(va, vb)


# ---------------------------------------------------------------- planar walls
def _incline(theta, n_steps, gamma=0.0):
    """One sphere resting, at its static overlap, on a frictionless plane through
    the origin tilted by theta about y, under vertical gravity.  The normal is
    n = (-sin, 0, cos); the tangent t = (cos, 0, sin) points up the slope."""
    R, g0, kn = 0.05, 2.0, 1e4
    n = np.array([-np.sin(theta), 0.0, np.cos(theta)])
    t = np.array([np.cos(theta), 0.0, np.sin(theta)])
    delta_star = g0 * np.cos(theta) / kn          # m = 1: kn delta = m g cos(theta)
    x0 = np.array([[0.0, 0.0, 0.0]]) + (R - delta_star) * n + 0.1 * t
    x0 = x0 + np.array([[5.0, 5.0, 5.0]])         # plane offset moves with the shift
    d = float(n @ np.array([5.0, 5.0, 5.0]))
    p = {"skin_mode": 0, "K": 200.0, "dt": 1e-3, "cell_size": 0.25, "eps": 0.0,
         "lo": (0, 0, 0), "hi": (10, 10, 10), "kn": kn, "gamma_n": gamma,
         "g": (0.0, 0.0, -g0), "planes": [(n[0], n[1], n[2], d, -1e9)]}
    return x0, p, n, t, d, R, delta_star, g0


@pytest.mark.parametrize("theta", [0.0, 0.3, 0.7])
def test_frictionless_incline(orc, theta):
    """A normal spring-dashpot plane exerts no tangential force, so the sphere slides
    down with the constant acceleration g sin(theta) of the textbook incline,
    exactly the Verlet trajectory x_t(n) = x_t(0) - (n dt)^2 g sin(theta) / 2,
    while its overlap stays at the static value m g cos(theta) / kn."""
    steps = 400
    x0, p, n, t, d, R, delta_star, g0 = _incline(theta, steps)
    xo, vo, _, _ = orc.run(p, x0, np.zeros((1, 3)), np.array([R]), np.array([1.0]), steps)
    T = steps * p["dt"]
    along = float((xo[0] - x0[0]) @ t)
    assert along == pytest.approx(-0.5 * g0 * np.sin(theta) * T * T, rel=1e-9, abs=1e-13)
    overlap = R - (float(xo[0] @ n) - d)
    assert overlap == pytest.approx(delta_star, rel=1e-6, abs=1e-12)


def test_floor_plane_equals_box_floor(orc):
    """A plane z = lo_z with normal +z reproduces the box's own floor bit for bit
    (a bouncing particle, gravity and damping on): same overlap, same law."""
    R = 2.0 ** -6
    x0 = np.array([[0.5, 0.5, 0.2]])
    v0 = np.array([[0.01, -0.02, -0.3]])
    base = {"skin_mode": 0, "K": 200.0, "dt": 2.0 ** -12, "cell_size": 2.0 ** -3, "eps": 0.0,
            "kn": 1e3, "gamma_n": 2.0, "g": (0.0, 0.0, -1.0), "hi": (1, 1, 1)}
    box = dict(base, lo=(0, 0, 0))
    plane = dict(base, lo=(0, 0, -4.0), planes=[(0.0, 0.0, 1.0, 0.0, -1e9)])
    for steps in (500, 3000):
        xa, va, ha, _ = orc.run(box, x0, v0, np.array([R]), np.array([1.0]), steps)
        xb, vb, hb, _ = orc.run(plane, x0, v0, np.array([R]), np.array([1.0]), steps)
        assert np.array_equal(xa, xb) and np.array_equal(va, vb)
    assert xa[0, 2] < 0.2 and xa[0, 2] > R * 0.5   # it fell and was held up


def test_plane_acts_only_above_its_height(orc):
    """Below z_min the wall is open (an outlet): the particle falls through on the
    exact constant-gravity trajectory; above it the same wall holds it."""
    dt = 2.0 ** -10
    g = np.array([0.0, 0.0, -2.0 ** -2])
    R = 2.0 ** -6
    x0 = np.array([[0.5, 0.5, 0.5]])
    v0 = np.zeros((1, 3))
    wall = (0.0, 0.0, 1.0, 0.5 - R / 2, 0.75)     # would overlap the particle by R/2
    p = {"skin_mode": 0, "K": 200.0, "dt": dt, "cell_size": 2.0 ** -3, "eps": 0.0,
         "lo": (0, 0, 0), "hi": (1, 1, 1), "kn": 1.0, "gamma_n": 0.0, "g": tuple(g),
         "planes": [wall]}
    n = 200
    xo, vo, _, _ = orc.run(p, x0, v0, np.array([R]), np.array([1.0]), n)
    assert np.array_equal(xo[0], x0[0] + 0.5 * n * n * dt * dt * g)
    held = dict(p, kn=1e4, planes=[wall[:4] + (0.25,)])
    xh, _, _, _ = orc.run(held, x0, v0, np.array([R]), np.array([1.0]), n)
    assert xh[0, 2] > x0[0, 2]                     # pushed up out of the overlap


def test_plane_count_is_bounded(orc):
    p = {"skin_mode": 0, "K": 1.0, "dt": 1e-3, "cell_size": 0.1, "lo": (0, 0, 0), "hi": (1, 1, 1),
         "kn": 1.0, "planes": [(0, 0, 1, 0, 0)] * 5}
    with pytest.raises(ValueError):
        orc.run(p, np.zeros((1, 3)) + 0.5, np.zeros((1, 3)), np.array([0.01]), np.array([1.0]), 1)


# ---------------------------------------------------------------- cylindrical walls
def _cylinder_base(**kw):
    p = {"skin_mode": 0, "K": 200.0, "dt": 2.0 ** -10, "cell_size": 2.0 ** -3, "eps": 0.0,
         "lo": (-1.0, -1.0, -1.0), "hi": (1.0, 1.0, 1.0), "kn": 1e3, "gamma_n": 2.0,
         "g": (0.0, 0.0, 0.0)}
    p.update(kw)
    return p


def test_cylinder_on_an_axis_line_equals_two_plane_walls_bitwise(orc):
    """Along a line through the axis the inside of a cylinder is, point for point,
    the pair of planes tangent to it there: the distance of the centre from the
    wall is R - |x| and the normal is -sign(x) e_x (sqrt(x^2) = |x| exactly in
    binary floating point).  Two particles fired outward along the x axis
    collide with a cylinder of radius 3/4 about the z axis and rebound exactly as
    from the planes x = 3/4 and x = -3/4 (the same spring-dashpot law), bit for
    bit, before, during and after contact."""
    x0 = np.array([[0.6, 0.0, 0.0], [-0.6, 0.0, 0.25]])
    v0 = np.array([[0.5, 0.0, 0.0], [-0.375, 0.0, 0.0]])
    rc = np.array([2.0 ** -5, 2.0 ** -5])
    invm = np.array([1.0, 2.0])
    cyl = _cylinder_base(cylinders=[(0.0, 0.0, 0.75, -np.inf)])
    planes = _cylinder_base(planes=[(-1.0, 0.0, 0.0, -0.75, -np.inf), (1.0, 0.0, 0.0, -0.75, -np.inf)])
    for steps in (150, 300, 600):
        xa, va, _, _ = orc.run(cyl, x0, v0, rc, invm, steps)
        xb, vb, _, _ = orc.run(planes, x0, v0, rc, invm, steps)
        assert np.array_equal(xa, xb) and np.array_equal(va, vb), steps
    assert va[0, 0] < 0 and va[1, 0] > 0                 # both came back
    assert abs(xa[0, 0]) < 0.75 and abs(xa[1, 0]) < 0.75


@pytest.mark.parametrize("theta", [0.3, 1.9, 4.0])
def test_cylinder_radial_impact_matches_its_tangent_plane(orc, theta):
    """A particle fired outward along a ray from the axis meets the wall head on;
    the normal stays the ray's direction, so the impact is that against the plane
    tangent to the cylinder where the ray crosses it: the same trajectory up to
    the rounding of the two geometries, and a restitution below one."""
    u = np.array([np.cos(theta), np.sin(theta), 0.0])
    c = np.array([0.125, -0.25, 0.0])
    R = 0.625
    x0 = (c + 0.4 * u)[None, :]
    v0 = (0.5 * u)[None, :]
    rc, invm = np.array([2.0 ** -5]), np.array([1.0])
    cyl = _cylinder_base(cylinders=[(c[0], c[1], R, -np.inf)])
    n = -u
    plane = _cylinder_base(planes=[(n[0], n[1], n[2], float(n @ (c + R * u)), -np.inf)])
    xa, va, _, _ = orc.run(cyl, x0, v0, rc, invm, 700)
    xb, vb, _, _ = orc.run(plane, x0, v0, rc, invm, 700)
    assert np.abs(xa - xb).max() < 1e-12 and np.abs(va - vb).max() < 1e-10
    vr = float(va[0] @ u)
    assert -0.5 < vr < 0.0                                # rebounded, energy dissipated


def test_cylinder_acts_only_above_its_height(orc):
    """Below z_min the silo is open: a particle fired outward under its lower
    edge flies out on the exact straight line (dyadic data); the same particle
    above z_min is turned back."""
    dt = 2.0 ** -10
    x0 = np.array([[0.5, 0.0, 0.0]])
    v0 = np.array([[0.5, 0.0, 0.0]])
    rc, invm = np.array([2.0 ** -5]), np.array([1.0])
    open_below = _cylinder_base(cylinders=[(0.0, 0.0, 0.75, 0.25)])
    n = 512
    xo, vo, _, _ = orc.run(open_below, x0, v0, rc, invm, n)
    assert np.array_equal(xo[0], x0[0] + n * dt * v0[0]) and np.array_equal(vo, v0)
    held = _cylinder_base(cylinders=[(0.0, 0.0, 0.75, -0.25)])
    xh, vh, _, _ = orc.run(held, x0, v0, rc, invm, n)
    assert xh[0, 0] < 0.75 and vh[0, 0] < 0


def test_cylinder_parameters_are_checked(orc):
    x, v = np.zeros((1, 3)), np.zeros((1, 3))
    with pytest.raises(ValueError):
        orc.run(_cylinder_base(cylinders=[(0.0, 0.0, 0.5, 0.0)] * 3), x, v, np.array([0.01]),
                np.array([1.0]), 1)
    with pytest.raises(ValueError):
        orc.run(_cylinder_base(cylinders=[(0.0, 0.0, 0.0, 0.0)]), x, v, np.array([0.01]),
                np.array([1.0]), 1)


def test_silo_stand_in_holds_its_column_and_discharges(orc):
    """The reduced silo stand-in over 5,000 steps, the paper's shortest run
    (Sec. 5.1), under the gravity of its column depth: sampled every 500 steps,
    every overlap (pairs, box faces and the cylinder above its lower edge) stays
    below 8 % of the smallest R_C, no centre above the lower edge lies outside
    the cylinder, and grains leave through the ring under the lower edge."""
    s = synth.silo_system(2000, 5)
    x, v, rc, invm = arrays(s)
    lo, hi = np.array(s.params["lo"]), np.array(s.params["hi"])
    cx, cy, R, z_min = s.params["cylinders"][0]
    worst = 0.0
    for c in range(10):
        x, v, h, _ = orc.run(dict(s.params, v_in_is_half_step=int(c > 0)), x, v, rc, invm, 500)
        pr = orc.contacts_brute(x, rc)
        if len(pr):
            worst = max(worst, (rc[pr[:, 0]] + rc[pr[:, 1]]
                                - np.linalg.norm(x[pr[:, 0]] - x[pr[:, 1]], axis=1)).max())
        worst = max(worst, np.maximum(rc[:, None] - (x - lo), rc[:, None] - (hi - x)).max())
        rho = np.hypot(x[:, 0] - cx, x[:, 1] - cy)
        above = x[:, 2] > z_min
        if above.any():
            worst = max(worst, (rc[above] - (R - rho[above])).max())
            assert (rho[above] < R).all()
    assert worst < 0.08 * rc.min(), worst / rc.min()
    assert (rho > R).sum() > 50                           # discharged through the ring


def test_mutation_check_patterns_match_the_oracle():
    """Every mistake oracle/mutation_check.py plants must still have its target
    text in orc.c (a stale pattern would silently test nothing)."""
    import ast
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = open(os.path.join(here, "oracle", "mutation_check.py")).read()
    tree = ast.parse(src)
    mut = next(node.value for node in tree.body if isinstance(node, ast.Assign)
               and getattr(node.targets[0], "id", None) == "MUT")
    orc_c = open(os.path.join(here, "oracle", "orc.c")).read()
    items = ast.literal_eval(mut)
    assert len(items) >= 20
    for name, target, _ in items:
        assert target in orc_c, name


# ---------------------------------------------------------------- friction (f2)
def _collide(u_n, u_t, p_extra, R=2.0 ** -6, k=1e6):
    """Two equal unit-mass spheres touching at the start of a collision: relative
    normal velocity u_n (approaching along x), relative tangential velocity u_t
    (along y); normal and tangential springs of stiffness k, no dashpots.  The
    contact lasts pi / sqrt(2 k) (about 290 steps at dt = 2^-17)."""
    x = np.array([[0.5, 0.5, 0.5], [0.5 + 2 * R - 1e-9, 0.5, 0.5]])
    v = np.array([[0.5 * u_n, 0.5 * u_t, 0.0], [-0.5 * u_n, -0.5 * u_t, 0.0]])
    p = {"skin_mode": 0, "K": 200.0, "dt": 2.0 ** -17, "cell_size": 2.0 ** -3, "eps": 0.0,
         "lo": (0, 0, 0), "hi": (1, 1, 1), "kn": k, "gamma_n": 0.0, "g": (0, 0, 0),
         "v_in_is_half_step": 1, "kt": k, "gamma_t": 0.0}
    p.update(p_extra)
    return x, v, np.full(2, R), np.ones(2), p


def test_friction_off_is_the_frictionless_law(orc):
    x, v, rc, invm, p = _collide(0.2, 0.1, {"mu": 0.0})
    a = orc.run(p, x, v, rc, invm, 300)
    for extra in ({"kt": 1e6, "gamma_t": 1.0, "mu": 0.0}, {"kt": 0.0, "gamma_t": 0.0, "mu": 0.5}):
        b = orc.run(dict(p, **extra), x, v, rc, invm, 300)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    c = orc.run(dict(p, mu=0.5), x, v, rc, invm, 300)
    assert not np.array_equal(a[1], c[1])                 # and friction on does act


def test_sliding_collision_transfers_mu_times_the_normal_impulse(orc):
    """While a contact slides, |F_t| = mu F_n at every step, so over a collision
    that slides throughout the tangential impulse is mu times the normal one
    (Coulomb's law): |du_t| = mu |du_n| = 2 mu u_n for the elastic normal
    rebound, and the sliding is slowed, never reversed."""
    mu, u_n, u_t = 0.3, 0.002, 0.003
    x, v, rc, invm, p = _collide(u_n, u_t, {"mu": mu})
    xo, vo, h, _ = orc.run(p, x, v, rc, invm, 400)
    assert h["contacts"][0] == 1 and h["contacts"][-1] == 0
    du = (vo[0] - vo[1]) - (v[0] - v[1])
    assert du[1] < 0 and (vo[0] - vo[1])[1] > 0
    # the normal turns by ~2e-4 rad while the spheres slide past each other,
    # which moves the ratio by ~u t_c / R (3.5e-4 here)
    assert abs(du[1]) / abs(du[0]) == pytest.approx(mu, rel=1e-3)
    assert abs(du[0]) == pytest.approx(2 * u_n, rel=1e-3)


def test_sticking_contact_is_an_elastic_tangential_rebound(orc):
    """An unbounded Coulomb limit (the contact sticks) and kt = kn: the tangential
    spring completes half a period while the normal one does, so the relative
    tangential velocity comes back reversed and the kinetic energy is the same
    (an elastic tangential rebound), to the integrator's error."""
    u_n, u_t = 0.2, 0.01
    x, v, rc, invm, p = _collide(u_n, u_t, {"mu": 1e30})
    _, vo, h, _ = orc.run(p, x, v, rc, invm, 400)
    assert h["contacts"][-1] == 0
    rel = vo[0] - vo[1]
    assert rel[1] == pytest.approx(-u_t, rel=2e-2)
    assert rel[0] == pytest.approx(-u_n, rel=1e-3)
    assert 0.5 * (vo ** 2).sum() == pytest.approx(0.5 * (v ** 2).sum(), rel=1e-3)
    # a finite mu and a fast slide: energy is lost
    x, v, rc, invm, p = _collide(u_n, 0.3, {"mu": 0.3})
    _, vo, _, _ = orc.run(p, x, v, rc, invm, 400)
    assert 0.5 * (vo ** 2).sum() < 0.99 * 0.5 * (v ** 2).sum()


def test_sticking_contact_with_tangential_damping_is_a_damped_oscillator(orc):
    """A contact that sticks throughout (unbounded Coulomb limit), kt = kn, no
    normal damping and a tangential dashpot gamma_t: the relative tangential
    motion s'' + 2 gamma_t s' + 2 kt s = 0 (unit masses) is a damped oscillator
    of w0 = sqrt(2 kt) and damping ratio z = gamma_t / w0, cut off when the
    undamped normal contact ends at t_c = pi / w0.  Its textbook solution fixes
    the relative tangential velocity the pair leaves with."""
    k, z, u_n, u_t = 1e6, 0.2, 0.2, 0.01
    w0 = np.sqrt(2 * k)
    x, v, rc, invm, p = _collide(u_n, u_t, {"mu": 1e30, "gamma_t": z * w0}, k=k)
    _, vo, h, _ = orc.run(p, x, v, rc, invm, 400)
    assert h["contacts"][0] == 1 and h["contacts"][-1] == 0
    wd, tc = w0 * np.sqrt(1 - z * z), np.pi / w0
    expect = u_t * np.exp(-z * w0 * tc) * (np.cos(wd * tc) - z / np.sqrt(1 - z * z) * np.sin(wd * tc))
    assert expect < -0.5 * u_t   # reversed, and damped to about half
    rel = vo[0] - vo[1]
    assert rel[1] == pytest.approx(expect, rel=2e-2)
    assert rel[0] == pytest.approx(-u_n, rel=1e-3)   # the normal rebound is undamped


def test_stored_springs_lie_in_the_tangent_plane_and_are_opposite(orc):
    """The tangential spring is an elongation in the contact's tangent plane:
    each step turns the previous spring into the plane normal to the current
    contact normal before adding v_t dt, so the spring a step stores is normal
    to the normal it was computed with (to rounding), however far the contact
    has turned since it began; and the two particles of a pair hold opposite
    springs.  A grazing collision that sticks (unbounded Coulomb limit, a soft
    tangential spring) turns the normal by about 10^-2 rad in 100 steps."""
    x, v, rc, invm, p = _collide(0.2, 0.5, {"mu": 1e30, "kt": 1e4})
    for steps in (20, 60, 100):
        xo, vo, h, (off, j, xi) = orc.run_springs(p, x, v, rc, invm, steps)
        xr, vr, _, _ = orc.run(p, x, v, rc, invm, steps)
        assert np.array_equal(xo, xr) and np.array_equal(vo, vr)
        assert h["contacts"][-1] == 1 and list(off) == [0, 1, 2] and list(j) == [1, 0]
        assert np.array_equal(xi[0], -xi[1])
        # the last step's positions: the drift x^S = x^{S-1} + dt v^{S-1/2}, undone
        xp = xo - p["dt"] * vo
        nrm = (xp[0] - xp[1]) / np.linalg.norm(xp[0] - xp[1])
        turned = np.arccos(np.clip(nrm @ (x[0] - x[1]) / np.linalg.norm(x[0] - x[1]), -1, 1))
        assert turned > 1e-3 * steps / 20
        assert abs(xi[0] @ nrm) <= 1e-12 * np.linalg.norm(xi[0])
        assert np.linalg.norm(xi[0]) > 0.5 * 0.5 * steps * p["dt"]   # it did grow


def test_springs_of_a_frictional_cascade_are_tangent_and_opposite(orc):
    """The same invariants over every contact of a frictional cascade: each
    particle's contacts come in ascending partner order, the two springs of a
    pair are exact opposites, and every spring is normal to its contact normal
    to rounding."""
    s = synth.config_systems("M1", seed=2, scale=0.4)[0]
    x, v, rc, invm = arrays(s)
    p = dict(s.params, kt=0.5 * s.params["kn"], gamma_t=0.5 * s.params["gamma_n"], mu=0.4,
             lo=(-10, -10, -10), hi=(11, 11, 11))
    xo, vo, h, (off, j, xi) = orc.run_springs(p, x, v, rc, invm, 150)
    assert len(j) == 2 * h["contacts"][-1] > 20 and off[-1] == len(j)
    xp = xo - p["dt"] * vo
    where = {}
    for i in range(len(rc)):
        part = j[off[i]:off[i + 1]]
        assert (np.diff(part) > 0).all()
        for e, jj in zip(range(off[i], off[i + 1]), part):
            where[(i, int(jj))] = e
    for (i, jj), e in where.items():
        assert np.array_equal(xi[e], -xi[where[(jj, i)]])
        nrm = (xp[i] - xp[jj]) / np.linalg.norm(xp[i] - xp[jj])
        assert abs(xi[e] @ nrm) <= 1e-12 * np.linalg.norm(xi[e]) + 1e-300


def _damped_normal_impulses(k, gamma_n, u_n):
    """Positive and negative parts of the normal impulse of a linear
    spring-dashpot collision of two unit masses: the overlap obeys
    d'' + 2 gamma_n d' + 2 k d = 0 with d(0) = 0, d'(0) = u_n, the force is
    k d + gamma_n d', and the contact lasts while d > 0 (t < pi / w_d)."""
    from scipy.integrate import quad
    from scipy.optimize import brentq
    w0 = np.sqrt(2 * k)
    z = gamma_n / w0
    wd = w0 * np.sqrt(1 - z * z)
    d = lambda t: u_n / wd * np.exp(-z * w0 * t) * np.sin(wd * t)
    dp = lambda t: u_n * np.exp(-z * w0 * t) * (np.cos(wd * t) - z * w0 / wd * np.sin(wd * t))
    f = lambda t: k * d(t) + gamma_n * dp(t)
    end = np.pi / wd
    t0 = brentq(f, 0.5 * end, end * (1 - 1e-12))   # the force turns attractive once
    pos = quad(f, 0.0, t0, epsabs=0.0, epsrel=1e-12)[0]
    neg = -quad(f, t0, end, epsabs=0.0, epsrel=1e-12)[0]
    return pos, neg, np.exp(-z * np.pi / np.sqrt(1 - z * z))


def test_sliding_limit_follows_the_compressive_part_of_the_normal_force(orc):
    """Coulomb's limit is mu times the normal force where it compresses and zero
    where the normal dashpot pulls the separating pair together: over a damped
    collision that slides throughout, the tangential impulse is mu times the
    positive part of the normal impulse, which the textbook solution of the
    damped normal contact gives (here the pulling part is 5 % of it).  The
    normal impulse itself gives the restitution coefficient exp(-z pi / sqrt(1 - z^2))."""
    k, z, u_n, u_t, mu = 1e6, 0.3, 0.002, 0.005, 0.3
    gamma_n = z * np.sqrt(2 * k)
    # a stiff tangential spring: the contact slides from its first step on
    x, v, rc, invm, p = _collide(u_n, u_t, {"mu": mu, "gamma_n": gamma_n, "kt": 1e8}, k=k)
    _, vo, h, _ = orc.run(p, x, v, rc, invm, 400)
    assert h["contacts"][0] == 1 and h["contacts"][-1] == 0
    pos, neg, e = _damped_normal_impulses(k, gamma_n, u_n)
    assert neg > 0.05 * pos
    du = (vo[0] - vo[1]) - (v[0] - v[1])
    # the dashpot's first-order time-step error: 1.4e-3 (normal) and 1.9e-3
    # (tangential) at dt = 2^-17, 0.7e-3 and 1.2e-3 at half of it
    assert abs(du[0]) == pytest.approx(2 * (pos - neg), rel=4e-3)
    assert abs(du[0]) == pytest.approx(u_n * (1 + e), rel=4e-3)
    assert du[1] < 0 and (vo[0] - vo[1])[1] > 0      # slowed, never reversed
    assert abs(du[1]) == pytest.approx(2 * mu * pos, rel=1e-2)


def test_slide_then_stick_settles_where_the_closed_form_puts_it(orc):
    """Sphere B on sphere A on the (frictionless) floor under gravity g, both at
    their static overlaps; B starts with a horizontal velocity u.  Unit masses,
    normal force g.  While the contact slides, the relative velocity w falls at
    2 mu g and the stored spring is the one that gives the force on the cone,
    kt s = mu g - gamma_t w; the trial force of the next instant exceeds the cone
    as long as kt w > 2 mu g gamma_t, so the contact sticks at
    w* = 2 mu g gamma_t / kt, after sliding (u^2 - w*^2) / (4 mu g).  The damped
    spring then relaxes to zero, which moves the pair back by its value at
    sticking, (mu g - gamma_t w*) / kt, and both spheres end at u / 2.  Storing
    the spring without its dashpot part would give u^2 / (4 mu g) - mu g / kt,
    3 % less here; keeping the slid distance in it would undo the slide."""
    R, g, kn, kt, mu, u = 2.0 ** -6, 1.0, 1e6, 1e6, 0.5, 4e-3
    gamma_t = 0.5 * np.sqrt(2 * kt)
    z_a = R - 2 * g / kn
    x = np.array([[0.5, 0.5, z_a], [0.5, 0.5, z_a + 2 * R - g / kn]])
    v = np.array([[0.0, 0.0, 0.0], [u, 0.0, 0.0]])
    p = {"skin_mode": 0, "K": 200.0, "dt": 2.0 ** -17, "cell_size": 2.0 ** -3, "eps": 0.0,
         "lo": (0, 0, 0), "hi": (1, 1, 1), "kn": kn, "gamma_n": 200.0, "g": (0, 0, -g),
         "kt": kt, "gamma_t": gamma_t, "mu": mu}
    xo, vo, h, _ = orc.run(p, x, v, np.full(2, R), np.ones(2), 2800)
    assert (h["contacts"] == 1).all()          # B stays on A throughout (walls not counted)
    w_stick = 2 * mu * g * gamma_t / kt
    assert (u - w_stick) / (2 * mu * g) < 0.25 * 2800 * p["dt"]   # then 12 decay times
    expect = (u * u - w_stick ** 2) / (4 * mu * g) - (mu * g - gamma_t * w_stick) / kt
    without_dashpot_part = u * u / (4 * mu * g) - mu * g / kt
    assert abs(without_dashpot_part - expect) > 0.03 * expect
    offset = (xo[1, 0] - xo[0, 0]) - (x[1, 0] - x[0, 0])
    # first-order time-step error: 8e-4 at dt = 2^-17, 6e-4 at half of it
    assert offset == pytest.approx(expect, rel=5e-3)
    assert vo[0, 0] == pytest.approx(0.5 * u, rel=1e-5) and vo[1, 0] == pytest.approx(0.5 * u, rel=1e-5)


def test_friction_conserves_momentum_and_the_method_stays_exact(orc):
    """A cascade of frictional collisions: total momentum is conserved to rounding
    (the pair's two springs stay opposite), and the local Verlet buffer gives the
    same bits as brute force every step (Sec. 4.2: the history belongs to the
    contact, not to the list)."""
    s = synth.config_systems("M1", seed=2, scale=0.4)[0]
    x = s.pos_r[:, :3].astype(np.float64)
    v = s.vel_m[:, :3].astype(np.float64)
    rc = s.pos_r[:, 3].astype(np.float64)
    invm = s.vel_m[:, 3].astype(np.float64)
    fr = {"kt": 0.5 * s.params["kn"], "gamma_t": 0.5 * s.params["gamma_n"], "mu": 0.4}
    p = dict(s.params, **fr)
    far = dict(p, lo=(-10, -10, -10), hi=(11, 11, 11))   # no walls touched
    xo, vo, h, _ = orc.run(far, x, v, rc, invm, 300)
    assert h["contacts"].max() > 10
    m = 1.0 / invm
    p0 = (m[:, None] * v).sum(axis=0)
    p1 = (m[:, None] * vo).sum(axis=0)
    assert np.abs(p1 - p0).max() <= 1e-12 * np.abs(m[:, None] * v).sum()
    xn, vn, hn, _ = orc.run(dict(p, skin_mode=orc.NAIVE), x, v, rc, invm, 300)
    xm, vm, hm, _ = orc.run(p, x, v, rc, invm, 300)
    assert np.array_equal(xn, xm) and np.array_equal(vn, vm)
    assert np.array_equal(hn["contacts"], hm["contacts"]) and hm["rebuilt"].sum() < 300


# ---------------------------------------------------------------- threads
@pytest.mark.parametrize("case", ["method", "friction", "naive", "hopper"])
def test_oracle_threads_give_identical_bits(orc, case):
    """The oracle's loops over particles may run on several threads (for the CPU
    baseline on all host cores; loops of 16,384 particles or list entries and
    more, and brute force over 512 particles or more); positions, velocities,
    every record field and the final list are the same bits on 1, 3 and 8
    threads."""
    if case == "hopper":
        s = synth.hopper_system(20000, 5)
        p = dict(s.params)
    elif case == "naive":
        s = synth.lattice_system(8, 8, 8, 3, 2, 0.3, 11, polydisperse=True)
        p = dict(s.params, skin_mode=orc.NAIVE)
    else:
        s = synth.config_systems("M1", seed=11)[0]
        p = dict(s.params)
        if case == "friction":
            p.update(kt=0.5 * p["kn"], gamma_t=0.5 * p["gamma_n"], mu=0.4)
    x, v, rc, invm = arrays(s)
    ref = None
    before = orc.get_threads()
    try:
        for t in (1, 3, 8):
            orc.set_threads(t)
            out = orc.run(p, x, v, rc, invm, 200, want_list=case != "naive")
            if ref is None:
                ref = out
                assert out[2]["contacts"].sum() > 0
                continue
            assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1]), t
            assert np.array_equal(out[2], ref[2]), t
            if case != "naive":
                assert np.array_equal(out[3], ref[3]), t
    finally:
        orc.set_threads(before)
