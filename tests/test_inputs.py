"""The seeded synthetic inputs (synth/) against their stated recipe, on the CPU.

The generators hold none of the method's arithmetic; both the oracle and the
HIP path read their output.  These checks pin what the inputs are: the sizes of
every named workload, the jittered lattice (spacing, jitter bound, radius, no
initial overlap), the velocity regions and their Gaussian noise, the walls and
gravity of the stand-ins, and that a seed fixes every value (also when the
systems of a batch are generated in a process pool).
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import synth
from synth import systems as S


@pytest.mark.parametrize("name,n", [
    ("M1", 16_384), ("M2", 4_194_304), ("H125", 125_847), ("H250", 254_700),
    ("H500", 504_498), ("SILO", 126_368), ("INCLINE", 249_860),
])
def test_workload_sizes(name, n):
    (s,) = synth.config_systems(name)
    assert s.n == n and s.pos_r.shape == (n, 4) and s.vel_m.shape == (n, 4)
    assert np.isfinite(s.pos_r).all() and np.isfinite(s.vel_m).all()
    lo, hi = np.array(s.params["lo"]), np.array(s.params["hi"])
    assert (s.pos_r[:, :3] > lo).all() and (s.pos_r[:, :3] < hi).all()


def test_batch_workload_sizes():
    """M3: 64 systems of uneven sides, 19,873,792 particles; M5: 16 systems of
    512 x 512 x 64, 268,435,456 particles (counted from the generator's
    arguments, without generating them)."""
    m3 = S._lattice_args("M3", 0, 1.0)
    m5 = S._lattice_args("M5", 0, 1.0)
    assert len(m3) == 64 and sum(a[0] * a[1] * a[2] for a in m3) == 19_873_792
    assert len({(a[0], a[1]) for a in m3}) > 5        # uneven sizes
    assert len(m5) == 16 and all(a[:3] == (512, 512, 64) for a in m5)
    assert sum(a[0] * a[1] * a[2] for a in m5) == 268_435_456
    assert len({a[-1] for a in m3}) == 64 and len({a[-1] for a in m5}) == 16   # one seed each


def test_a_seed_fixes_every_value():
    a = synth.lattice_system(12, 10, 6, 3, 2, 0.1, 7)
    b = synth.lattice_system(12, 10, 6, 3, 2, 0.1, 7)
    c = synth.lattice_system(12, 10, 6, 3, 2, 0.1, 8)
    assert np.array_equal(a.pos_r, b.pos_r) and np.array_equal(a.vel_m, b.vel_m)
    assert a.params == b.params
    assert not np.array_equal(a.pos_r, c.pos_r) and not np.array_equal(a.vel_m, c.vel_m)
    h1, h2 = synth.config_systems("H125", scale=0.5), synth.config_systems("H125", scale=0.5)
    assert np.array_equal(h1[0].pos_r, h2[0].pos_r) and np.array_equal(h1[0].vel_m, h2[0].vel_m)


def test_a_process_pool_generates_the_same_batch():
    serial = synth.config_systems("M3", seed=1, scale=0.125)
    pooled = synth.config_systems("M3", seed=1, scale=0.125, workers=2)
    assert len(serial) == len(pooled) == 64
    for s, p in zip(serial, pooled):
        assert np.array_equal(s.pos_r, p.pos_r) and np.array_equal(s.vel_m, p.vel_m)


def test_jittered_lattice_recipe():
    """Spacing a = 1/(largest side + 1); each particle within 0.04 a of its site
    (index + 1) a along every axis, in lattice order (x fastest, then y, then z);
    R_C = 0.45 a and unit mass; so neighbours are at least 0.92 a apart and no
    two particles overlap at the start (0.92 a > 2 R_C = 0.9 a)."""
    (s,) = synth.config_systems("M1")
    nx, ny, nz = 32, 32, 16
    a = 1.0 / 33
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    site = (np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1) + 1.0) * a
    off = s.pos_r[:, :3].astype(np.float64) - site
    assert np.abs(off).max() <= 0.04 * a * (1 + 1e-6)
    assert np.abs(off).max() > 0.039 * a                  # the jitter spans its range
    assert np.allclose(s.pos_r[:, 3], 0.45 * a, rtol=1e-7)
    assert np.array_equal(s.vel_m[:, 3], np.ones(s.n, np.float32))
    assert s.params["hi"] == pytest.approx(((nx + 1) * a, (ny + 1) * a, (nz + 1) * a), rel=1e-7)
    pairs = cKDTree(s.pos_r[:, :3].astype(np.float64)).query_pairs(0.9 * a)
    assert len(pairs) == 0


def test_velocity_regions_and_noise():
    """Without noise the velocities are piecewise constant: at most one value per
    box or ball plus rest, each of speed at most v_max, with particles at rest.
    The noise is what the same seed adds on top: i.i.d. Gaussian of standard
    deviation sigma v_max per component."""
    args = (32, 32, 16, 8, 4)
    s0 = synth.lattice_system(*args, 0.0, 3)
    s1 = synth.lattice_system(*args, 0.05, 3)
    v_max = s0.meta["v_max"]
    v0 = s0.vel_m[:, :3].astype(np.float64)
    distinct = np.unique(v0, axis=0)
    assert 2 <= len(distinct) <= 8 + 4 + 1
    assert (np.linalg.norm(distinct, axis=1) <= v_max * (1 + 1e-6)).all()
    at_rest = (v0 == 0).all(axis=1).mean()
    assert 0.05 < at_rest < 0.95
    assert np.array_equal(s0.pos_r, s1.pos_r)             # the noise comes last
    noise = s1.vel_m[:, :3].astype(np.float64) - v0
    sd = 0.05 * v_max
    m = noise.size
    assert abs(noise.mean()) < 5 * sd / np.sqrt(m)
    assert noise.std() == pytest.approx(sd, rel=0.02)
    # Gaussian tails: about 0.27 % beyond three standard deviations
    assert (np.abs(noise) > 3 * sd).mean() == pytest.approx(0.0027, abs=0.001)


def test_gravity_stand_in_geometries():
    """The hopper's two walls are unit normals at 30 degrees from the vertical
    (n_z = sin 30 degrees), acting above the outlet (11 spacings: a 10-site bin);
    the silo's cylinder stands on the box's axis and acts above its 4-spacing gap;
    the incline's gravity is tilted by 25 degrees about y.  No particle starts
    overlapping a wall, and radii are polydisperse in [0.35 a, 0.45 a] with
    mass proportional to volume."""
    (h,) = synth.config_systems("H125")
    a = h.meta["a"]
    x = h.pos_r[:, :3].astype(np.float64)
    r = h.pos_r[:, 3].astype(np.float64)
    assert len(h.params["planes"]) == 2
    for pl in h.params["planes"]:
        n = np.array(pl[:3])
        assert np.linalg.norm(n) == pytest.approx(1.0, abs=1e-15)
        assert n[2] == pytest.approx(0.5, rel=1e-7) and abs(n[0]) == pytest.approx(np.sqrt(0.75), rel=1e-7)
        assert pl[4] == pytest.approx(11 * a, rel=1e-6)
        above = x[:, 2] > pl[4]
        assert above.all() and ((x @ n - pl[3]) - r > 0).all()
    assert r.min() >= 0.35 * a * (1 - 1e-6) and r.max() <= 0.45 * a * (1 + 1e-6)
    m = 1.0 / h.vel_m[:, 3].astype(np.float64)
    assert np.allclose(m, (r / (0.45 * a)) ** 3, rtol=1e-5)
    assert h.params["g"][0] == 0 and h.params["g"][1] == 0 and h.params["g"][2] < 0

    (s,) = synth.config_systems("SILO")
    a = s.meta["a"]
    x = s.pos_r[:, :3].astype(np.float64)
    r = s.pos_r[:, 3].astype(np.float64)
    (cx, cy, R, z_min), = s.params["cylinders"]
    hi = np.array(s.params["hi"])
    assert cx == pytest.approx(0.5 * hi[0], rel=1e-6) and cy == pytest.approx(0.5 * hi[1], rel=1e-6)
    assert z_min == pytest.approx(4.5 * a, rel=1e-6)
    assert ((R - np.hypot(x[:, 0] - cx, x[:, 1] - cy)) - r > 0).all()

    (i,) = synth.config_systems("INCLINE")
    g = np.array(i.params["g"])
    assert np.degrees(np.arctan2(g[0], -g[2])) == pytest.approx(25.0, abs=1e-5) and g[1] == 0
