"""Synthetic DEM workloads standing in for the paper's test cases.

The paper's own cases (hopper discharge, inclined plane, avalanche, biomass
furnace, powder levelling; Sec. 5.2) need geometry and CFD data that are not
published, so every input here is drawn from a seeded generator with the
structure the paper stresses: several coexisting flow regimes (Sec. 1), i.e.
regions moving at different speeds next to regions at rest.

Placement: a jittered simple-cubic lattice of nx*ny*nz sites with spacing
a = 1/(max(nx,ny,nz)+1); site (i,j,k) sits at ((i+1)a, (j+1)a, (k+1)a) plus a
uniform jitter of +-0.04a per axis; the box is [0,(nx+1)a] x [0,(ny+1)a] x
[0,(nz+1)a] with a wall on every face, so its longest side is 1.
Particles: radius R_C = 0.45a (or U[0.35a,0.45a] when polydisperse), mass
m = (R_C/0.45a)^3.
Velocities: n_boxes axis-aligned boxes and n_balls balls drawn in lattice-index
space, each with a speed U[0,1] v_max along a direction uniform on the sphere,
painted in draw order (boxes, then balls; later regions overwrite earlier ones);
particles outside every region are at rest; then i.i.d. N(0, (sigma v_max)^2)
noise is added to every component of every particle.
Particle index order is the lattice order (x fastest, then y, then z).

Physical constants (the paper gives none; Sec. 5.1 names the model only):
kn = 1e5, reference reduced mass m_eff = 1/2, t_c = pi sqrt(m_eff/kn),
dt = t_c/50, v_max = 2e-3 a / dt, gamma_n for a restitution coefficient of 0.9,
no gravity.  Method parameters: K = 200 (the paper's recommended default,
Sec. 5.4), cell size L_C = 1.7a, eps = 2e-6 box units, cap mode 0.
Every float parameter is rounded to float32 so that the FP32 and FP64 paths see
identical values.
"""
from dataclasses import dataclass, field

import numpy as np


def _f32(x: float) -> float:
    return float(np.float32(x))


def physics_constants(a: float, restitution: float = 0.9, kn: float = 1e5,
                      m_eff: float = 0.5, dt_frac: float = 1.0 / 50.0) -> dict:
    """Contact-law and time-step constants for lattice spacing a."""
    omega0 = np.sqrt(kn / m_eff)
    t_c = np.pi / omega0
    dt = t_c * dt_frac
    ln_e = np.log(restitution)
    zeta = -ln_e / np.sqrt(np.pi ** 2 + ln_e ** 2)
    gamma_n = 2.0 * zeta * np.sqrt(m_eff * kn)
    return {"kn": _f32(kn), "gamma_n": _f32(gamma_n), "dt": _f32(dt),
            "v_max": _f32(2e-3 * a / dt)}


@dataclass
class ParticleSystem:
    """One particle system: float32 arrays in the caller's (original) order."""
    pos_r: np.ndarray          # [N,4] float32: x, y, z, R_C
    vel_m: np.ndarray          # [N,4] float32: vx, vy, vz, 1/m
    params: dict               # method and physical parameters (float32-exact values)
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos_r.shape[0])


def _unit_vector(rng) -> np.ndarray:
    while True:
        u = rng.normal(size=3)
        nrm = np.linalg.norm(u)
        if nrm > 1e-12:
            return u / nrm


def lattice_system(nx: int, ny: int, nz: int, n_boxes: int, n_balls: int, sigma: float,
                   seed: int, polydisperse: bool = False, K: float = 200.0,
                   cell_factor: float = 1.7, eps: float = 2e-6, skin_mode: int = 0,
                   cap_mode: int = 0, max_neighbors: int = 32,
                   gravity=(0.0, 0.0, 0.0)) -> ParticleSystem:
    rng = np.random.Generator(np.random.PCG64(seed))
    a = 1.0 / (max(nx, ny, nz) + 1)
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    # lattice order: x fastest, then y, then z
    idx = np.stack([ii.transpose(2, 1, 0).ravel(), jj.transpose(2, 1, 0).ravel(),
                    kk.transpose(2, 1, 0).ravel()], axis=1)
    n = idx.shape[0]
    pos = (idx + 1.0) * a + rng.uniform(-0.04 * a, 0.04 * a, size=(n, 3))
    if polydisperse:
        rad = rng.uniform(0.35 * a, 0.45 * a, size=n)
    else:
        rad = np.full(n, 0.45 * a)
    mass = (rad / (0.45 * a)) ** 3
    phys = physics_constants(a)
    v_max = phys["v_max"]
    # velocity field painted on the lattice grid, indexed [k, j, i] (z, y, x)
    grid = np.zeros((nz, ny, nx, 3))
    dims = np.array([nx, ny, nz])
    for _ in range(n_boxes):
        lo = np.zeros(3, dtype=np.int64)
        hi = np.zeros(3, dtype=np.int64)
        for ax in range(3):
            L = int(rng.integers(max(1, dims[ax] // 10), max(2, (4 * dims[ax]) // 10) + 1))
            L = min(L, int(dims[ax]))
            s = int(rng.integers(0, dims[ax] - L + 1))
            lo[ax], hi[ax] = s, s + L
        speed = rng.uniform(0.0, 1.0) * v_max
        vv = speed * _unit_vector(rng)
        grid[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = vv
    for _ in range(n_balls):
        c = rng.uniform(0.0, 1.0, size=3) * dims
        r = rng.uniform(0.05, 0.2) * dims.max()
        speed = rng.uniform(0.0, 1.0) * v_max
        vv = speed * _unit_vector(rng)
        # sites with (index + 1/2 - c)^2 summed <= r^2, searched in the ball's bounding box
        b0 = np.maximum(np.floor(c - r - 1).astype(np.int64), 0)
        b1 = np.minimum(np.ceil(c + r + 1).astype(np.int64), dims)
        if np.any(b1 <= b0):
            continue
        gi = np.arange(b0[0], b1[0]) + 0.5 - c[0]
        gj = np.arange(b0[1], b1[1]) + 0.5 - c[1]
        gk = np.arange(b0[2], b1[2]) + 0.5 - c[2]
        inside = (gi[None, None, :] ** 2 + gj[None, :, None] ** 2) + gk[:, None, None] ** 2 <= r * r
        sub = grid[b0[2]:b1[2], b0[1]:b1[1], b0[0]:b1[0]]
        sub[inside] = vv
    vel = grid.reshape(n, 3)
    vel = vel + rng.normal(0.0, sigma * v_max, size=(n, 3))

    pos_r = np.empty((n, 4), dtype=np.float32)
    pos_r[:, :3] = pos
    pos_r[:, 3] = rad
    vel_m = np.empty((n, 4), dtype=np.float32)
    vel_m[:, :3] = vel
    vel_m[:, 3] = 1.0 / mass
    params = {
        "skin_mode": skin_mode, "cap_mode": cap_mode, "K": _f32(K), "dt": phys["dt"],
        "cell_size": _f32(cell_factor * a), "skin_uniform": _f32(0.45 * a), "eps": _f32(eps),
        "lo": (0.0, 0.0, 0.0),
        "hi": (_f32((nx + 1) * a), _f32((ny + 1) * a), _f32((nz + 1) * a)),
        "kn": phys["kn"], "gamma_n": phys["gamma_n"],
        "g": tuple(_f32(t) for t in gravity), "max_neighbors": max_neighbors,
        "fixed_interval": 1,
    }
    meta = {"a": a, "v_max": v_max, "lattice": (nx, ny, nz), "n_boxes": n_boxes,
            "n_balls": n_balls, "sigma": sigma, "seed": seed, "polydisperse": polydisperse}
    return ParticleSystem(pos_r, vel_m, params, meta)


def free_flight_system(n_side: int, speeds, seed: int, K: float, dt: float = 2.0 ** -10,
                       cell_size: float = 2.0 ** -3, radius: float = 2.0 ** -6) -> ParticleSystem:
    """Particles far apart on a coarse grid in a large box, each moving along one
    axis at a speed taken from `speeds` (exact binary fractions), no contacts and
    no walls within reach: the free-flight case whose rebuild cadence has a closed
    form.  Every value is a dyadic rational, exact in float32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = np.arange(n_side, dtype=np.float64)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    n = n_side ** 3
    spacing = 2.0 ** -2
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1) * spacing + 2.0 ** -1
    vel = np.zeros((n, 3))
    sp = np.asarray(speeds, dtype=np.float64)
    choice = rng.integers(0, len(sp), size=n)
    axis = rng.integers(0, 3, size=n)
    sign = rng.choice([-1.0, 1.0], size=n)
    vel[np.arange(n), axis] = sign * sp[choice]
    pos_r = np.zeros((n, 4), dtype=np.float32)
    pos_r[:, :3] = pos
    pos_r[:, 3] = radius
    vel_m = np.zeros((n, 4), dtype=np.float32)
    vel_m[:, :3] = vel
    vel_m[:, 3] = 1.0
    side = spacing * (n_side - 1) + 2 * 2.0 ** -1
    params = {
        "skin_mode": 0, "cap_mode": 0, "K": float(K), "dt": float(dt), "cell_size": cell_size,
        "skin_uniform": 0.0, "eps": 2.0 ** -17, "lo": (0.0, 0.0, 0.0), "hi": (side, side, side),
        "kn": 1.0, "gamma_n": 0.0, "g": (0.0, 0.0, 0.0), "max_neighbors": 32,
        "fixed_interval": 1,
    }
    return ParticleSystem(pos_r, vel_m, params, {"n_side": n_side})


# The workloads, restated from the image-grid configurations as particle systems
# (one pixel -> one particle, one iteration -> one time step):
#   M1: 32x32x16 = 16,384 particles, 8 boxes + 4 balls, sigma 0.05, 200 steps
#   M2: 256x256x64 = 4,194,304 particles, 64 boxes + 32 balls, sigma 0.1, 500 steps
#   M3: 64 systems of (sx/4)x(sy/4)x16 with sx, sy from {256,...,1024}, 5000 steps
#   M5: 16 systems of 512x512x64 = 16,777,216 particles each, 1000 steps
CONFIGS = {
    "M1": {"steps": 200},
    "M2": {"steps": 500},
    "M3": {"steps": 5000},
    "M5": {"steps": 1000},
}


STATIC_OVERLAP = 0.01  # largest static overlap under gravity, in units of the smallest R_C


def _gravity_for_depth(kn: float, depth: int, r_min: float, m_max: float = 1.0) -> float:
    """Gravity of the gravity-driven stand-ins: the largest under which a column of
    `depth` particles compresses its lowest contact by at most STATIC_OVERLAP
    times the smallest radius.  That contact carries at most the column's weight
    depth m_max g, which compresses a linear spring of stiffness kn by
    depth m_max g / kn (walls carrying part of the weight only lower it).  With
    dt = t_c / 50 fixed by the contact, this is the one free ratio of the
    contact law to gravity: a stiffer spring at the same dt is the same run in
    other units."""
    return STATIC_OVERLAP * r_min * kn / (depth * m_max)


def hopper_system(n_target: int, seed: int, alpha_deg: float = 30.0, outlet: int = 8,
                  polydisperse: bool = True, K: float = 200.0, cell_factor: float = 1.7,
                  eps: float = 2e-6, sigma: float = 0.05) -> ParticleSystem:
    """A wedge hopper (two planar walls at alpha from the vertical, extruded along
    y) holding about n_target particles on a jittered lattice, above an outlet
    slit `outlet` lattice spacings wide and a collection bin; gravity along -z.
    The walls act only above the outlet height, so particles leave through the
    slit.  A stand-in for the hopper discharge cases of Sec. 5.2, whose geometry
    is not published."""
    rng = np.random.Generator(np.random.PCG64(seed))
    tan_a = np.tan(np.radians(alpha_deg))
    side = max(8, int(round((n_target / 0.6) ** (1.0 / 3.0))))  # hopper top width and depth
    ny = side
    bin_h = 10                                                    # collection bin, in sites
    # fill the wedge layer by layer until n_target sites
    rows = []
    k = 0
    total = 0
    while total < n_target:
        half = 0.5 * outlet + k * tan_a                           # half width at layer k (sites)
        half = min(half, 0.5 * side)
        w = int(np.floor(2 * half - 1.0))                          # sites clear of both walls
        if w > 0:
            rows.append((k, w))
            total += w * ny
        k += 1
        if k > 100000:
            raise ValueError("hopper does not fill")
    nz = bin_h + k + 2
    nx = side + 2
    a = 1.0 / (max(nx, ny, nz) + 1)
    xc = 0.5 * (nx + 1) * a
    z_o = (bin_h + 1) * a
    pts = []
    for k, w in rows:
        xs = xc + (np.arange(w) - 0.5 * (w - 1)) * a
        ys = (np.arange(ny) + 1.0) * a
        X, Y = np.meshgrid(xs, ys, indexing="xy")
        Z = np.full_like(X, z_o + (k + 0.5) * a)
        pts.append(np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1))
    pos = np.concatenate(pts, axis=0)
    n = pos.shape[0]
    pos = pos + rng.uniform(-0.04 * a, 0.04 * a, size=(n, 3))
    rad = rng.uniform(0.35 * a, 0.45 * a, size=n) if polydisperse else np.full(n, 0.45 * a)
    mass = (rad / (0.45 * a)) ** 3
    phys = physics_constants(a)
    v_max = phys["v_max"]
    vel = rng.normal(0.0, sigma * v_max, size=(n, 3))
    # the tallest column: the box height in lattice sites (bin, fill, headroom)
    g0 = _gravity_for_depth(phys["kn"], nz, rad.min(), mass.max())
    ca, sa = np.cos(np.radians(alpha_deg)), np.sin(np.radians(alpha_deg))
    planes = [  # (n, d, z_min): left wall (normal to +x and up), right wall
        (_f32(ca), 0.0, _f32(sa), float(np.float32((xc - 0.5 * outlet * a) * ca + z_o * sa)), _f32(z_o)),
        (_f32(-ca), 0.0, _f32(sa), float(np.float32(-(xc + 0.5 * outlet * a) * ca + z_o * sa)), _f32(z_o)),
    ]
    # normals rounded to float32 stay unit length to ~1e-8: renormalise in FP64
    planes = [tuple(np.array(pl[:3]) / np.linalg.norm(pl[:3])) + pl[3:] for pl in planes]
    return _system(pos, rad, mass, vel, a, phys, (nx + 1) * a, (ny + 1) * a, (nz + 1) * a,
                   (0.0, 0.0, -g0), planes, K, cell_factor, eps,
                   {"kind": "hopper", "alpha_deg": alpha_deg, "outlet_sites": outlet,
                    "layers": k, "depth": nz, "seed": seed, "v_max": v_max, "a": a,
                    "static_overlap_bound": STATIC_OVERLAP * float(rad.min())})


def incline_system(n_target: int, seed: int, theta_deg: float = 25.0,
                   polydisperse: bool = True, K: float = 200.0, cell_factor: float = 1.7,
                   eps: float = 2e-6, sigma: float = 0.05) -> ParticleSystem:
    """A slab of about n_target particles resting on a frictionless floor with
    gravity tilted by theta about y (the frame of an inclined plane), so the
    slab flows along +x and piles up against the far wall.  A stand-in for the
    inclined-plane flow case of Sec. 5.2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nz = max(4, int(round((n_target / 8.0) ** (1.0 / 3.0))))
    nx = 4 * nz
    ny = max(1, int(round(n_target / (nx * nz))))
    lx = nx + nx // 2                                          # room to flow
    a = 1.0 / (max(lx, ny, 3 * nz) + 1)
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    pos = np.stack([i.transpose(2, 1, 0).ravel(), j.transpose(2, 1, 0).ravel(),
                    k.transpose(2, 1, 0).ravel()], axis=1)
    pos = (pos + 1.0) * a
    n = pos.shape[0]
    pos = pos + rng.uniform(-0.04 * a, 0.04 * a, size=(n, 3))
    rad = rng.uniform(0.35 * a, 0.45 * a, size=n) if polydisperse else np.full(n, 0.45 * a)
    mass = (rad / (0.45 * a)) ** 3
    phys = physics_constants(a)
    v_max = phys["v_max"]
    vel = rng.normal(0.0, sigma * v_max, size=(n, 3))
    th = np.radians(theta_deg)
    # the slab's weight along the floor normal, g cos(theta), bounded as for a column
    g0 = _gravity_for_depth(phys["kn"], nz, rad.min(), mass.max()) / np.cos(th)
    return _system(pos, rad, mass, vel, a, phys, (lx + 1) * a, (ny + 1) * a, (3 * nz + 1) * a,
                   (g0 * np.sin(th), 0.0, -g0 * np.cos(th)), [], K, cell_factor, eps,
                   {"kind": "incline", "theta_deg": theta_deg, "seed": seed, "v_max": v_max,
                    "a": a, "depth": nz, "static_overlap_bound": STATIC_OVERLAP * float(rad.min())})


def silo_system(n_target: int, seed: int, gap: int = 4, polydisperse: bool = True,
                K: float = 200.0, cell_factor: float = 1.7, eps: float = 2e-6,
                sigma: float = 0.05) -> ParticleSystem:
    """A vertical cylindrical silo (a cylinder wall of diameter s lattice spacings
    about the centre of a box twice as wide) holding about n_target particles on a
    jittered lattice, a column about twice as tall as it is wide, on the box
    floor; gravity along -z.  The cylinder acts only above `gap` spacings, so the
    grains discharge through the ring between the silo's lower edge and the floor
    and spread over the floor.  A stand-in for the silo and hopper discharge cases
    of Sec. 5.2, whose geometry is not published."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = max(6, int(round((2.0 * n_target / np.pi) ** (1.0 / 3.0))))  # diameter, in sites
    r_wall = 0.5 * s + 0.5                                             # wall radius, in sites
    nxy = 2 * s + 2                                                    # box width, in sites
    c = 0.5 * (nxy + 1)                                                # axis, in sites
    g = np.arange(nxy) + 1.0
    X, Y = np.meshgrid(g, g, indexing="xy")
    inside = np.hypot(X - c, Y - c) <= r_wall - 0.5                    # clear of the wall
    col = np.stack([X[inside], Y[inside]], axis=1)
    layers = max(2, int(np.ceil(n_target / len(col))))
    nz = layers + 2
    a = 1.0 / (max(nxy, nz) + 1)
    pos = np.concatenate([np.concatenate([col, np.full((len(col), 1), k + 1.0)], axis=1)
                          for k in range(layers)], axis=0) * a
    n = pos.shape[0]
    pos = pos + rng.uniform(-0.04 * a, 0.04 * a, size=(n, 3))
    rad = rng.uniform(0.35 * a, 0.45 * a, size=n) if polydisperse else np.full(n, 0.45 * a)
    mass = (rad / (0.45 * a)) ** 3
    phys = physics_constants(a)
    v_max = phys["v_max"]
    vel = rng.normal(0.0, sigma * v_max, size=(n, 3))
    g0 = _gravity_for_depth(phys["kn"], layers, rad.min(), mass.max())
    cylinders = [(float(np.float32(c * a)), float(np.float32(c * a)), float(np.float32(r_wall * a)),
                  float(np.float32((gap + 0.5) * a)))]
    sysm = _system(pos, rad, mass, vel, a, phys, (nxy + 1) * a, (nxy + 1) * a, (nz + 1) * a,
                   (0.0, 0.0, -g0), [], K, cell_factor, eps,
                   {"kind": "silo", "diameter_sites": s, "gap_sites": gap, "layers": layers,
                    "depth": layers, "seed": seed, "v_max": v_max, "a": a,
                    "static_overlap_bound": STATIC_OVERLAP * float(rad.min())})
    sysm.params["cylinders"] = cylinders
    return sysm


def _system(pos, rad, mass, vel, a, phys, hx, hy, hz, gravity, planes, K, cell_factor, eps, meta):
    n = pos.shape[0]
    pos_r = np.empty((n, 4), dtype=np.float32)
    pos_r[:, :3] = pos
    pos_r[:, 3] = rad
    vel_m = np.empty((n, 4), dtype=np.float32)
    vel_m[:, :3] = vel
    vel_m[:, 3] = 1.0 / mass
    params = {
        "skin_mode": 0, "cap_mode": 0, "K": _f32(K), "dt": phys["dt"],
        "cell_size": _f32(cell_factor * a), "skin_uniform": _f32(0.45 * a), "eps": _f32(eps),
        "lo": (0.0, 0.0, 0.0), "hi": (_f32(hx), _f32(hy), _f32(hz)),
        "kn": phys["kn"], "gamma_n": phys["gamma_n"],
        "g": tuple(_f32(t) for t in gravity), "max_neighbors": 32, "fixed_interval": 1,
        "planes": [tuple(float(t) for t in pl) for pl in planes],
    }
    return ParticleSystem(pos_r, vel_m, params, dict(meta))


def _lattice_args(name: str, seed: int, scale: float):
    """Arguments of lattice_system for every system of a named workload."""
    def sc(v):
        return max(2, int(round(v * scale)))

    if name == "M1":
        return [(sc(32), sc(32), sc(16), 8, 4, 0.05, seed)]
    if name == "M2":
        return [(sc(256), sc(256), sc(64), 64, 32, 0.1, seed)]
    if name == "M3":
        rng = np.random.Generator(np.random.PCG64(12345 + seed))
        sides = np.array([256, 384, 512, 768, 1024])
        out = []
        for b in range(64):
            sx, sy = rng.choice(sides, size=2)
            nx, ny, nz = sc(sx // 4), sc(sy // 4), sc(16)
            nb = nx * ny * nz
            B = int(round(8 * np.sqrt(nb / 16384.0)))
            D = int(np.ceil(B / 2))
            sigma = float(rng.uniform(0.02, 0.15))
            out.append((nx, ny, nz, B, D, sigma, 1000 + b + seed))
        return out
    if name == "M5":
        rng = np.random.Generator(np.random.PCG64(54321 + seed))
        return [(sc(512), sc(512), sc(64), 256, 128, float(rng.uniform(0.05, 0.2)), 2000 + b + seed)
                for b in range(16)]
    raise KeyError(name)


def _make(args):
    return lattice_system(*args)


def config_systems(name: str, seed: int = 0, scale: float = 1.0, workers: int = 1):
    """The list of systems of a named workload.  `scale` < 1 shrinks every lattice
    side (for tests); the shapes of the distributions are unchanged.  With
    workers > 1 the systems are generated in a process pool (same output: every
    system has its own seed)."""
    if name in ("H125", "H250", "H500"):
        n = int(round({"H125": 125000, "H250": 250000, "H500": 500000}[name] * scale ** 3))
        return [hopper_system(max(n, 200), 3000 + seed)]
    if name == "INCLINE":
        return [incline_system(max(int(round(250000 * scale ** 3)), 200), 4000 + seed)]
    if name == "SILO":
        return [silo_system(max(int(round(125000 * scale ** 3)), 200), 5000 + seed)]
    args = _lattice_args(name, seed, scale)
    if workers <= 1 or len(args) == 1:
        return [_make(a) for a in args]
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=min(workers, len(args))) as ex:
        return list(ex.map(_make, args))
