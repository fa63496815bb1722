"""The margin of the step kernel's contact pre-test, checked on the CPU.

The step kernel filters each Verlet-list row on 8-byte coded positions before
the exact FP64 test of Eq. delta (Sec. 3.2): centres rounded to a grid of
2^19 - 1 steps over the box plus two cells on each side, radii replaced by an
upper bound rlo + c (rhi - rlo)/126, and a margin of 2.5 grid steps.  This
models that arithmetic in numpy (FP64 rounding of the centres, FP32 distance
and reach with fused multiply-adds) and checks that no pair at or inside
touching distance is rejected, in the worst case the margin is sized for: a
grid spanning only four cells and radii up to a whole cell.
"""
import numpy as np

QBITS = 19
QMAX = (1 << QBITS) - 1
MARGIN = 2.5


def f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32)


def fma32(a, b, c):
    # a*b is exact in FP64 for FP32 operands; one rounding of the sum to FP32
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def encode(x, r, qlo, qinv, rlo, rhi):
    t = (x - qlo) * qinv
    assert (t >= 0).all() and (t < QMAX).all()
    q = np.floor(t + 0.5).astype(np.int64)
    step = (f32(rhi) - f32(rlo)) * np.float32(1.0 / 126.0)
    if step > 0:
        c = np.ceil((f32(r) - f32(rlo)) / step).clip(0, 126).astype(np.int64)
        bound = fma32(f32(c), np.full_like(f32(c), step), np.full_like(f32(c), f32(rlo)))
        c = np.where(bound < f32(r), np.minimum(c + 1, 126), c)
    else:
        c = np.zeros(len(r), dtype=np.int64)
    return q, c, step


def pretest(qi, ri, qj, cj, qinv32, rlo, step, margin):
    d = (qi - qj).astype(np.float32)                      # exact: |d| < 2^19
    d2 = fma32(d[:, 0], d[:, 0], fma32(d[:, 1], d[:, 1], d[:, 2] * d[:, 2]))
    reach0 = fma32(f32(ri), np.full(len(ri), qinv32, np.float32), np.full(len(ri), margin, np.float32))
    rlo_q = np.float32(f32(rlo) * qinv32)
    step_q = np.float32(step * qinv32)
    reach = reach0 + fma32(f32(cj), np.full(len(cj), step_q), np.full(len(cj), rlo_q))
    return d2 <= reach * reach


def touching_pairs(rng, n, qlo, span, rmin, rmax):
    """Pairs just inside touching distance with both centres on the grid (a
    centre off it passes every pre-test and needs no check here)."""
    ri = f32(rng.uniform(rmin, rmax, n)).astype(np.float64)
    rj = f32(rng.uniform(rmin, rmax, n)).astype(np.float64)
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    xi = qlo + rng.uniform(0.0, span, size=(n, 3))
    xj = xi + (ri + rj)[:, None] * (1.0 - 1e-15) * u
    top = qlo + span * (1.0 - 1e-12)
    keep = ((xi >= qlo) & (xi < top) & (xj >= qlo) & (xj < top)).all(axis=1)
    return xi[keep], ri[keep], xj[keep], rj[keep]


def run_case(seed, L, box, rmin, rmax, margin=MARGIN, n=400_000):
    rng = np.random.default_rng(seed)
    lo, hi = np.zeros(3), np.array(box, dtype=np.float64)
    qlo = lo - 2 * L
    span = (hi - lo + 4 * L).max()
    qinv = QMAX / span
    qinv32 = np.float32(qinv)
    xi, ri, xj, rj = touching_pairs(rng, n, qlo, span, rmin, rmax)
    assert len(ri) > n // 10
    rall = np.concatenate([ri, rj])
    rlo, rhi = f32(rall.min()), f32(rall.max())
    qi, _, step = encode(xi, ri, qlo, qinv, rlo, rhi)
    qj, cj, _ = encode(xj, rj, qlo, qinv, rlo, rhi)
    return pretest(qi, ri, qj, cj, qinv32, rlo, step, margin)


def test_touching_pairs_pass_on_the_smallest_grid():
    # a box of zero extent beyond its four cells: each grid step is 4 L / 2^19,
    # and radii of up to a whole cell reach 2^18 steps
    ok = run_case(1, L=1.0, box=(1e-9, 1e-9, 1e-9), rmin=0.5, rmax=1.0)
    assert ok.all()


def test_touching_pairs_pass_on_a_workload_grid():
    ok = run_case(2, L=1.7 / 256, box=(1.0, 1.0, 0.25), rmin=0.35 / 256, rmax=0.45 / 256)
    assert ok.all()


def test_touching_pairs_pass_with_equal_radii():
    ok = run_case(3, L=0.02, box=(1.0, 1.0, 1.0), rmin=0.006, rmax=0.006)
    assert ok.all()


def test_a_margin_below_the_rounding_bound_rejects_contacts():
    # the rounding of two centres moves their difference by up to sqrt(3) steps:
    # a margin of one step lets the pre-test drop pairs that touch
    ok = run_case(4, L=0.02, box=(1.0, 1.0, 1.0), rmin=0.004, rmax=0.008, margin=1.0)
    assert not ok.all()


def test_worst_case_rounding_needs_sqrt3_steps():
    """Pairs along the (1,1,1) diagonal placed so that one centre rounds down
    and the other up by almost half a step on every axis: the coded distance
    exceeds the true one by almost sqrt(3) steps.  The kernel's margin keeps
    every such touching pair; 1.6 steps would drop them."""
    rng = np.random.default_rng(5)
    L, n = 0.02, 50_000
    qlo = -2 * L
    span = 1.0 + 4 * L
    qinv = QMAX / span
    delta = 1e-3                                   # fractional offsets, in grid steps
    k = rng.integers(1000, QMAX // 2, size=n).astype(np.float64)
    sep = rng.integers(50, 2000, size=n) + 2 * delta   # per-axis separation, in steps
    ti = k + 0.5 - delta                           # rounds down by 0.5 - delta
    tj = ti + sep                                  # fractional part 0.5 + delta: rounds up
    xi = qlo + np.repeat(ti[:, None], 3, axis=1) / qinv
    xj = qlo + np.repeat(tj[:, None], 3, axis=1) / qinv
    d = np.linalg.norm(xj - xi, axis=1)
    r = np.nextafter(f32(d / 2), np.float32(np.inf)).astype(np.float64)   # touching: 2r > d
    assert (2 * r > d).all()
    qi = np.floor((xi - qlo) * qinv + 0.5).astype(np.int64)
    qj = np.floor((xj - qlo) * qinv + 0.5).astype(np.int64)
    excess = np.linalg.norm(qj - qi, axis=1) - d * qinv
    assert excess.max() > 1.7                      # the construction reaches the bound
    for margin, keeps_all in ((MARGIN, True), (1.6, False)):
        # per-pair radius range of one: the radius code is exact (c = 0)
        ok = np.array([pretest(qi[m:m + 1], r[m:m + 1], qj[m:m + 1], np.zeros(1, np.int64),
                               np.float32(qinv), f32(r[m]), np.float32(0.0), margin)[0]
                       for m in range(0, n, 50)])
        assert ok.all() == keeps_all, margin
