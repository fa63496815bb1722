"""The K tuner's search (no GPU): on a synthetic cost per step with a known
optimum it settles on the closest K of its geometric grid, advances exactly the
requested steps, and never leaves the allowed range; driven through the binding's
calls, with K taking effect only at a broad phase as in the library, it still
finds the optimum."""
import math

import pytest

from paper_2208_13770_amd.autotune import tune, tuned_run


def model(k_opt):
    def run_window(K, steps, probe=True):  # seconds for `steps` steps at K
        return steps * (1.0 + math.log2(K / k_opt) ** 2)
    return run_window


class LaggingK:
    """Stands in for the library: vb_set_K shapes the skins from the next broad
    phase on, which runs when forced or after K steps (a free-flight cadence).
    Cost: C_BP per broad phase, 1 + K/100 per step (rows grow with K), so the
    cost per step C_BP/K + 1 + K/100 is least at K = sqrt(100 C_BP) = 63.2: on
    the tuner's grid 200, 100, 50, 25 the best point is 50."""
    C_BP = 40.0

    def __init__(self):
        self.K_set = self.K_used = 200.0
        self.since = 0
        self.force = False
        self.clock = 0.0
        self.rebuilds = 0

    def vb_set_K(self, ctx, K):
        self.K_set = K

    def vb_force_rebuild(self, ctx):
        self.force = True

    def vb_run(self, ctx, steps, want_history=False):
        for _ in range(steps):
            if self.force or self.since >= self.K_used:
                self.K_used, self.since, self.force = self.K_set, 0, False
                self.clock += self.C_BP
                self.rebuilds += 1
            self.clock += 1.0 + self.K_used / 100.0
            self.since += 1


def test_tuner_measures_each_k_on_its_own_rows():
    lib = LaggingK()
    log, K = tuned_run(lib, None, 4000, timer=lambda: lib.clock, window=50, exploit=400)
    assert K == 50.0
    assert sum(s for _, s, _ in log) == 4000
    assert sum(s for k, s, _ in log if k == K) > 2000


@pytest.mark.parametrize("k_opt,expect", [(137.0, 100.0), (900.0, 800.0), (30.0, 25.0)])
def test_tuner_settles_on_the_nearest_grid_point(k_opt, expect):
    log, K = tune(model(k_opt), 5000, K0=200.0, factor=2.0, window=50, exploit=400)
    assert sum(s for _, s, _ in log) == 5000
    assert K == pytest.approx(expect)
    # most steps run at the settled K
    assert sum(s for k, s, _ in log if k == K) > 2500


def test_tuner_respects_bounds_and_short_runs():
    log, K = tune(model(1e6), 1000, K0=200.0, K_max=1000.0)
    assert max(k for k, _, _ in log) <= 1000.0
    assert K == 1000.0
    log, K = tune(model(200.0), 30, window=50)
    assert sum(s for _, s, _ in log) == 30
    assert tune(model(200.0), 0) == ([], 200.0)


def test_tuner_rejects_bad_parameters():
    with pytest.raises(ValueError):
        tune(model(100.0), 10, factor=1.0)
