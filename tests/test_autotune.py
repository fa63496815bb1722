"""The K tuner's search (no GPU): on a synthetic cost per step with a known
optimum it settles on the closest K of its geometric grid, advances exactly the
requested steps, and never leaves the allowed range."""
import math

import pytest

from paper_2208_13770_amd.autotune import tune


def model(k_opt):
    def run_window(K, steps):  # seconds for `steps` steps at K
        return steps * (1.0 + math.log2(K / k_opt) ** 2)
    return run_window


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
