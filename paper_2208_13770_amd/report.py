"""Reporting arithmetic of the paper's performance summary (Sec. 5.4)."""


def improvement(t_without: float, t_case: float) -> float:
    """Eq. impr: gain over the run without Verlet buffer, in percent."""
    return (t_without - t_case) / t_without * 100.0


def overhead_to_optimum(t_default: float, t_opt: float) -> float:
    """Overhead column of Tab. summary: the extra time of the default K over the
    optimum K, in percent of the default run's time (the denominator that
    reproduces the printed values)."""
    return (t_default - t_opt) / t_default * 100.0


def executed_fraction(n_rebuild_steps: int, n_steps: int) -> float:
    """Executed broad phases over the total number of steps, in percent (the
    quantity plotted against K in Sec. 5.4)."""
    return 100.0 * n_rebuild_steps / max(n_steps, 1)
