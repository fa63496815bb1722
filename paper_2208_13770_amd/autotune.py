"""Runtime selection of the skin factor K from measured costs.

The optimum K depends on the case (Sec. 5.4, Tab. summary: from 50 to 1000 for
the paper's test cases) and drifts as the flow evolves. A small K rebuilds
often. A large K makes every row longer, so every step dearer. The theorem of
Sec. 4.2 makes the results independent of K, so K may change while the
simulation runs without changing any result. The tuner uses that freedom.

It runs the simulation in windows. Around the current K it measures the cost
per step of K, K/f and K*f, one window each, and moves to the cheapest. Once the
current K is the cheapest of the three, it runs a longer exploitation window at
that K and then probes again. Every step of every window is a real step of the
simulation.
"""
import time


def tune(run_window, total_steps, K0=200.0, factor=2.0, window=50, exploit=400,
         K_min=1.0, K_max=1e5):
    """Advance total_steps steps through run_window(K, steps) -> seconds, choosing K
    as described above.  Returns (windows, K): the windows as a list of
    (K, steps, seconds) and the K the search settled on."""
    if total_steps < 0 or window < 1 or exploit < 1 or factor <= 1.0:
        raise ValueError("bad tuner parameters")
    log = []
    done = 0
    K = min(max(float(K0), K_min), K_max)

    def measure(k, steps):
        t = float(run_window(k, steps))
        log.append((k, steps, t))
        return t / steps

    while done < total_steps:
        costs = {}
        for k in (K, K / factor, K * factor):  # K first: a cut-short round still has it
            k = min(max(k, K_min), K_max)
            if k in costs or done >= total_steps:
                continue
            s = min(window, total_steps - done)
            costs[k] = measure(k, s)
            done += s
        if not costs:
            break
        best = min(costs, key=lambda k: (costs[k], k))
        if best == K and done < total_steps:
            s = min(exploit, total_steps - done)
            measure(K, s)
            done += s
        K = best
    return log, K


def tuned_run(vb, ctx, total_steps, **kw):
    """Run total_steps steps of context ctx with K chosen by tune(); returns
    (windows, K).  Each window's wall time includes the call's own
    synchronisation."""
    def run_window(K, steps):
        vb.vb_set_K(ctx, K)
        t0 = time.perf_counter()
        vb.vb_run(ctx, steps, want_history=False)
        return time.perf_counter() - t0
    return tune(run_window, total_steps, **kw)

