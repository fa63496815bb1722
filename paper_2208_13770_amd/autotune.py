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

A new K shapes the skins from the next broad phase on (Def. autoverlet: the list
in use stays valid until its own validity test fails).  A probe window shorter
than the rebuild interval would therefore mostly time the list built under an
earlier K.  Each probe window starts with a broad phase under its own K, so its
rows are the ones it measures; that broad phase is charged to every candidate
alike.  Exploitation windows keep the list they find.
"""
import time


def tune(run_window, total_steps, K0=200.0, factor=2.0, window=50, exploit=400,
         K_min=1.0, K_max=1e5):
    """Advance total_steps steps through run_window(K, steps, probe) -> seconds,
    choosing K as described above (probe is True for the windows that compare
    candidates, False for exploitation).  Returns (windows, K): the windows as a
    list of (K, steps, seconds) and the K the search settled on."""
    if total_steps < 0 or window < 1 or exploit < 1 or factor <= 1.0:
        raise ValueError("bad tuner parameters")
    log = []
    done = 0
    K = min(max(float(K0), K_min), K_max)

    def measure(k, steps, probe):
        t = float(run_window(k, steps, probe))
        log.append((k, steps, t))
        return t / steps

    while done < total_steps:
        costs = {}
        for k in (K, K / factor, K * factor):  # K first: a cut-short round still has it
            k = min(max(k, K_min), K_max)
            if k in costs or done >= total_steps:
                continue
            s = min(window, total_steps - done)
            costs[k] = measure(k, s, True)
            done += s
        if not costs:
            break
        best = min(costs, key=lambda k: (costs[k], k))
        if best == K and done < total_steps:
            s = min(exploit, total_steps - done)
            measure(K, s, False)
            done += s
        K = best
    return log, K


def window_runner(vb, ctx, timer=time.perf_counter, on_records=None):
    """run_window for tune() over context ctx: sets K, requests a broad phase for
    a probe window (so that the window runs on rows built under its own K), runs
    the steps and returns their wall time, the call's own synchronisation
    included.  on_records, if given, receives each window's step records."""
    def run_window(K, steps, probe=True):
        vb.vb_set_K(ctx, K)
        if probe:
            vb.vb_force_rebuild(ctx)
        t0 = timer()
        h = vb.vb_run(ctx, steps, want_history=on_records is not None)
        dt = timer() - t0
        if on_records is not None:
            on_records(h)
        return dt
    return run_window


def tuned_run(vb, ctx, total_steps, timer=time.perf_counter, **kw):
    """Run total_steps steps of context ctx with K chosen by tune(); returns
    (windows, K)."""
    return tune(window_runner(vb, ctx, timer), total_steps, **kw)
