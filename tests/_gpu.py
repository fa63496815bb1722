"""Helpers of the GPU tests: run synthetic systems through the C ABI."""
import sys

import numpy as np

import paper_2208_13770_amd as vb


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def host_arrays(systems):
    pos = np.concatenate([s.pos_r for s in systems], axis=0)
    vel = np.concatenate([s.vel_m for s in systems], axis=0)
    return (pos[:, :3].astype(np.float64), vel[:, :3].astype(np.float64),
            pos[:, 3].astype(np.float64), vel[:, 3].astype(np.float64))


class GpuSession:
    """One context over a list of systems (a batch when more than one)."""

    def __init__(self, systems, overrides=None):
        import torch
        self.torch = torch
        self.systems = systems
        ov = overrides or {}
        self.params = [dict(s.params, **ov) for s in systems]
        self.ctx = vb.vb_batch_create(self.params, [s.n for s in systems])
        self.x, self.v, self.rc, self.invm = vb.state_tensors(systems)
        vb.vb_set_state(self.ctx, self.x, self.v, self.rc, self.invm)

    def run(self, steps):
        return vb.vb_run(self.ctx, steps)

    def state(self):
        xo = self.torch.empty_like(self.x)
        vo = self.torch.empty_like(self.v)
        half = vb.vb_get_state(self.ctx, xo, vo)
        return xo.cpu().numpy(), vo.cpu().numpy(), half

    def pairs(self, sys, which):
        n = vb.vb_get_pairs(self.ctx, sys, which)
        t = self.torch
        p = t.empty((max(n, 1), 2), dtype=t.int32, device="cuda")
        d = t.empty((max(n, 1),), dtype=t.float64, device="cuda")
        m = vb.vb_get_pairs(self.ctx, sys, which, p, d)
        assert m == n
        return p[:n].cpu().numpy(), d[:n].cpu().numpy()

    def info(self):
        return vb.vb_get_info(self.ctx)

    def close(self):
        if self.ctx is not None:
            vb.vb_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def gpu_trajectory(systems, steps, **overrides):
    with GpuSession(systems, overrides) as g:
        hist = g.run(steps)
        x, v, half = g.state()
    return x, v, hist


def oracle_digest(args, steps):
    """The oracle on one lattice system, built from its generator arguments in the
    calling process (a worker of a process pool): SHA-256 of its final FP64
    positions and velocities, and its contact and broad-phase records."""
    import hashlib

    import oracle
    import synth
    s = synth.lattice_system(*args)
    x, v, rc, invm = host_arrays([s])
    xo, vo, ho, _ = oracle.run(s.params, x, v, rc, invm, steps)
    return (hashlib.sha256(xo.tobytes()).hexdigest(), hashlib.sha256(vo.tobytes()).hexdigest(),
            ho["contacts"].copy(), ho["rebuilt"].copy())
