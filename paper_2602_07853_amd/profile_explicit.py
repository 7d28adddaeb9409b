"""Driver for kernel-trace runs of the explicit branch of Integrate.

    rocprofv3 --kernel-trace --stats -d OUT -- python3 -m paper_2602_07853_amd.profile_explicit

Runs the jelly-falling workload (256^3 grid, about 1.1M particles, dt = 6e-5)
for a few untimed explicit steps and then ``--steps`` more, each step being
unload, nodal force and update, and load.  Prints the step rate and sizes.
"""
from __future__ import annotations

import json
import time


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    a = ap.parse_args(argv)
    import torch
    from paper_2602_07853_amd import mpmlite, scenes
    sc = scenes.jelly_falling()
    ctx = mpmlite.Context((sc.n,) * 3, sc.dx, sc.materials, opts=dict(hv_precision=mpmlite.F64))
    parts = mpmlite.particles_to_device(sc.particles)
    t = 0.0
    for _ in range(a.warmup):
        ctx.step_explicit(parts, parts, sc.dt, sc.gravity, sc.bcs, t)
        t += sc.dt
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        st = ctx.step_explicit(parts, parts, sc.dt, sc.gravity, sc.bcs, t)
        t += sc.dt
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    print(json.dumps({"workload": sc.name, "particles": sc.n_particles,
                      "active_cells": st["active_cells"], "active_nodes": st["active_nodes"],
                      "steps": a.steps, "ms_per_step": round(1e3 * el / a.steps, 4)}), flush=True)


if __name__ == "__main__":
    main()
