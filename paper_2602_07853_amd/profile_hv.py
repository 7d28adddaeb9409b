"""Driver for hardware-counter runs of the Hessian-vector product.

    rocprofv3 --pmc FETCH_SIZE -d OUT -- python3 -m paper_2602_07853_amd.profile_hv

Sets up one Newton system of the 128^3 stiff plastic workload (unload,
stretch reconstruction, FP32 tangent at vhat), runs a fixed number of Jacobi
PCG iterations (each one fused Hessian-vector product launch), then one
plain device-to-device copy of a known size whose counter readings calibrate
the byte counts.  Prints the sizes needed to interpret the counters.
"""
from __future__ import annotations

import json
import sys


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--copy-mib", type=int, default=512)
    a = ap.parse_args(argv)
    import torch
    from paper_2602_07853_amd import mpmlite, scenes
    sc = scenes.CONFIGS[a.config]()
    ctx = mpmlite.Context((sc.n,) * 3, sc.dx, sc.materials,
                          opts=dict(hv_precision=mpmlite.F32, newton_rtol=1e-6, pcg_rtol=1e-30,
                                    max_pcg=a.iters, pcg_check_every=a.iters))
    parts = mpmlite.particles_to_device(sc.particles)
    ctx.unload(parts, sc.dt, sc.gravity, sc.bcs, 0.0)
    ctx.reconstruct()
    ctx.build_tangent(None, mpmlite.F32)
    _, g = ctx.energy_grad(None, True)
    x, it, rel = ctx.pcg(-g)
    n = a.copy_mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    mi = ctx.export("mass_i")[:, 0]
    fixed = ctx.export("fixed")[:, 0]
    info = {"workload": sc.name, "pcg_iters": it, "copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n,
            "kernel_version": mpmlite.library().mpl_version().decode(),
            "active_cells": int(ctx.export("mass_c").gt(0).sum().item()),
            "active_nodes": int(mi.gt(0).sum().item()),
            "free_dofs": 3 * int((mi.gt(0) & fixed.eq(0)).sum().item())}
    print(json.dumps(info), flush=True)


if __name__ == "__main__":
    sys.exit(main())
