"""Driver for profiling runs of the learned preconditioner's network.

    rocprofv3 --kernel-trace --stats -d OUT -- python3 -m paper_2602_07853_amd.profile_nn
    rocprofv3 --pmc SQ_INSTS_VALU_MFMA_MOPS_BF16 SQ_VALU_MFMA_BUSY_CYCLES GRBM_GUI_ACTIVE \\
        -d OUT -- python3 -m paper_2602_07853_amd.profile_nn

Runs the network forward a few times on the box the solver uses for a grid
of the given size (all grid nodes, each axis padded to a multiple of 8; 136^3
at 128^3), with He-initialised weights and a random input whose channels
5-15 are zero as in the solver.  Prints the box and the dense FLOP count of
one forward.
"""
from __future__ import annotations

import json
import sys


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args(argv)
    import torch
    from paper_2602_07853_amd import mpmlite, precond_train, scenes
    ctx = mpmlite.Context((a.n,) * 3, 1.0 / a.n, [scenes.material(scenes.NEOHOOKEAN, 1e5, 0.3)])
    ctx.precond_set_weights(precond_train.init_weights(0, out_scale=1.0))
    b = ((a.n + 1 + 7) // 8) * 8
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn((b, b, b, 16), dtype=torch.float32, device="cuda", generator=g)
    x[..., 5:] = 0
    for _ in range(a.reps):
        ctx.nn_forward(x)
    torch.cuda.synchronize()
    print(json.dumps({"box": [b, b, b], "reps": a.reps,
                      "flop_per_forward": precond_train.forward_flops((b, b, b))}), flush=True)


if __name__ == "__main__":
    sys.exit(main())
