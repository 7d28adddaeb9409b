"""One small implicit step on cuda:0 through the C-ABI, checked against the
CPU oracle (the 16^3 split Neo-Hookean scene)."""
from __future__ import annotations

import numpy as np


def run() -> None:
    import torch
    from oracle import oracle as O
    from paper_2602_07853_amd import mpmlite, scenes

    if not torch.cuda.is_available():
        raise RuntimeError("smoke needs cuda:0")
    sc = scenes.config1()
    g, mats, bcs = O.grid_of(sc), O.materials_of(sc), O.bcs_of(sc)
    po, st_or, _, rc = O.step(g, mats, sc.dt, sc.gravity, bcs, 0.0,
                              O.SolverOpts(1e-11, 1e-11), sc.particles)
    assert rc == 0, rc
    ctx = mpmlite.Context((sc.n,) * 3, sc.dx, sc.materials,
                          opts=dict(hv_precision=mpmlite.F64, newton_rtol=1e-11, pcg_rtol=1e-11))
    dp = mpmlite.particles_to_device(sc.particles)
    st = ctx.step(dp, dp, sc.dt, sc.gravity, sc.bcs, 0.0)
    torch.cuda.synchronize()
    worst = 0.0
    for k in ("x", "v", "G", "F"):
        a = dp[k].cpu().numpy()
        r = np.linalg.norm(a - po[k]) / max(np.linalg.norm(po[k]), 1e-300)
        worst = max(worst, r)
    print(f"smoke: newton {st['newton_iters']} pcg {st['pcg_iters']} worst rel err {worst:.3e}",
          flush=True)
    if worst > 1e-10:
        raise AssertionError(f"GPU step differs from the oracle: {worst:.3e}")


if __name__ == "__main__":
    run()
