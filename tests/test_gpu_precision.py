"""FP32 against FP64 on the GPU over a trajectory: the 64^3 fixed-corotated
scene with the sinusoidal velocity field (884,736 particles), 10 implicit
steps at dt = 2e-3, once with the FP32 tangent and Hessian-vector product
(FP64 reductions, residual, energy and line search) and once with everything
in FP64.  Newton is driven to a relative gradient of 1e-8 in both, so the two
runs reach the same minimisers and the particle states agree to what the
solver tolerances leave; the differences are printed per field."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2602_07853_amd import scenes
from tests.parity_util import gpu_context, rel

pytestmark = pytest.mark.gpu


def run(sc, precision):
    from paper_2602_07853_amd import mpmlite
    ctx = gpu_context(sc, precision, newton_rtol=1e-8, pcg_rtol=1e-6, warm_start=1)
    dp = mpmlite.particles_to_device(sc.particles)
    stats = []
    for k in range(sc.steps):
        stats.append(ctx.step(dp, dp, sc.dt, sc.gravity, sc.bcs, k * sc.dt))
    return {k: v.detach().cpu().numpy() for k, v in dp.items()}, stats


def test_fp32_trajectory_matches_fp64_variant():
    sc = scenes.config2()
    assert sc.steps == 10
    p32, s32 = run(sc, 0)
    p64, s64 = run(sc, 1)
    print(f"[precision] {sc.name}: newton/pcg per step f32 "
          f"{[(s['newton_iters'], s['pcg_iters']) for s in s32]}", flush=True)
    print(f"[precision] f64 {[(s['newton_iters'], s['pcg_iters']) for s in s64]}", flush=True)
    errs = {k: rel(p32[k], p64[k]) for k in ("x", "v", "G", "F")}
    dx = np.abs(p32["x"] - p64["x"]).max() / sc.dx
    print(f"[precision] after {sc.steps} steps: rel err x {errs['x']:.2e} v {errs['v']:.2e} "
          f"G {errs['G']:.2e} F {errs['F']:.2e}; max |dx| {dx:.2e} cells", flush=True)
    for s in s32 + s64:
        assert s["g_norm"] <= 1e-8 * s["g0_norm"]
    # both runs end each step within 1e-8 of the same minimiser's gradient
    assert errs["x"] <= 1e-10
    assert errs["v"] <= 1e-6
    assert errs["G"] <= 1e-6
    assert errs["F"] <= 1e-9
    assert dx <= 1e-6
