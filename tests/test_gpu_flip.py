"""GPU tests of the FLIP/PIC degradation of the transfers (Sec. 3,
Degradation to FLIP/PIC) through the C-ABI: whole implicit and explicit steps
against the oracle's FLIP/PIC step on the same seeded inputs."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2602_07853_amd import scenes
from tests.parity_util import gpu_context, rel, small_scenes

pytestmark = pytest.mark.gpu

SCENES = small_scenes()


def host(t):
    return t.detach().cpu().numpy()


def flip_both(sc, flip, nsteps, implicit, precision=1, rtol=1e-11):
    from paper_2602_07853_amd import mpmlite
    g, mats, bcs = O.grid_of(sc), O.materials_of(sc), O.bcs_of(sc)
    p = sc.particles
    ctx = gpu_context(sc, precision, newton_rtol=rtol, pcg_rtol=rtol if precision == 1 else 1e-6,
                      transfer=mpmlite.TRANSFER_FLIP_PIC, flip_ratio=flip)
    dp = mpmlite.particles_to_device(p)
    t = 0.0
    for _ in range(nsteps):
        opts = O.SolverOpts(rtol, rtol) if implicit else None
        p, _, rc = O.step_flip(g, mats, sc.dt, sc.gravity, bcs, t, p, flip, opts)
        assert rc == 0
        if implicit:
            ctx.step(dp, dp, sc.dt, sc.gravity, sc.bcs, t)
        else:
            ctx.step_explicit(dp, dp, sc.dt, sc.gravity, sc.bcs, t)
        t += sc.dt
    return p, {k: host(v) for k, v in dp.items()}


@pytest.mark.parametrize("name", ["fcr_two_materials", "water_block"])
@pytest.mark.parametrize("precision", [1, 0])
def test_flip_implicit_steps_match_oracle(name, precision):
    po, pg = flip_both(SCENES[name], 0.95, 2, True, precision)
    for k in ("x", "v", "G", "F"):
        e = rel(pg[k], po[k])
        print(f"[flip] implicit {name} precision {precision} {k} rel {e:.2e}", flush=True)
        assert e <= 1e-10, k


@pytest.mark.parametrize("flip", [0.0, 1.0])
def test_flip_explicit_steps_match_oracle(flip):
    po, pg = flip_both(SCENES["sand_water"], flip, 3, False)
    for k in ("x", "v", "G", "F"):
        assert rel(pg[k], po[k]) <= 1e-10, k


def test_flip_ratio_checked():
    from paper_2602_07853_amd import mpmlite
    sc = SCENES["nh_strained"]
    ctx = gpu_context(sc, 1)
    with pytest.raises(mpmlite.MplError):
        ctx.set_opts(transfer=mpmlite.TRANSFER_FLIP_PIC, flip_ratio=1.5)
    with pytest.raises(mpmlite.MplError):
        ctx.set_opts(transfer=7)
