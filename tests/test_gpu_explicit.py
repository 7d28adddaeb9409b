"""GPU tests of the explicit branch of Integrate (Sec. 4 opening, Eq.
explicitforce) through the C-ABI: the nodal force and node update after the
unload, and whole explicit steps (unload, force, load), against the
oracle's explicit step on the same seeded inputs."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2602_07853_amd import scenes
from tests.parity_util import gpu_context, oracle_state, rel, small_scenes

pytestmark = pytest.mark.gpu

SCENES = small_scenes()


def host(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name", list(SCENES))
def test_integrate_explicit_matches_oracle(name):
    from paper_2602_07853_amd import mpmlite
    sc = SCENES[name]
    ref = oracle_state(sc)
    ctx = gpu_context(sc, 1)
    parts = mpmlite.particles_to_device(sc.particles)
    ctx.unload(parts, sc.dt, sc.gravity, sc.bcs, 0.0)
    v, f = ctx.integrate_explicit(want_force=True)
    fo = O.explicit_force(ref["grid"], ref["Vck"], ref["tauck"])
    act = ref["mi"] > 0
    fx = O.fixed_components(ref["fixed"]) & act[:, None]
    free = act[:, None] & ~fx
    vo = ref["vhat"].copy()
    vo[free] += sc.dt * fo[free] / np.broadcast_to(ref["mi"][:, None], fo.shape)[free]
    ef, ev = rel(host(f), np.where(act[:, None], fo, 0.0)), rel(host(v), vo)
    print(f"[explicit] {name}: force rel {ef:.2e}, velocity rel {ev:.2e}", flush=True)
    assert ef <= 1e-12
    assert ev <= 1e-12
    assert np.all(host(v)[~act] == 0.0)
    assert np.array_equal(host(v)[fx], ref["vhat"][fx])


def explicit_both(sc, nsteps):
    from paper_2602_07853_amd import mpmlite
    g, mats, bcs = O.grid_of(sc), O.materials_of(sc), O.bcs_of(sc)
    p = sc.particles
    ctx = gpu_context(sc, 1)
    dp = mpmlite.particles_to_device(p)
    t = 0.0
    for _ in range(nsteps):
        p, vnode, rc = O.step_explicit(g, mats, sc.dt, sc.gravity, bcs, t, p)
        assert rc == 0
        st = ctx.step_explicit(dp, dp, sc.dt, sc.gravity, sc.bcs, t)
        t += sc.dt
    return p, {k: host(v) for k, v in dp.items()}, st


@pytest.mark.parametrize("name", list(SCENES))
def test_explicit_steps_match_oracle(name):
    sc = SCENES[name]
    po, pg, st = explicit_both(sc, 3)
    print(f"[explicit] {name} 3 steps, stats {st}", flush=True)
    assert st["newton_iters"] == 0 and st["pcg_iters"] == 0
    for k in ("x", "v", "G", "F"):
        assert rel(pg[k], po[k]) <= 1e-10, k


def test_explicit_plastic_moving_plate():
    """Fixed-corotated + von Mises under a moving plate: the load's plastic
    projection and moving Dirichlet boxes over several explicit steps."""
    sc = scenes.small_block(n=12, lo=3, hi=9, model=scenes.FIXED_COROTATED, E=7e6, strain=0.0,
                            plastic=scenes.PLASTIC_VON_MISES, yield_stress=2e3, seed=32,
                            vel_std=0.05, gravity=(0.0, 0.0, 0.0), dt=2e-5)
    sc.bcs.append(dict(kind=scenes.BC_MOVING_BOX, lo=(-1.0, 9 * sc.dx, -1.0), hi=(2.0, 2.0, 2.0),
                       velocity=(0.0, -0.5, 0.0)))
    po, pg, st = explicit_both(sc, 4)
    print(f"[explicit] plastic plate max eps {np.abs(po['eps']).max():.3e}", flush=True)
    for k in ("x", "v", "G", "F"):
        assert rel(pg[k], po[k]) <= 1e-10, k
    assert rel(pg["plastic"], po["eps"]) <= 1e-8 or np.abs(po["eps"]).max() == 0


def test_jelly_falling_small_matches_oracle():
    """The explicit workload at 32^3 (two falling cubes over a slab), 5 steps."""
    sc = scenes.jelly_falling(n=32)
    po, pg, st = explicit_both(sc, 5)
    print(f"[explicit] jelly 32^3: {sc.n_particles} particles, stats {st}", flush=True)
    for k in ("x", "v", "G", "F"):
        assert rel(pg[k], po[k]) <= 1e-10, k


def test_explicit_step_is_deterministic():
    from paper_2602_07853_amd import mpmlite
    sc = SCENES["fcr_two_materials"]
    outs = []
    for _ in range(2):
        ctx = gpu_context(sc, 1)
        dp = mpmlite.particles_to_device(sc.particles)
        ctx.step_explicit(dp, dp, sc.dt, sc.gravity, sc.bcs, 0.0)
        outs.append({k: host(v) for k, v in dp.items()})
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k]), k


def test_integrate_explicit_needs_unload():
    from paper_2602_07853_amd import mpmlite
    sc = SCENES["nh_strained"]
    ctx = gpu_context(sc, 1)
    with pytest.raises(mpmlite.MplError):
        ctx.integrate_explicit()


def test_explicit_step_empty_particle_set():
    from paper_2602_07853_amd import mpmlite
    sc = scenes.small_block(n=8, lo=2, hi=3)
    p = {k: v[:0] for k, v in sc.particles.items()}
    dp = mpmlite.particles_to_device(p)
    for opts in (dict(), dict(vbd_sweeps=2), dict(plasticity=mpmlite.PLASTICITY_FIXED_POINT),
                 dict(transfer=mpmlite.TRANSFER_FLIP_PIC, flip_ratio=0.9)):
        ctx = gpu_context(sc, 0, **opts)
        st = ctx.step_explicit(dp, dp, sc.dt, sc.gravity, sc.bcs, 0.0)
        assert st["active_cells"] == 0
        st = ctx.step(dp, dp, sc.dt, sc.gravity, sc.bcs, 0.0)
        assert st["active_cells"] == 0 and st["pcg_iters"] == 0


def test_explicit_particle_outside_grid_is_rejected():
    from paper_2602_07853_amd import mpmlite
    sc = scenes.small_block(n=8, lo=2, hi=4)
    p = dict(sc.particles)
    p["x"] = p["x"].copy()
    p["x"][0] = [0.01, 0.5, 0.5]  # stencil would reach cell -1
    ctx = gpu_context(sc, 0)
    dp = mpmlite.particles_to_device(p)
    before = host(dp["x"]).copy()
    with pytest.raises(mpmlite.MplError) as e:
        ctx.step_explicit(dp, dp, sc.dt, sc.gravity, sc.bcs, 0.0)
    assert e.value.status == -7
    assert np.array_equal(host(dp["x"]), before)
