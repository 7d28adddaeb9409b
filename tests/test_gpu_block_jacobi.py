"""GPU parity of the 3x3 nodal block-Jacobi preconditioner (precond =
MPL_PRECOND_BLOCK_JACOBI), called through the C-ABI, against the FP64 CPU
oracle on the same seeded inputs.

Bars: the inverted node blocks within 1e-10 relative from the FP64 tangent
and 1e-5 from the FP32 one (its stored entries round once, the inverse
keeps the blocks' small condition number); solutions within 1e-10 of the
oracle's minimiser, as for Jacobi."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2602_07853_amd import mpmlite, scenes
from tests.parity_util import gpu_context, oracle_state, rel, small_scenes

pytestmark = pytest.mark.gpu

SCENES = small_scenes()


def host(t):
    return t.detach().cpu().numpy()


def unloaded(sc, precision, **opts):
    ctx = gpu_context(sc, precision, precond=mpmlite.PRECOND_BLOCK_JACOBI, **opts)
    parts = mpmlite.particles_to_device(sc.particles)
    ctx.unload(parts, sc.dt, sc.gravity, sc.bcs, 0.0)
    ctx.reconstruct()
    return ctx


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("name", sorted(SCENES))
def test_node_blocks_match_oracle(name, precision):
    sc = SCENES[name]
    print(f"[block-jacobi] blocks scene {name} precision {precision}", flush=True)
    ref = oracle_state(sc)
    ctx = unloaded(sc, precision)
    rng = np.random.default_rng(41)
    act = (ref["mi"] > 0)[:, None]
    v = ref["vhat"] + 0.3 * rng.normal(size=ref["vhat"].shape) * act
    ctx.build_tangent(torch.tensor(v, device="cuda"), precision)
    B = host(ctx.export("block_diag")).reshape(-1, 3, 3)
    Ao, rc = O.tangent(ref["grid"], ref["mats"], sc.dt, ref["Vck"], ref["S"], v, project=True)
    assert rc == 0
    Bo, rc = O.block_jacobi(ref["grid"], ref["mc"], ref["mi"], ref["fixed"], Ao)
    assert rc == 0
    notdof = O.fixed_components(ref["fixed"]) | (ref["mi"] <= 0)[:, None]   # [nodes, 3]
    free = ~notdof.any(axis=1)   # nodes with every component free
    assert rel(B, Bo) <= (1e-10 if precision == 1 else 1e-5)
    # rows and columns of fixed components and massless nodes are 0
    assert np.all(B[notdof] == 0.0) and np.all(np.transpose(B, (0, 2, 1))[notdof] == 0.0)
    assert np.allclose(B, np.transpose(B, (0, 2, 1)), rtol=0, atol=0)
    # not a diagonal in disguise: the blocks couple the components
    off = np.abs(Bo[free] - Bo[free] * np.eye(3)).max() / np.abs(Bo[free]).max()
    assert off > 1e-4


def test_pcg_residual_with_block_jacobi():
    sc = SCENES["hencky_ragged"]
    ref = oracle_state(sc)
    ctx = unloaded(sc, 1, pcg_rtol=1e-10)
    v = ref["vhat"]
    ctx.build_tangent(torch.tensor(v, device="cuda"), 1)
    Ao, _ = O.tangent(ref["grid"], ref["mats"], sc.dt, ref["Vck"], ref["S"], v, project=True)
    free = (ref["mi"] > 0)[:, None] & ~O.fixed_components(ref["fixed"])
    b = np.random.default_rng(43).normal(size=v.shape) * free
    x, iters, relres = ctx.pcg(torch.tensor(b, device="cuda"))
    r = b - O.hv(ref["grid"], ref["mc"], ref["mi"], ref["fixed"], Ao, host(x))
    assert iters > 0 and relres <= 1e-10
    assert np.linalg.norm(r) <= 1e-9 * np.linalg.norm(b)


@pytest.mark.parametrize("precision", [1, 0])
def test_newton_with_block_jacobi_matches_oracle(precision):
    """GPU Newton with block-Jacobi CG lands on the oracle's block-Jacobi
    minimiser (the same v* as with Jacobi) to 1e-10."""
    sc = SCENES["fcr_two_materials"]
    ref = oracle_state(sc)
    args = (ref["grid"], ref["mats"], sc.dt, ref["mc"], ref["mi"], ref["vhat"], ref["fixed"], ref["Vck"],
            ref["S"])
    v_or, st_or, rc = O.solve(*args, O.SolverOpts(1e-12, 1e-12, block_jacobi=1))
    assert rc == 0
    ctx = unloaded(sc, precision, newton_rtol=1e-12, pcg_rtol=1e-12 if precision == 1 else 1e-6)
    v, st = ctx.solve()
    print(f"[block-jacobi] precision {precision} gpu {st} oracle {st_or}", flush=True)
    assert st["g_norm"] <= 1e-12 * st["g0_norm"]
    assert rel(host(v), v_or) <= 1e-10


@pytest.mark.parametrize("warm", [0, 1, 4])
def test_steps_with_block_jacobi_match_jacobi_steps(warm):
    """Three steps of a plastic scene under a moving plate (warm starts of
    the CG included): block-Jacobi and Jacobi reach the same particles."""
    sc = scenes.small_block(n=12, lo=3, hi=9, model=scenes.FIXED_COROTATED, E=7e6, strain=0.0,
                            plastic=scenes.PLASTIC_VON_MISES, yield_stress=2e3, seed=32,
                            vel_std=0.05, gravity=(0.0, 0.0, 0.0))
    sc.bcs.append(dict(kind=scenes.BC_MOVING_BOX, lo=(-1.0, 9 * sc.dx, -1.0), hi=(2.0, 2.0, 2.0),
                       velocity=(0.0, -0.5, 0.0)))
    res = {}
    for pre in (mpmlite.PRECOND_JACOBI, mpmlite.PRECOND_BLOCK_JACOBI):
        ctx = gpu_context(sc, 0, newton_rtol=1e-12, pcg_rtol=1e-8, warm_start=warm, precond=pre)
        dp = mpmlite.particles_to_device(sc.particles)
        its = []
        for k in range(3):
            st = ctx.step(dp, dp, sc.dt, sc.gravity, sc.bcs, k * sc.dt)
            its.append(st["pcg_iters"])
        res[pre] = {key: host(v) for key, v in dp.items()}
        print(f"[block-jacobi] warm_start={warm} precond={pre} pcg per step {its}", flush=True)
    for key in ("x", "v", "G", "F"):
        assert rel(res[1][key], res[0][key]) <= 1e-10, key


def test_block_jacobi_option_checks(monkeypatch):
    sc = SCENES["nh_strained"]
    ctx = gpu_context(sc, 1)
    parts = mpmlite.particles_to_device(sc.particles)
    ctx.unload(parts, sc.dt, sc.gravity, sc.bcs, 0.0)
    ctx.reconstruct()
    ref = oracle_state(sc)
    ctx.build_tangent(torch.tensor(ref["vhat"], device="cuda"), 1)
    # blocks are built with the tangent only when block-Jacobi is selected
    with pytest.raises(mpmlite.MplError, match="STATE"):
        ctx.export("block_diag")
    ctx.set_opts(precond=mpmlite.PRECOND_BLOCK_JACOBI)
    b = torch.zeros((ref["vhat"].shape[0], 3), dtype=torch.float64, device="cuda")
    with pytest.raises(mpmlite.MplError, match="STATE"):
        ctx.pcg(b)
    monkeypatch.setenv("MPL_CG_CLASSIC", "1")
    with pytest.raises(mpmlite.MplError, match="INVALID_ARG"):
        gpu_context(sc, 1, precond=mpmlite.PRECOND_BLOCK_JACOBI)
