"""GPU parity of the multigrid-preconditioned CG (precond =
MPL_PRECOND_MULTIGRID), called through the C-ABI, against the FP64 oracle
of the same V-cycle (oracle/multigrid.py) on the same seeded inputs.

Bars: coarse masses and fixed components exactly as the oracle's
(restriction of FP64 masses, so within rounding); coarse tangents and
diagonals within 1e-12 from the FP64 tangent and 1e-5 from the FP32 one
(which rounds every entry once and, with one material, stores the
factored form, 2e-6 per cell); one V-cycle within 1e-10 in FP64 and 1e-6
in FP32, where it chains about fifteen FP32 products and sweeps (measured
1.6e-15 and 9e-8); the damping of every level within 1e-9 (FP64) and 1e-6
(FP32) of the oracle's power iteration; solutions within 1e-10 of the oracle's
minimiser, as for Jacobi."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import multigrid as MG
from oracle import oracle as O
from paper_2602_07853_amd import mpmlite, scenes
from tests.parity_util import gpu_context, oracle_state, rel, slip_walls

pytestmark = pytest.mark.gpu

NU, NU_COARSE = 2, 4


def host(t):
    return t.detach().cpu().numpy()


def _scenes():
    return {
        # stiffness-to-mass ratio dt^2 E / (rho dx^2) = 100 on a 16^3 grid: 3 levels
        "stiff_block16": scenes.small_block(n=16, lo=4, hi=12, strain=0.05, model=scenes.FIXED_COROTATED,
                                            E=3.9e8, seed=51, gravity=(0.0, 0.0, 0.0)),
        # two materials: the FP32 tangent takes its layout per cell block; 2 levels
        "fcr_two_materials": scenes.small_block(n=12, lo=3, hi=9, strain=0.05, E=1e6,
                                                model=scenes.FIXED_COROTATED, n_mats=2, seed=12),
        # boundary nodes with every combination of fixed components; 2 levels
        "slip_walls": slip_walls(),
    }


SCENES = _scenes()


def unloaded(sc, precision, **opts):
    o = dict(precond=mpmlite.PRECOND_MULTIGRID, mg_smooth=NU, mg_coarse_sweeps=NU_COARSE)
    o.update(opts)
    ctx = gpu_context(sc, precision, **o)
    parts = mpmlite.particles_to_device(sc.particles)
    ctx.unload(parts, sc.dt, sc.gravity, sc.bcs, 0.0)
    ctx.reconstruct()
    return ctx


def oracle_levels(sc, ref, v):
    A, rc = O.tangent(ref["grid"], ref["mats"], sc.dt, ref["Vck"], ref["S"], v, project=True)
    assert rc == 0
    return MG.hierarchy(ref["grid"], ref["mc"], ref["mi"], ref["fixed"], A, max_levels=4), A


def state_at(sc, seed=61):
    ref = oracle_state(sc)
    rng = np.random.default_rng(seed)
    act = (ref["mi"] > 0)[:, None]
    v = ref["vhat"] + 0.2 * rng.normal(size=ref["vhat"].shape) * act
    return ref, v


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("name", sorted(SCENES))
def test_levels_match_oracle(name, precision):
    sc = SCENES[name]
    print(f"[multigrid] levels scene {name} precision {precision}", flush=True)
    ref, v = state_at(sc)
    levels, _ = oracle_levels(sc, ref, v)
    ctx = unloaded(sc, precision)
    ctx.build_tangent(torch.tensor(v, device="cuda"), precision)
    tol = 1e-12 if precision == 1 else 1e-5
    for l in range(1, len(levels)):
        lv = levels[l]
        m = host(ctx.mg_export(l, "mass"))
        assert rel(m, lv.mi) <= 1e-14
        fixed = host(ctx.mg_export(l, "fixed")).astype(np.uint8)
        has_mass = lv.mi > 0
        assert np.array_equal(fixed[has_mass], lv.fixed[has_mass])
        A = host(ctx.mg_export(l, "abar"))
        assert rel(A, lv.A) <= tol
        D = host(ctx.mg_export(l, "diag"))
        Dinv = np.where(lv.free, 1.0 / np.where(lv.free, lv.D, 1.0), 0.0)
        assert rel(D, Dinv) <= tol
        assert np.all(D[~lv.free] == 0.0)


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("name", sorted(SCENES))
def test_vcycle_matches_oracle(name, precision):
    sc = SCENES[name]
    print(f"[multigrid] cycle scene {name} precision {precision}", flush=True)
    ref, v = state_at(sc)
    levels, _ = oracle_levels(sc, ref, v)
    ctx = unloaded(sc, precision)
    ctx.build_tangent(torch.tensor(v, device="cuda"), precision)
    rng = np.random.default_rng(62)
    fr = levels[0].free
    for k in range(2):
        r = rng.normal(size=fr.shape) * fr
        z, nlev, omega = ctx.mg_apply(torch.tensor(r, device="cuda"))
        assert nlev == len(levels)
        om_ref = [lv.omega for lv in levels]
        assert np.allclose(omega, om_ref, rtol=1e-9 if precision == 1 else 1e-6, atol=0)
        z_ref = MG.vcycle(levels, r, nu=NU, nu_coarse=NU_COARSE)
        e = rel(host(z), z_ref)
        print(f"  cycle {k}: levels {nlev} omega {omega} rel err {e:.2e}", flush=True)
        assert e <= (1e-10 if precision == 1 else 1e-6)
        assert np.all(host(z)[~fr] == 0.0)


def test_vcycle_is_symmetric_on_the_gpu():
    sc = SCENES["stiff_block16"]
    ref, v = state_at(sc)
    ctx = unloaded(sc, 1)
    ctx.build_tangent(torch.tensor(v, device="cuda"), 1)
    fr = (ref["mi"] > 0)[:, None] & ~O.fixed_components(ref["fixed"])
    rng = np.random.default_rng(63)
    x = rng.normal(size=fr.shape) * fr
    y = rng.normal(size=fr.shape) * fr
    bx = host(ctx.mg_apply(torch.tensor(x, device="cuda"))[0])
    by = host(ctx.mg_apply(torch.tensor(y, device="cuda"))[0])
    assert abs(np.sum(bx * y) - np.sum(x * by)) <= 1e-12 * np.linalg.norm(bx) * np.linalg.norm(y)
    assert np.sum(bx * x) > 0.0


@pytest.mark.parametrize("precision", [1, 0])
def test_mg_pcg_matches_oracle(precision):
    sc = SCENES["stiff_block16"]
    ref, v = state_at(sc)
    levels, A = oracle_levels(sc, ref, v)
    fr = levels[0].free
    b = np.random.default_rng(64).normal(size=fr.shape) * fr
    rtol = 1e-10 if precision == 1 else 1e-6
    x_or, it_or, rel_or = MG.pcg(levels, b, rtol, nu=NU, nu_coarse=NU_COARSE)
    ctx = unloaded(sc, precision, pcg_rtol=rtol)
    ctx.build_tangent(torch.tensor(v, device="cuda"), precision)
    x, iters, relres = ctx.pcg(torch.tensor(b, device="cuda"))
    print(f"[multigrid] pcg precision {precision}: gpu {iters} iterations ({relres:.2e}), "
          f"oracle {it_or} ({rel_or:.2e})", flush=True)
    r = b - O.hv(ref["grid"], ref["mc"], ref["mi"], ref["fixed"], A, host(x))
    assert relres <= rtol
    if precision == 1:
        assert abs(iters - it_or) <= 1
        assert np.linalg.norm(r) <= 1e-9 * np.linalg.norm(b)
        assert rel(host(x), x_or) <= 1e-8
    else:
        # FP32 products: the true residual against the FP64 matrix
        assert np.linalg.norm(r) <= 2e-5 * np.linalg.norm(b)
        assert iters <= it_or + 3


@pytest.mark.parametrize("precision", [1, 0])
@pytest.mark.parametrize("name", ["fcr_two_materials", "slip_walls"])
def test_newton_with_multigrid_matches_oracle(name, precision):
    """GPU Newton with multigrid-preconditioned CG lands on the oracle's
    minimiser (the same v* as with Jacobi)."""
    sc = SCENES[name]
    ref = oracle_state(sc)
    args = (ref["grid"], ref["mats"], sc.dt, ref["mc"], ref["mi"], ref["vhat"], ref["fixed"], ref["Vck"],
            ref["S"])
    v_or, st_or, rc = O.solve(*args, O.SolverOpts(1e-12, 1e-12))
    assert rc == 0
    ctx = unloaded(sc, precision, newton_rtol=1e-12, pcg_rtol=1e-12 if precision == 1 else 1e-6)
    v, st = ctx.solve()
    print(f"[multigrid] newton {name} precision {precision} gpu {st['newton_iters']} / {st['pcg_iters']}, "
          f"oracle {st_or}", flush=True)
    assert st["g_norm"] <= 1e-12 * st["g0_norm"]
    assert rel(host(v), v_or) <= 1e-10


def test_steps_with_multigrid_match_jacobi_steps():
    """Three steps of a plastic scene under a moving plate with the Galerkin
    warm start: multigrid and Jacobi reach the same particles."""
    sc = scenes.small_block(n=16, lo=4, hi=12, model=scenes.FIXED_COROTATED, E=7e6, strain=0.0,
                            plastic=scenes.PLASTIC_VON_MISES, yield_stress=2e3, seed=52,
                            vel_std=0.05, gravity=(0.0, 0.0, 0.0))
    sc.bcs.append(dict(kind=scenes.BC_MOVING_BOX, lo=(-1.0, 12 * sc.dx, -1.0), hi=(2.0, 2.0, 2.0),
                       velocity=(0.0, -0.5, 0.0)))
    res = {}
    for pre in (mpmlite.PRECOND_JACOBI, mpmlite.PRECOND_MULTIGRID):
        ctx = gpu_context(sc, 0, newton_rtol=1e-12, pcg_rtol=1e-8, warm_start=4, precond=pre)
        dp = mpmlite.particles_to_device(sc.particles)
        its = []
        for k in range(3):
            out = {key: t.clone() for key, t in dp.items()}
            st = ctx.step(dp, out, sc.dt, sc.gravity, sc.bcs, k * sc.dt)
            its.append(st["pcg_iters"])
            dp = out
        res[pre] = ({key: host(t) for key, t in dp.items()}, its)
    (pj, itj), (pm, itm) = res[mpmlite.PRECOND_JACOBI], res[mpmlite.PRECOND_MULTIGRID]
    print(f"[multigrid] steps: jacobi CG {itj}, multigrid CG {itm}", flush=True)
    for key in ("x", "v", "F"):
        assert rel(pm[key], pj[key]) <= (1e-12 if key == "x" else 1e-6)


@pytest.mark.parametrize("case", ["one_level", "two_levels"])
def test_level_counts_match_oracle(case):
    """A 4^3-cell grid has no coarser level (the cycle is the coarsest
    level's sweeps alone); mg_levels = 2 stops the 16^3 hierarchy after one
    coarsening.  Both against the oracle's cycle, FP64."""
    if case == "one_level":
        sc = scenes.small_block(n=4, lo=1, hi=3, strain=0.05, model=scenes.FIXED_COROTATED, E=1e6, seed=53)
        opts, max_levels = {}, 4
    else:
        sc = SCENES["stiff_block16"]
        opts, max_levels = dict(mg_levels=2), 2
    ref, v = state_at(sc)
    A, _ = O.tangent(ref["grid"], ref["mats"], sc.dt, ref["Vck"], ref["S"], v, project=True)
    levels = MG.hierarchy(ref["grid"], ref["mc"], ref["mi"], ref["fixed"], A, max_levels=max_levels)
    ctx = unloaded(sc, 1, **opts)
    ctx.build_tangent(torch.tensor(v, device="cuda"), 1)
    fr = levels[0].free
    assert fr.any()
    r = np.random.default_rng(65).normal(size=fr.shape) * fr
    z, nlev, omega = ctx.mg_apply(torch.tensor(r, device="cuda"))
    print(f"[multigrid] {case}: levels {nlev} omega {omega}", flush=True)
    assert nlev == len(levels) == (1 if case == "one_level" else 2)
    assert rel(host(z), MG.vcycle(levels, r, nu=NU, nu_coarse=NU_COARSE)) <= 1e-10


def test_multigrid_entry_point_errors():
    sc = SCENES["fcr_two_materials"]
    ctx = unloaded(sc, 1)
    nn = (sc.n + 1) ** 3
    r = torch.zeros((nn, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError, match="STATE"):
        ctx.mg_apply(r)                      # no tangent yet
    ref = oracle_state(sc)
    ctx.build_tangent(torch.tensor(ref["vhat"], device="cuda"), 1)
    z, nlev, _ = ctx.mg_apply(r)             # a zero residual gives a zero correction
    assert nlev == 2 and float(z.abs().max()) == 0.0
    for level in (0, nlev):
        with pytest.raises(RuntimeError, match="INVALID_ARG"):
            ctx.mg_export(level, "mass")
    good = dict(mg_levels=0, mg_omega=0.0, mg_smooth=NU)
    for bad in (dict(mg_levels=1), dict(mg_levels=7), dict(mg_omega=2.0), dict(mg_smooth=-1)):
        with pytest.raises(RuntimeError, match="INVALID_ARG"):
            ctx.set_opts(**bad)
        ctx.set_opts(**good)
