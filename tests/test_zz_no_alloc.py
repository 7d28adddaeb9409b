"""The allocation-free Hessian-vector product (mpl_hv_noalloc) against the
allocating entry point (mpl_hv), through the C-ABI: the same kernels, so the
results must agree bitwise (stricter than the 1e-5 per-product bar of the
FP32 product).  Two calls in a row share the fixed scratch array, the second
on a smaller grid, so stale contents of the first call would show; a grid
whose buffers exceed the array is rejected with an error and leaves the
output untouched."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2602_07853_amd import scenes
from tests.parity_util import gpu_context

pytestmark = pytest.mark.gpu


def prepared(sc, precision):
    from paper_2602_07853_amd import mpmlite
    ctx = gpu_context(sc, precision)
    parts = mpmlite.particles_to_device(sc.particles)
    ctx.unload(parts, sc.dt, sc.gravity, sc.bcs, 0.0)
    ctx.reconstruct()
    ctx.build_tangent(None, precision)
    return ctx


def random_u(sc, dtype, seed):
    n1 = sc.n + 1
    u = np.random.default_rng(seed).normal(size=(n1 ** 3, 3))
    return torch.tensor(u, dtype=dtype, device="cuda")


def compare(ctx, sc, precision, seed):
    from paper_2602_07853_amd import mpmlite
    dt = torch.float32 if precision == mpmlite.F32 else torch.float64
    u = random_u(sc, dt, seed)
    ref = ctx.hv(u, precision)
    out = torch.full_like(ref, float("nan"))
    ctx.hv_noalloc(u, out, precision)
    torch.cuda.synchronize()
    same = torch.equal(out, ref)
    print(f"[no-alloc] {sc.name} precision {precision}: bitwise equal {same}, "
          f"|Hu| {float(ref.norm()):.6e}", flush=True)
    assert same


def test_noalloc_hv_matches_hv_on_two_calls():
    """Call 1 on the 128^3 one-million-cell workload (FP32, factored tangent,
    about 59 MiB of scratch), call 2 on the 16^3 scene (FP32, then FP64)."""
    from paper_2602_07853_amd import mpmlite
    big = scenes.config3()
    print(f"[no-alloc] {big.name}: {big.n_particles} particles", flush=True)
    ctx = prepared(big, mpmlite.F32)
    compare(ctx, big, mpmlite.F32, 1)
    small = scenes.config1()
    ctx_s = prepared(small, mpmlite.F32)
    compare(ctx_s, small, mpmlite.F32, 2)
    ctx_d = prepared(small, mpmlite.F64)
    compare(ctx_d, small, mpmlite.F64, 3)
    # the big grid again after the small ones: no leftovers of the small call
    compare(ctx, big, mpmlite.F32, 4)


def test_noalloc_hv_rejects_grids_beyond_its_scratch():
    """The 128^3 workload in FP64 needs about 118 MiB: rejected, output untouched."""
    from paper_2602_07853_amd import mpmlite
    big = scenes.config3()
    ctx = prepared(big, mpmlite.F64)
    u = random_u(big, torch.float64, 5)
    out = torch.full_like(u, 7.0)
    with pytest.raises(mpmlite.MplError) as ei:
        ctx.hv_noalloc(u, out, mpmlite.F64)
    print(f"[no-alloc] rejected: {ei.value}", flush=True)
    assert ei.value.status == -1
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
