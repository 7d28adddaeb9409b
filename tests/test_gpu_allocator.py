"""Device-memory ownership at the boundary: a context created with
allocator callbacks (the binding's default passes PyTorch's caching
allocator) takes all of its grid scratch from them, so PyTorch owns the
memory, and steps bitwise like a context on hipMalloc."""
import pytest

torch = pytest.importorskip("torch")

from paper_2602_07853_amd import scenes

pytestmark = pytest.mark.gpu


def run(sc, torch_allocator):
    from paper_2602_07853_amd import mpmlite
    ctx = mpmlite.Context((sc.n,) * 3, sc.dx, sc.materials,
                          opts=dict(hv_precision=mpmlite.F32, newton_rtol=1e-8, pcg_rtol=1e-8),
                          torch_allocator=torch_allocator)
    parts = mpmlite.particles_to_device(sc.particles)
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    for k in range(2):
        ctx.step(parts, parts, sc.dt, sc.gravity, sc.bcs, k * sc.dt)
    torch.cuda.synchronize()
    m1 = torch.cuda.memory_allocated()
    return ctx, parts, m0, m1


def test_torch_allocator_owns_the_scratch_and_steps_bitwise():
    sc = scenes.small_block(n=16, lo=4, hi=12, strain=0.05, E=1e6, model=scenes.FIXED_COROTATED, seed=61)
    ctx_t, pt, m0t, m1t = run(sc, True)
    live = ctx_t.allocator.bytes_live
    print(f"[alloc] torch allocator: {live} bytes live in the library, memory_allocated "
          f"{m0t} -> {m1t}", flush=True)
    assert live > 1 << 20
    assert m1t - m0t >= live
    ctx_h, ph, m0h, m1h = run(sc, False)
    print(f"[alloc] hipMalloc context: memory_allocated {m0h} -> {m1h}", flush=True)
    assert m1h == m0h
    for k in ("x", "v", "F", "G"):
        assert torch.equal(pt[k], ph[k]), k
    before = torch.cuda.memory_allocated()
    ctx_t.close()
    torch.cuda.synchronize()
    after = torch.cuda.memory_allocated()
    print(f"[alloc] after destroy: memory_allocated {before} -> {after}", flush=True)
    assert before - after >= live
    assert ctx_t.allocator.bytes_live == 0
