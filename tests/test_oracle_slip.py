"""Pins of the oracle's frictionless walls (slip planes) by what the
mechanics fixes.  A constraint that fixes only the normal velocity
component exerts its reaction along the normal only, and the internal
forces of the Q1 mesh sum to zero (the corner gradients of every cell sum
to zero), while the transfers move momentum between particles and nodes
without loss (partition of unity and linear reproduction of the two-hop
weights).  So over one implicit step, a block sliding on a frictionless
floor under vertical gravity keeps its horizontal momentum up to the
solver tolerance; on a sticky floor it loses part of it; the floor nodes
have zero vertical and nonzero horizontal velocity."""
import numpy as np

from oracle import oracle as O
from paper_2602_07853_amd import scenes


def block_on_floor(kind, n=16, seed=8):
    dx = 1.0 / n
    rng = np.random.Generator(np.random.PCG64(seed))
    cells = scenes.box_cells((5, 2, 5), (11, 8, 11))
    x = scenes.fill_cells(cells, dx, 2, rng)
    mats = [scenes.material(scenes.NEOHOOKEAN, 1e5, 0.3)]
    p = scenes.make_particles(x, np.zeros(len(x), np.int32), mats, dx, 8)
    p["v"] = np.tile([0.4, 0.0, -0.3], (len(x), 1)) + rng.normal(0.0, 0.05, size=(len(x), 3))
    p["G"] = rng.normal(0.0, 0.5, size=(len(x), 9))
    big = 10.0
    normal = (0.0, 1.0, 0.0) if kind == O.BC_SLIP_PLANE else (0.0, 0.0, 0.0)
    bcs = [O.BC(kind, (-big, -big, -big), (big, 3 * dx, big), normal)]
    omats = [O.Material(m["model"], m["E"], m["nu"], m["plastic"], m["yield_stress"], m["friction_deg"])
             for m in mats]
    return O.Grid(n, dx), omats, bcs, p


def momentum(p):
    return np.sum(np.asarray(p["m"])[:, None] * np.asarray(p["v"]), axis=0)


def test_block_keeps_horizontal_momentum_on_a_frictionless_floor():
    g, mats, bcs, p = block_on_floor(O.BC_SLIP_PLANE)
    out, st, vnode, rc = O.step(g, mats, 1e-3, (0.0, -9.81, 0.0), bcs, 0.0, O.SolverOpts(1e-12, 1e-13), p)
    assert rc == 0
    p0, p1 = momentum(p), momentum(out)
    scale = np.linalg.norm(p0)
    print(f"[slip] momentum before {p0}, after {p1}")
    assert abs(p1[0] - p0[0]) <= 1e-9 * scale
    assert abs(p1[2] - p0[2]) <= 1e-9 * scale
    # the floor pushed back vertically: the change is not gravity alone
    grav = -9.81 * 1e-3 * np.sum(p["m"])
    assert abs((p1[1] - p0[1]) - grav) > 1e-3 * abs(grav)
    # on the constrained nodes the normal component is 0 and the tangential ones move
    u = O.unload(g, p, mats)
    fixed, _ = O.node_bcs(g, u["mi"], bcs, 0.0)
    on = (fixed == 2) & (u["mi"] > 0)
    assert on.sum() > 50 and np.all(fixed[u["mi"] > 0] & 5 == 0)
    assert np.all(vnode[on, 1] == 0.0)
    assert np.all(np.abs(vnode[on, 0]) > 0.1)


def test_sticky_floor_takes_horizontal_momentum():
    g, mats, bcs, p = block_on_floor(O.BC_STICKY_BOX)
    out, st, vnode, rc = O.step(g, mats, 1e-3, (0.0, -9.81, 0.0), bcs, 0.0, O.SolverOpts(1e-12, 1e-13), p)
    assert rc == 0
    p0, p1 = momentum(p), momentum(out)
    assert p1[0] < 0.99 * p0[0]
    assert p1[2] > 0.99 * p0[2]   # p0[2] < 0: the magnitude drops too
