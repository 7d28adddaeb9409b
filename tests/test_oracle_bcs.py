"""Pin of the oracle's Dirichlet node sets (the reading of the boundary
conditions the paper leaves unspecified): sticky walls hold every node with
an index <= 1 or >= N-1 on some axis, a sticky floor holds the nodes with
y <= 3 dx, and a moving plate holds the nodes above its lower face, which
moves with the plate's velocity; box tests have a tolerance of 1e-6 dx, a
later box overrides an earlier one, and massless nodes are never fixed.
A slip plane fixes only the velocity component along its normal axis, to 0,
and leaves the other two free; a component stays fixed once any box fixes
it.  The expected sets are enumerated here node by node from that
statement, one bit per component (7: all three fixed)."""
import numpy as np

from oracle import oracle as O
from paper_2602_07853_amd import scenes


def _bcs(n, dx, plate_lo_j, v_plate):
    bcs = [O.BC(b["kind"], b["lo"], b["hi"], b["velocity"]) for b in scenes.wall_bcs(n, dx)]
    bcs.append(O.BC(scenes.BC_STICKY_BOX, (-10.0, -10.0, -10.0), (10.0, 3 * dx, 10.0)))
    bcs.append(O.BC(scenes.BC_MOVING_BOX, (-10.0, plate_lo_j * dx, -10.0), (10.0, 10.0, 10.0),
                    (0.0, v_plate, 0.0)))
    return bcs


def _expected(n, dx, mi, plate_lo_y, v_plate):
    fixed = np.zeros((n + 1,) * 3, dtype=np.uint8)
    vel = np.zeros((n + 1,) * 3 + (3,))
    for i in range(n + 1):
        for j in range(n + 1):
            for k in range(n + 1):
                if mi[i, j, k] == 0.0:
                    continue
                wall = min(i, j, k) <= 1 or max(i, j, k) >= n - 1
                floor = j <= 3
                plate = j * dx >= plate_lo_y - 1e-6 * dx
                if wall or floor or plate:
                    fixed[i, j, k] = 7
                if plate:  # the plate is the last box: its velocity wins
                    vel[i, j, k] = (0.0, v_plate, 0.0)
    return fixed.ravel(), vel.reshape(-1, 3)


def test_node_sets_enumerated_by_hand():
    n = 10
    dx = 1.0 / n
    g = O.Grid(n, dx)
    rng = np.random.default_rng(4)
    mi = (rng.uniform(size=(n + 1,) * 3) > 0.2).astype(np.float64)
    v = -0.2
    # the plate's lower face at j = 7 at time 0; after dt the face has moved
    # by v dt: half a cell (7 -> 6.5, no new row), a whole cell (row 6 joins,
    # exactly on the face, inside the 1e-6 dx tolerance), and a whole cell
    # minus 1e-5 dx (row 6 stays out: beyond the tolerance)
    for shift, t in ((0.0, 0.0), (0.5, 0.5 * dx / 0.2), (1.0, dx / 0.2), (1.0 - 1e-5, (1.0 - 1e-5) * dx / 0.2)):
        fixed, vfix = O.node_bcs(g, mi.ravel(), _bcs(n, dx, 7, v), t)
        ef, ev = _expected(n, dx, mi, (7 - shift) * dx, v)
        assert np.array_equal(fixed, ef), shift
        assert np.allclose(vfix, ev, rtol=0, atol=1e-15), shift
    # the rows that the statement fixes, counted directly on a full-mass grid
    mi1 = np.ones((n + 1,) * 3)
    fixed, vfix = O.node_bcs(g, mi1.ravel(), _bcs(n, dx, 7, v), 0.0)
    f = fixed.reshape((n + 1,) * 3)
    interior_free = [(i, j, k) for i in range(2, n - 1) for j in range(4, 7) for k in range(2, n - 1)]
    assert int((f == 0).sum()) == len(interior_free) == 7 * 3 * 7
    for (i, j, k) in interior_free:
        assert f[i, j, k] == 0
    assert np.all(vfix.reshape((n + 1,) * 3 + (3,))[:, 7:, :, 1] == v)
    assert np.all(vfix.reshape((n + 1,) * 3 + (3,))[:, :7, :, :] == 0.0)


def test_slip_planes_fix_the_normal_component_only():
    """A frictionless floor (normal +y) over the whole grid at y <= 2 dx and a
    frictionless side wall (normal -x) at x >= 8 dx, plus a sticky box in one
    corner: bit 1 on the floor, bit 0 on the wall, both on their edge, all
    three in the sticky box, none elsewhere; prescribed values 0."""
    n = 10
    dx = 1.0 / n
    g = O.Grid(n, dx)
    rng = np.random.default_rng(6)
    mi = (rng.uniform(size=(n + 1,) * 3) > 0.2).astype(np.float64)
    bcs = [O.BC(O.BC_SLIP_PLANE, (-10.0, -10.0, -10.0), (10.0, 2 * dx, 10.0), (0.0, 1.0, 0.0)),
           O.BC(O.BC_SLIP_PLANE, (8 * dx, -10.0, -10.0), (10.0, 10.0, 10.0), (-1.0, 0.0, 0.0)),
           O.BC(O.BC_STICKY_BOX, (-10.0, -10.0, -10.0), (1 * dx, 10.0, 1 * dx))]
    fixed, vfix = O.node_bcs(g, mi.ravel(), bcs, 0.3)
    f = fixed.reshape((n + 1,) * 3)
    for i in range(n + 1):
        for j in range(n + 1):
            for k in range(n + 1):
                want = 0
                if mi[i, j, k] != 0.0:
                    if j <= 2:
                        want |= 2
                    if i >= 8:
                        want |= 1
                    if i <= 1 and k <= 1:
                        want = 7
                assert f[i, j, k] == want, (i, j, k, f[i, j, k], want)
    assert np.all(vfix == 0.0)
    fc = O.fixed_components(fixed)
    assert fc.shape == (fixed.size, 3)
    assert np.array_equal(fc[:, 1], (fixed & 2) > 0)


def test_slip_plane_normal_must_name_one_axis():
    n = 4
    g = O.Grid(n, 1.0 / n)
    mi = np.ones((n + 1) ** 3)
    for normal in ((0.0, 0.0, 0.0), (1.0, 1.0, 0.0)):
        bcs = [O.BC(O.BC_SLIP_PLANE, (-1.0, -1.0, -1.0), (2.0, 0.1, 2.0), normal)]
        try:
            O.node_bcs(g, mi, bcs, 0.0)
        except ValueError:
            continue
        raise AssertionError(f"normal {normal} accepted")
