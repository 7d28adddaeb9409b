"""Seeded synthetic scenes shaped like the paper's implicit workloads.

This module only draws inputs: particle positions, velocities, masses,
volumes, material ids, material parameters, boundary boxes and time steps.
It holds none of the method's arithmetic, so both the HIP path and the CPU
oracle may take their inputs from it.

Common recipe (unit cube, origin 0, ``dx = 1/N``):

* occupied cells are filled with ``ppc_axis^3`` particles per cell, one per
  sub-cell at a uniform random position inside the sub-cell (stratified
  jitter, NumPy PCG64 seeded per scene);
* ``F_p = I``, ``m_p = rho dx^3 / ppc``, ``V_p = dx^3 / ppc``;
* sticky walls: every node whose index is <= 1 or >= N-1 on some axis
  (``BC_SLIP_PLANE`` boxes, frictionless walls with their normal in
  ``velocity``, appear in the test scenes).

Material and model codes match ``include/mpmlite.h``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

NEOHOOKEAN, FIXED_COROTATED, HENCKY, WATER = 0, 1, 2, 3
PLASTIC_NONE, PLASTIC_VON_MISES, PLASTIC_DRUCKER_PRAGER = 0, 1, 2
BC_STICKY_BOX, BC_MOVING_BOX, BC_SLIP_PLANE = 0, 1, 2


@dataclass
class Scene:
    name: str
    n: int
    dx: float
    dt: float
    steps: int
    gravity: tuple
    materials: list          # dicts: model, plastic, E, nu, rho, yield_stress, friction_deg
    bcs: list                # dicts: kind, lo, hi, velocity
    particles: dict          # x, v, G, F, m, V, mat, eps
    newton_rtol: float = 1e-6
    pcg_rtol: float = 1e-6
    occupied_cells: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n_particles(self) -> int:
        return int(self.particles["m"].shape[0])


def material(model, E, nu, rho=1000.0, plastic=PLASTIC_NONE, yield_stress=0.0, friction_deg=0.0):
    return dict(model=model, plastic=plastic, E=float(E), nu=float(nu), rho=float(rho),
                yield_stress=float(yield_stress), friction_deg=float(friction_deg))


def wall_bcs(n: int, dx: float) -> list:
    """Sticky boxes holding every node with index <= 1 or >= n-1 on some axis."""
    out = []
    big = 10.0
    for a in range(3):
        lo = [-big] * 3
        hi = [big] * 3
        hi[a] = 1.0 * dx
        out.append(dict(kind=BC_STICKY_BOX, lo=tuple(lo), hi=tuple(hi), velocity=(0.0, 0.0, 0.0)))
        lo = [-big] * 3
        hi = [big] * 3
        lo[a] = (n - 1) * dx
        out.append(dict(kind=BC_STICKY_BOX, lo=tuple(lo), hi=tuple(hi), velocity=(0.0, 0.0, 0.0)))
    return out


def fill_cells(cells: np.ndarray, dx: float, ppc_axis: int, rng: np.random.Generator):
    """Stratified jitter: one particle per sub-cell of every occupied cell."""
    cells = np.asarray(cells, dtype=np.int64).reshape(-1, 3)
    s = np.stack(np.meshgrid(*[np.arange(ppc_axis)] * 3, indexing="ij"), -1).reshape(-1, 3)
    base = cells[:, None, :].astype(np.float64) + s[None, :, :] / ppc_axis
    jit = rng.random(base.shape) / ppc_axis
    return ((base + jit) * dx).reshape(-1, 3)


def make_particles(x, mat_ids, materials, dx, ppc):
    n = x.shape[0]
    rho = np.array([materials[k]["rho"] for k in range(len(materials))])[mat_ids]
    Vp = np.full(n, dx ** 3 / ppc)
    return dict(x=np.ascontiguousarray(x, dtype=np.float64), v=np.zeros((n, 3)),
                G=np.zeros((n, 9)), F=np.tile(np.eye(3).reshape(1, 9), (n, 1)),
                m=rho * Vp, V=Vp, mat=np.asarray(mat_ids, dtype=np.int32), eps=np.zeros(n))


def box_cells(lo, hi):
    g = np.stack(np.meshgrid(*[np.arange(l, h) for l, h in zip(lo, hi)], indexing="ij"), -1)
    return g.reshape(-1, 3)


# ---------------------------------------------------------------------------
def config1(seed: int = 1) -> Scene:
    """16^3, 8^3 occupied cells, split Neo-Hookean E=1e5 nu=0.3, gravity,
    v ~ N(0, 0.01^2), one step at dt = 1e-3, tolerances 1e-8."""
    n, dx = 16, 1.0 / 16
    rng = np.random.Generator(np.random.PCG64(seed))
    mats = [material(NEOHOOKEAN, 1e5, 0.3, 1000.0)]
    cells = box_cells((4, 4, 4), (12, 12, 12))
    x = fill_cells(cells, dx, 2, rng)
    p = make_particles(x, np.zeros(len(x), np.int32), mats, dx, 8)
    p["v"] = rng.normal(0.0, 0.01, size=(len(x), 3))
    return Scene("config1_nh_16", n, dx, 1e-3, 1, (0.0, -9.81, 0.0), mats, wall_bcs(n, dx), p,
                 newton_rtol=1e-8, pcg_rtol=1e-8, occupied_cells=len(cells))


def config2(seed: int = 2, n: int = 64, ppc_axis: int = 2) -> Scene:
    """64^3 grid, [8,56)^3 occupied, fixed-corotated E=1e6 nu=0.35, sinusoidal
    initial velocity (amplitude 0.5 m/s) with its analytic gradient as G_p,
    10 steps at dt = 2e-3, no gravity."""
    dx = 1.0 / n
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = n // 8, n - n // 8
    mats = [material(FIXED_COROTATED, 1e6, 0.35, 1000.0)]
    cells = box_cells((lo,) * 3, (hi,) * 3)
    x = fill_cells(cells, dx, ppc_axis, rng)
    p = make_particles(x, np.zeros(len(x), np.int32), mats, dx, ppc_axis ** 3)
    x0, L = lo * dx, (hi - lo) * dx
    xh = (x - x0) / L
    A, k = 0.5, 2.0 * math.pi
    p["v"] = A * np.stack([np.sin(k * xh[:, 1]), np.sin(k * xh[:, 2]), np.sin(k * xh[:, 0])], 1)
    G = np.zeros((len(x), 3, 3))
    G[:, 0, 1] = A * k / L * np.cos(k * xh[:, 1])
    G[:, 1, 2] = A * k / L * np.cos(k * xh[:, 2])
    G[:, 2, 0] = A * k / L * np.cos(k * xh[:, 0])
    p["G"] = G.reshape(-1, 9)
    return Scene(f"config2_fcr_{n}", n, dx, 2e-3, 10, (0.0, 0.0, 0.0), mats, wall_bcs(n, dx), p,
                 occupied_cells=len(cells))


def _union_mask(n, shapes, scale):
    c = (np.arange(n) + 0.5) / n
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    mask = np.zeros((n, n, n), dtype=bool)
    for s in shapes:
        if s[0] == "box":
            _, ctr, half = s
            h = np.asarray(half) * scale
            mask |= ((np.abs(X - ctr[0]) <= h[0]) & (np.abs(Y - ctr[1]) <= h[1]) &
                     (np.abs(Z - ctr[2]) <= h[2]))
        else:
            _, ctr, r = s
            mask |= (X - ctr[0]) ** 2 + (Y - ctr[1]) ** 2 + (Z - ctr[2]) ** 2 <= (r * scale) ** 2
    return mask


def config3(seed: int = 3, n: int = 128, target_cells: int = 1_000_000, ppc_axis: int = 2) -> Scene:
    """Stiff plastic solid: a seeded union of 6 boxes (sides U[0.15,0.45]) and
    6 spheres (r U[0.08,0.2]), centres in [0.2,0.8]^3, scaled until the
    occupied cell count is within 5% of ``target_cells``; fixed-corotated
    E=7e7 nu=0.3 with von Mises yield 1e5; resting on a sticky floor
    (nodes y <= 3 dx) and pressed by a plate (nodes above the top face)
    moving at (0, -0.2, 0) m/s; dt = 1e-3, 20 steps, no gravity."""
    dx = 1.0 / n
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = []
    for _ in range(6):
        ctr = rng.uniform(0.2, 0.8, 3)
        side = rng.uniform(0.15, 0.45, 3)
        shapes.append(("box", ctr, side / 2))
    for _ in range(6):
        ctr = rng.uniform(0.2, 0.8, 3)
        shapes.append(("sphere", ctr, rng.uniform(0.08, 0.2)))
    margin = 3  # keep the body inside cells [3, n-4]
    lo_s, hi_s = 0.2, 4.0
    mask = None
    for _ in range(60):
        s = 0.5 * (lo_s + hi_s)
        mask = _union_mask(n, shapes, s)
        mask[:margin] = mask[n - margin - 1:] = False
        mask[:, :margin] = mask[:, n - margin - 1:] = False
        mask[:, :, :margin] = mask[:, :, n - margin - 1:] = False
        cnt = int(mask.sum())
        if abs(cnt - target_cells) <= 0.05 * target_cells:
            break
        if cnt < target_cells:
            lo_s = s
        else:
            hi_s = s
    cells = np.argwhere(mask)
    # rest the body on the floor: lowest occupied row -> row `margin`
    jmin = cells[:, 1].min()
    cells[:, 1] += margin - jmin
    cells = cells[cells[:, 1] <= n - margin - 1]
    jmax = int(cells[:, 1].max())
    mats = [material(FIXED_COROTATED, 7e7, 0.3, 1000.0, PLASTIC_VON_MISES, 1e5)]
    x = fill_cells(cells, dx, ppc_axis, rng)
    p = make_particles(x, np.zeros(len(x), np.int32), mats, dx, ppc_axis ** 3)
    bcs = wall_bcs(n, dx)
    bcs.append(dict(kind=BC_STICKY_BOX, lo=(-10.0, -10.0, -10.0), hi=(10.0, margin * dx, 10.0),
                    velocity=(0.0, 0.0, 0.0)))
    bcs.append(dict(kind=BC_MOVING_BOX, lo=(-10.0, (jmax + 1) * dx, -10.0), hi=(10.0, 10.0, 10.0),
                    velocity=(0.0, -0.2, 0.0)))
    return Scene(f"config3_fcr_vm_{n}", n, dx, 1e-3, 20, (0.0, 0.0, 0.0), mats, bcs, p,
                 occupied_cells=len(cells), meta=dict(jmax=jmax))


def config5(seed: int = 5, n: int = 256, ppc_axis: int = 2) -> Scene:
    """Three seeded spheres (r in [0.24, 0.28], disjoint or touching) of split
    Neo-Hookean (E=1e5, nu=0.3), Hencky + Drucker-Prager sand (E=1e6, nu=0.3,
    30 deg, rho 2000) and near-incompressible jelly (split NH, E=1e5,
    nu=0.45) falling under gravity onto a sticky floor (nodes y <= 3 dx);
    dt = 2e-3, 50 steps."""
    dx = 1.0 / n
    rng = np.random.Generator(np.random.PCG64(seed))
    # Rejection sampling of three such spheres with uniform centres almost
    # never succeeds (they fill ~22% of the cube), so the candidates are
    # jittered corners of the cube of admissible centres, three corners that
    # differ in at least two coordinates (face or body diagonals apart),
    # redrawn until the spheres are disjoint or touching.
    corners = np.array([[(k >> 2) & 1, (k >> 1) & 1, k & 1] for k in range(8)], dtype=np.float64)
    spheres = []
    while len(spheres) < 3:
        spheres = []
        order = rng.permutation(8)
        picked = []
        for k in order:
            if all(np.abs(corners[k] - corners[j]).sum() >= 2 for j in picked):
                picked.append(k)
            if len(picked) == 3:
                break
        for k in picked:
            r = rng.uniform(0.24, 0.28)
            lo, hi = r + 4 * dx, 1 - r - 4 * dx
            ctr = lo + corners[k] * (hi - lo) + rng.uniform(-0.02, 0.02, 3)
            ctr = np.clip(ctr, lo, hi)
            if all(np.linalg.norm(ctr - c) >= r + rr for c, rr in spheres):
                spheres.append((ctr, r))
    c = (np.arange(n) + 0.5) * dx
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    owner = np.full((n, n, n), -1, np.int32)
    for k, (ctr, r) in enumerate(spheres):
        inside = (X - ctr[0]) ** 2 + (Y - ctr[1]) ** 2 + (Z - ctr[2]) ** 2 <= r * r
        owner[inside & (owner < 0)] = k
    cells = np.argwhere(owner >= 0)
    mat_cell = owner[cells[:, 0], cells[:, 1], cells[:, 2]]
    mats = [material(NEOHOOKEAN, 1e5, 0.3, 1000.0),
            material(HENCKY, 1e6, 0.3, 2000.0, PLASTIC_DRUCKER_PRAGER, 0.0, 30.0),
            material(NEOHOOKEAN, 1e5, 0.45, 1000.0)]
    x = fill_cells(cells, dx, ppc_axis, rng)
    ids = np.repeat(mat_cell, ppc_axis ** 3).astype(np.int32)
    p = make_particles(x, ids, mats, dx, ppc_axis ** 3)
    bcs = wall_bcs(n, dx)
    bcs.append(dict(kind=BC_STICKY_BOX, lo=(-10.0, -10.0, -10.0), hi=(10.0, 3 * dx, 10.0),
                    velocity=(0.0, 0.0, 0.0)))
    return Scene(f"config5_mixed_{n}", n, dx, 2e-3, 50, (0.0, -9.81, 0.0), mats, bcs, p,
                 occupied_cells=len(cells))


def small_block(n=8, lo=2, hi=6, model=NEOHOOKEAN, E=1e5, nu=0.3, seed=11, vel_std=0.05,
                strain=0.0, ppc_axis=2, plastic=PLASTIC_NONE, yield_stress=0.0,
                friction_deg=0.0, n_mats=1, gravity=(0.0, -9.81, 0.0), dt=1e-3) -> Scene:
    """Small test scene: a block of occupied cells with random velocities,
    random affine G_p and (optionally) random pre-strained F_p = I + strain*N(0,1)
    with det F_p > 0; with ``n_mats`` > 1 material ids alternate by cell."""
    dx = 1.0 / n
    rng = np.random.Generator(np.random.PCG64(seed))
    models = [model, FIXED_COROTATED, NEOHOOKEAN][:n_mats]
    mats = [material(models[k], E * (1 + k), nu, 1000.0 * (1 + 0.5 * k), plastic, yield_stress,
                     friction_deg) for k in range(n_mats)]
    cells = box_cells((lo,) * 3, (hi,) * 3)
    x = fill_cells(cells, dx, ppc_axis, rng)
    ppc = ppc_axis ** 3
    ids = (np.repeat(np.arange(len(cells)) % n_mats, ppc)).astype(np.int32)
    p = make_particles(x, ids, mats, dx, ppc)
    p["v"] = rng.normal(0.0, vel_std, size=(len(x), 3))
    p["G"] = rng.normal(0.0, vel_std / dx * 0.1, size=(len(x), 9))
    if strain > 0:
        F = np.eye(3)[None] + strain * rng.normal(size=(len(x), 3, 3))
        bad = np.linalg.det(F) <= 0.2
        F[bad] = np.eye(3)
        p["F"] = F.reshape(-1, 9)
    return Scene(f"small_{n}", n, dx, dt, 1, gravity, mats, wall_bcs(n, dx), p,
                 newton_rtol=1e-10, pcg_rtol=1e-10, occupied_cells=len(cells))


def colliding_cubes(n=32, seed=14, speed=0.5, E=5e3, nu=0.3) -> Scene:
    """Two 0.1 m-ish elastic cubes approaching along x with opposite velocities
    (linear-momentum study); no gravity, no walls touched."""
    dx = 1.0 / n
    rng = np.random.Generator(np.random.PCG64(seed))
    side = max(2, int(round(0.1 / dx)))
    mid = n // 2
    a = box_cells((mid - side - 1, mid - side // 2, mid - side // 2),
                  (mid - 1, mid - side // 2 + side, mid - side // 2 + side))
    b = box_cells((mid + 1, mid - side // 2, mid - side // 2),
                  (mid + side + 1, mid - side // 2 + side, mid - side // 2 + side))
    cells = np.concatenate([a, b])
    mats = [material(NEOHOOKEAN, E, nu, 1000.0)]
    x = fill_cells(cells, dx, 2, rng)
    p = make_particles(x, np.zeros(len(x), np.int32), mats, dx, 8)
    p["v"][:, 0] = np.where(x[:, 0] < mid * dx, speed, -speed)
    return Scene(f"cubes_{n}", n, dx, 1e-3, 10, (0.0, 0.0, 0.0), mats, wall_bcs(n, dx), p,
                 newton_rtol=1e-10, pcg_rtol=1e-10, occupied_cells=len(cells))


def spinning_rod(n=32, seed=15, omega=4.0, E=5e3, nu=0.3) -> Scene:
    """A rod along z (radius 0.05 m, length 0.4 m, scaled to the grid) spinning
    about z at ``omega`` rad/s (angular-momentum study); no gravity."""
    dx = 1.0 / n
    rng = np.random.Generator(np.random.PCG64(seed))
    c = (np.arange(n) + 0.5) * dx
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    r = max(0.05, 1.6 * dx)
    inside = ((X - 0.5) ** 2 + (Y - 0.5) ** 2 <= r * r) & (np.abs(Z - 0.5) <= 0.2)
    cells = np.argwhere(inside)
    mats = [material(NEOHOOKEAN, E, nu, 1000.0)]
    x = fill_cells(cells, dx, 2, rng)
    p = make_particles(x, np.zeros(len(x), np.int32), mats, dx, 8)
    rx, ry = x[:, 0] - 0.5, x[:, 1] - 0.5
    p["v"] = np.stack([-omega * ry, omega * rx, np.zeros_like(rx)], 1)
    G = np.zeros((len(x), 3, 3))
    G[:, 0, 1] = -omega
    G[:, 1, 0] = omega
    p["G"] = G.reshape(-1, 9)
    return Scene(f"rod_{n}", n, dx, 1e-3, 10, (0.0, 0.0, 0.0), mats, wall_bcs(n, dx), p,
                 newton_rtol=1e-10, pcg_rtol=1e-10, occupied_cells=len(cells))


def jelly_falling(seed: int = 6, n: int = 256, ppc_axis: int = 2, speed: float = 1.0) -> Scene:
    """Explicit workload shaped like the paper's Jelly Falling example: StVK
    with Hencky strain, E = 5e3, nu = 0.4, rho = 1000, dt = 6e-5, gravity and
    sticky walls.  A slab of 3/8 n x n/32 x 3/8 n cells rests on the floor and
    two n/8-cubes fall onto it at ``speed`` m/s; at n = 256 that is 139,264
    occupied cells and 1,114,112 particles at 8 per cell."""
    dx = 1.0 / n
    rng = np.random.Generator(np.random.PCG64(seed))
    mats = [material(HENCKY, 5e3, 0.4, 1000.0)]
    e = n // 8
    base = box_cells((5 * n // 16, 2, 5 * n // 16), (11 * n // 16, 2 + max(n // 32, 1), 11 * n // 16))
    c1 = box_cells((23 * n // 64, 5 * n // 32, 23 * n // 64),
                   (23 * n // 64 + e, 5 * n // 32 + e, 23 * n // 64 + e))
    c2 = box_cells((33 * n // 64, 15 * n // 64, 33 * n // 64),
                   (33 * n // 64 + e, 15 * n // 64 + e, 33 * n // 64 + e))
    cells = np.concatenate([base, c1, c2])
    x = fill_cells(cells, dx, ppc_axis, rng)
    p = make_particles(x, np.zeros(len(x), np.int32), mats, dx, ppc_axis ** 3)
    ppc = ppc_axis ** 3
    falling = np.repeat(np.arange(len(cells)) >= len(base), ppc)
    p["v"][falling, 1] = -speed
    return Scene(f"jelly_falling_{n}", n, dx, 6e-5, 100, (0.0, -9.81, 0.0), mats, wall_bcs(n, dx), p,
                 occupied_cells=len(cells))


def two_material_bar(seed: int = 7, n: int = 64, ppc_axis: int = 2, speed: float = 0.5) -> Scene:
    """Soft-stiff-soft bar shaped like the paper's VBD comparison: split
    Neo-Hookean, E = 1e4 at both ends and 1e5 in the middle third, nu = 0.3,
    rho = 1000, dt = 1e-3, gravity.  The bar runs along z over 48 cells with a
    16 x 16 section; the nodes of its first 2 cell layers are held and those
    of its last 2 layers are dragged along +x at ``speed`` m/s (the paper
    twists the end; the boxes here translate).  At n = 64: 12,288 cells,
    98,304 particles."""
    dx = 1.0 / n
    rng = np.random.Generator(np.random.PCG64(seed))
    mats = [material(NEOHOOKEAN, 1e4, 0.3, 1000.0), material(NEOHOOKEAN, 1e5, 0.3, 1000.0)]
    x0, x1 = 3 * n // 8, 5 * n // 8
    z0, z1 = n // 8, 7 * n // 8
    cells = box_cells((x0, x0, z0), (x1, x1, z1))
    third = (z1 - z0) // 3
    ids_c = ((cells[:, 2] >= z0 + third) & (cells[:, 2] < z1 - third)).astype(np.int32)
    x = fill_cells(cells, dx, ppc_axis, rng)
    ppc = ppc_axis ** 3
    p = make_particles(x, np.repeat(ids_c, ppc), mats, dx, ppc)
    big = 10.0
    bcs = wall_bcs(n, dx) + [
        dict(kind=BC_STICKY_BOX, lo=(-big, -big, -big), hi=(big, big, (z0 + 2) * dx), velocity=(0.0, 0.0, 0.0)),
        dict(kind=BC_MOVING_BOX, lo=(-big, -big, (z1 - 2) * dx), hi=(big, big, big), velocity=(speed, 0.0, 0.0)),
    ]
    return Scene(f"two_material_bar_{n}", n, dx, 1e-3, 10, (0.0, -9.81, 0.0), mats, bcs, p,
                 occupied_cells=len(cells))


def sand_cone(theta_deg: float, seed: int = 41, n: int = 48, radius: float = 0.3, E: float = 1e6,
              friction_deg: float = 30.0, ppc_axis: int = 2, dt: float = 2e-3) -> Scene:
    """A right circular cone of Drucker-Prager sand (Hencky, E = 1e6, nu = 0.3,
    rho = 2000, friction angle ``friction_deg``) standing on the sticky floor of
    the unit box: apex over the box centre, base radius ``radius`` at
    y = 2 dx, flank slope ``theta_deg``; the cells whose centre lies inside
    the cone are filled.  At rest, gravity, dt = 2e-3 (the sand-pile setting
    of the paper's fixed-point plasticity comparison).  At n = 48 the 45 and
    20 degree cones hold 25,120 and 9,120 particles."""
    dx = 1.0 / n
    rng = np.random.Generator(np.random.PCG64(seed))
    t = math.tan(math.radians(theta_deg))
    y0 = 2 * dx
    c = (np.arange(n) + 0.5) * dx
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    r = np.hypot(X - 0.5, Z - 0.5)
    inside = (Y >= y0) & (Y - y0 <= radius * t - r * t)
    cells = np.argwhere(inside)
    mats = [material(HENCKY, E, 0.3, 2000.0, PLASTIC_DRUCKER_PRAGER, 0.0, friction_deg)]
    x = fill_cells(cells, dx, ppc_axis, rng)
    ppc = ppc_axis ** 3
    p = make_particles(x, np.zeros(len(x), np.int32), mats, dx, ppc)
    return Scene(f"sand_cone_{int(round(theta_deg))}deg_{n}", n, dx, dt, 400, (0.0, -9.81, 0.0), mats,
                 wall_bcs(n, dx), p, newton_rtol=1e-5, pcg_rtol=1e-5, occupied_cells=len(cells),
                 meta=dict(theta_deg=theta_deg, radius=radius, floor_y=y0))


CONFIGS = {1: config1, 2: config2, 3: config3, 5: config5}
