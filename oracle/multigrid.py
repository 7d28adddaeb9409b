"""FP64 oracle of the multigrid-preconditioned CG on the incremental
potential — TEST INFRASTRUCTURE ONLY (tests, smoke, bench CPU-baseline leg).

The paper names multigrid-preconditioned CG, next to plain PCG, as an
off-the-shelf solver for the same incremental potential (Sec. 7, the vertex
block descent comparison) and does not define it.  What is written here is
the textbook geometric V-cycle (Briggs, Henson and McCormick, "A Multigrid
Tutorial", ch. 3-4; Trottenberg, Oosterlee and Schueller, "Multigrid",
ch. 2) on the voxel mesh, with these readings:

* Levels.  Level 0 is the step's grid (N^3 cells, spacing dx).  Level l+1
  halves every axis: cell (I, J, K) of level l+1 is the union of the eight
  cells (2I + a, 2J + b, 2K + c), a, b, c in {0, 1}, of level l, and its
  nodes sit on the even nodes of level l.  Levels are added while the cell
  count per axis stays even and the coarse count stays >= ``min_cells``.
* Coarse operator (rediscretisation).  The coarse cell's tangent is the sum
  of its eight children's (each already carries its dt^2 V factor), and the
  coarse product is the same one-point Q1 product (Sec. 3.3 gradients with
  the coarse spacing).  For a field that is linear in space the coarse and
  the fine elastic energies are then equal.  Coarse masses are the
  restricted fine masses, m_C = P^T m (lumped).
* Transfer.  P is trilinear interpolation of a coarse node field to the fine
  nodes (weight 1 on a co-located node, 1/2 per axis on an odd offset), and
  the restriction is its transpose.  Both act on free degrees of freedom
  only: a prolonged correction is zeroed on fixed or massless fine DOFs,
  and a restricted residual on fixed or massless coarse DOFs.
* Dirichlet sets on coarse levels.  Component a of coarse node I is fixed
  when the co-located fine node 2I carries mass and has component a fixed.
* Smoother.  ``nu`` damped-Jacobi sweeps x <- x + omega_l D^-1 (b - A x)
  before the coarse correction (the first from x = 0) and ``nu`` after it;
  the coarsest level takes ``nu_coarse`` sweeps from x = 0.  D is the
  diagonal of the level's matrix on its free DOFs.  The damping is
  omega_l = ``omega_scale`` / lambda_l, where lambda_l estimates the largest
  eigenvalue of D^-1/2 A D^-1/2 by ``power_iters`` power iterations (Rayleigh
  quotient of the last iterate) from x_0 = +-1 on the free DOFs, the sign of
  DOF q = 3 node + a being the top bit of SplitMix64(q) (Steele, Lea and
  Flood 2014): a start with no structure, since a checkerboard is an
  hourglass pattern of the one-point rule, near the bottom of the spectrum.
  One-point Q1 elasticity puts lambda_max near 5, so a fixed omega that
  suits the Laplacian (2/3) would not contract.  Pre- and post-smoothing
  with the same symmetric sweep and R = P^T make the V-cycle a symmetric
  operator, positive definite when every level's sweep contracts in the
  energy norm (omega lambda_max(D^-1 A) < 2); any symmetric positive
  definite coarse matrix keeps it so, whether or not it equals P^T A P.

All arrays follow ``oracle/oracle.py``: dense cells ``(i*N + j)*N + k`` and
nodes ``(i*(N+1) + j)*(N+1) + k``, node vectors [nodes, 3].
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from oracle import oracle as O


@dataclass
class Level:
    grid: O.Grid
    mc: np.ndarray      # [cells] cell mass (> 0: the cell carries quadrature)
    mi: np.ndarray      # [nodes] lumped node mass
    fixed: np.ndarray   # [nodes] uint8, bit a: component a prescribed
    A: np.ndarray       # [cells, 81] projected tangent dt^2 sum_k V A_k (row-major 9x9)
    D: np.ndarray       # [nodes, 3] diagonal of the level's matrix on free DOFs, 0 elsewhere
    omega: float = 0.0  # damping of the level's Jacobi sweeps (set by ``hierarchy``)

    @property
    def free(self):
        """[nodes, 3] bool: free degrees of freedom."""
        return (self.mi[:, None] > 0.0) & ~O.fixed_components(self.fixed)

    def apply(self, u):
        """The level's matrix times u (the one-point Q1 product plus lumped
        mass, Sec. 3.3 / Alg. 3), masked to free DOFs on both sides."""
        return O.hv(self.grid, self.mc, self.mi, self.fixed, self.A, u)


def splitmix64(q):
    """SplitMix64 output for the counters q (uint64 array): the state
    q * 0x9E3779B97F4A7C15 + 0x9E3779B97F4A7C15 through the published
    finaliser (shifts 30, 27, 31; multipliers 0xBF58476D1CE4E5B9,
    0x94D049BB133111EB), all arithmetic modulo 2^64."""
    with np.errstate(over="ignore"):
        z = (np.asarray(q, dtype=np.uint64) + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def power_start(lv: Level):
    """x_0 of the power iteration (module docstring), [nodes, 3]."""
    q = np.arange(3 * lv.mi.size, dtype=np.uint64)
    sgn = np.where((splitmix64(q) >> np.uint64(63)) == 0, 1.0, -1.0).reshape(-1, 3)
    return np.where(lv.free, sgn, 0.0)


def lambda_max_estimate(lv: Level, iters: int) -> float:
    """Power iteration on D^-1/2 A D^-1/2 over the free DOFs (module
    docstring); the Rayleigh quotient of the last iterate."""
    fr = lv.free
    x = power_start(lv)
    s = np.where(fr, 1.0 / np.sqrt(np.where(fr, lv.D, 1.0)), 0.0)
    lam = 0.0
    for _ in range(iters):
        nx = np.linalg.norm(x)
        if nx == 0.0:
            return 0.0
        x = x / nx
        y = s * lv.apply(s * x)
        lam = float(np.sum(x * y))
        x = y
    return lam


def _level(grid, mc, mi, fixed, A):
    D = O.jacobi_diag(grid, mc, mi, fixed, A)
    return Level(grid, np.asarray(mc, float), np.asarray(mi, float),
                 np.ascontiguousarray(fixed, dtype=np.uint8), np.asarray(A, float), D)


def _interp_1d(n_fine: int) -> np.ndarray:
    """[n_fine + 1, n_fine // 2 + 1] trilinear weights along one axis: fine
    node x takes coarse node X with weight 1 (x = 2X) or 1/2 (|x - 2X| = 1)."""
    nc = n_fine // 2
    P = np.zeros((n_fine + 1, nc + 1))
    for x in range(n_fine + 1):
        if x % 2 == 0:
            P[x, x // 2] = 1.0
        else:
            P[x, (x - 1) // 2] = 0.5
            P[x, (x + 1) // 2] = 0.5
    return P


def prolong_field(n_fine: int, uc):
    """Trilinear interpolation of a coarse node field [(nc+1)^3, k] to the
    fine nodes [(n_fine+1)^3, k] (no masking)."""
    P1 = _interp_1d(n_fine)
    nc = n_fine // 2
    u = np.asarray(uc, float).reshape(nc + 1, nc + 1, nc + 1, -1)
    u = np.einsum("xX,XYZc->xYZc", P1, u)
    u = np.einsum("yY,xYZc->xyZc", P1, u)
    u = np.einsum("zZ,xyZc->xyzc", P1, u)
    return u.reshape((n_fine + 1) ** 3, -1)


def restrict_field(n_fine: int, uf):
    """The transpose of ``prolong_field``: fine node field -> coarse nodes."""
    P1 = _interp_1d(n_fine)
    nf = n_fine + 1
    u = np.asarray(uf, float).reshape(nf, nf, nf, -1)
    u = np.einsum("xX,xyzc->Xyzc", P1, u)
    u = np.einsum("yY,Xyzc->XYzc", P1, u)
    u = np.einsum("zZ,XYzc->XYZc", P1, u)
    return u.reshape((n_fine // 2 + 1) ** 3, -1)


def coarsen(fine: Level) -> Level:
    """The next coarser level (module docstring: rediscretised operator,
    restricted masses, co-located Dirichlet components)."""
    n = fine.grid.n
    assert n % 2 == 0, "a level is coarsened only when its cell count per axis is even"
    nc = n // 2
    A = fine.A.reshape(nc, 2, nc, 2, nc, 2, 81).sum(axis=(1, 3, 5)).reshape(nc ** 3, 81)
    mc = fine.mc.reshape(nc, 2, nc, 2, nc, 2).sum(axis=(1, 3, 5)).reshape(-1)
    mi = restrict_field(n, fine.mi[:, None])[:, 0]
    nf = n + 1
    ff = fine.fixed.reshape(nf, nf, nf)[::2, ::2, ::2].reshape(-1)
    fm = fine.mi.reshape(nf, nf, nf)[::2, ::2, ::2].reshape(-1)
    fixed = np.where(fm > 0.0, ff, 0).astype(np.uint8)
    return _level(O.Grid(nc, 2.0 * fine.grid.dx), mc, mi, fixed, A)


def hierarchy(grid, mc, mi, fixed, A, max_levels: int = 5, min_cells: int = 4,
              omega_scale: float = 1.6, power_iters: int = 20):
    """Level 0 from the step's grid data, then coarser levels while the cell
    count per axis is even and the coarse count stays >= ``min_cells``; each
    level's damping omega_l = omega_scale / lambda_l (module docstring)."""
    levels = [_level(grid, mc, mi, fixed, A)]
    while (len(levels) < max_levels and levels[-1].grid.n % 2 == 0
           and levels[-1].grid.n // 2 >= min_cells):
        levels.append(coarsen(levels[-1]))
    for lv in levels:
        lam = lambda_max_estimate(lv, power_iters)
        lv.omega = omega_scale / lam if lam > 0.0 else 0.0
    return levels


def restrict(fine: Level, coarse: Level, r):
    """Masked restriction R = P^T of a fine residual to the coarse level."""
    rc = restrict_field(fine.grid.n, np.where(fine.free, r, 0.0))
    return np.where(coarse.free, rc, 0.0)


def prolong(fine: Level, coarse: Level, ec):
    """Masked trilinear prolongation of a coarse correction."""
    e = prolong_field(fine.grid.n, np.where(coarse.free, ec, 0.0))
    return np.where(fine.free, e, 0.0)


def _jacobi_step(lv: Level, b, x):
    omega = lv.omega
    fr = lv.free
    Dinv = np.where(fr, 1.0 / np.where(fr, lv.D, 1.0), 0.0)
    if x is None:
        return omega * Dinv * b
    return x + omega * Dinv * (b - lv.apply(x))


def vcycle(levels, b, nu: int = 1, nu_coarse: int = 4, level: int = 0, coarse_solve=None):
    """One symmetric V-cycle z = B b from level ``level`` down (module
    docstring).  ``coarse_solve`` (tests only) replaces the coarsest sweeps
    by a given exact solver."""
    lv = levels[level]
    b = np.where(lv.free, b, 0.0)
    if level == len(levels) - 1:
        if coarse_solve is not None:
            return coarse_solve(b)
        x = None
        for _ in range(nu_coarse):
            x = _jacobi_step(lv, b, x)
        return x
    x = None
    for _ in range(nu):
        x = _jacobi_step(lv, b, x)
    r = b - lv.apply(x)
    nxt = levels[level + 1]
    ec = vcycle(levels, restrict(lv, nxt, r), nu, nu_coarse, level + 1, coarse_solve)
    x = x + prolong(lv, nxt, ec)
    for _ in range(nu):
        x = _jacobi_step(lv, b, x)
    return x


def pcg(levels, b, rtol: float, max_iter: int = 10000, nu: int = 1, nu_coarse: int = 4,
        precond: str = "mg"):
    """Preconditioned CG (Hestenes-Stiefel, x0 = 0) on level 0's matrix with
    the V-cycle (``precond="mg"``) or Jacobi (``"jacobi"``); stops when
    |b - A x| <= rtol |b| over free DOFs.  Returns (x, iterations, the true
    relative residual)."""
    lv = levels[0]
    fr = lv.free
    b = np.where(fr, b, 0.0)

    def prec(r):
        if precond == "jacobi":
            return np.where(fr, r / np.where(fr, lv.D, 1.0), 0.0)
        return vcycle(levels, r, nu, nu_coarse)

    x = np.zeros_like(b)
    r = b.copy()
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return x, 0, 0.0
    z = prec(r)
    p = z.copy()
    rz = float(np.sum(r * z))
    it = 0
    while it < max_iter and np.linalg.norm(r) > rtol * bn:
        q = lv.apply(p)
        alpha = rz / float(np.sum(p * q))
        x = x + alpha * p
        r = r - alpha * q
        z = prec(r)
        rz_new = float(np.sum(r * z))
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    true_rel = np.linalg.norm(b - lv.apply(x)) / bn
    return x, it, true_rel
