"""Pins of the multigrid oracle (oracle/multigrid.py), each against
something other than the oracle's own code path:

* the transfer operators against trilinear hat functions evaluated at the
  fine nodes (partition of unity, exact interpolation of linear fields,
  restriction = transpose of prolongation);
* the rediscretised coarse operator against the fine one on linear fields
  (equal elastic energies) and the total mass;
* the two-level V-cycle against the textbook two-grid operator assembled
  from dense matrices (smoother polynomial, coarse correction with an exact
  coarse solve);
* the multilevel V-cycle's symmetry and positive definiteness, the power
  iteration's estimate against the dense spectrum, and the MG-preconditioned
  CG against a dense solve.
"""
import numpy as np
import pytest

from oracle import multigrid as MG
from oracle import oracle as O
from paper_2602_07853_amd import scenes
from tests.parity_util import oracle_state


def _hat_matrix(n_fine: int) -> np.ndarray:
    """Dense [(n_fine+1)^3, (n_fine/2+1)^3] matrix of the coarse trilinear
    hat functions phi_X(x) = prod_a max(0, 1 - |x_a - 2 X_a| / 2) at the fine
    nodes (node units of the fine grid)."""
    nf, nc = n_fine + 1, n_fine // 2 + 1
    xf = np.stack(np.meshgrid(*(np.arange(nf),) * 3, indexing="ij"), -1).reshape(-1, 3)
    xc = 2 * np.stack(np.meshgrid(*(np.arange(nc),) * 3, indexing="ij"), -1).reshape(-1, 3)
    d = np.abs(xf[:, None, :] - xc[None, :, :]).astype(float)
    return np.prod(np.maximum(0.0, 1.0 - d / 2.0), axis=-1)


def test_transfer_is_trilinear_interpolation():
    n = 6
    P = _hat_matrix(n)
    rng = np.random.default_rng(1)
    uc = rng.normal(size=((n // 2 + 1) ** 3, 3))
    assert np.allclose(MG.prolong_field(n, uc), P @ uc, rtol=0, atol=1e-14)
    uf = rng.normal(size=((n + 1) ** 3, 2))
    assert np.allclose(MG.restrict_field(n, uf), P.T @ uf, rtol=0, atol=1e-13)
    # partition of unity and exact interpolation of a linear field
    assert np.allclose(P.sum(axis=1), 1.0, atol=0)
    nc = n // 2 + 1
    Xc = 2.0 * np.stack(np.meshgrid(*(np.arange(nc),) * 3, indexing="ij"), -1).reshape(-1, 3)
    Xf = np.stack(np.meshgrid(*(np.arange(n + 1),) * 3, indexing="ij"), -1).reshape(-1, 3)
    M, t = rng.normal(size=(3, 3)), rng.normal(size=3)
    assert np.allclose(MG.prolong_field(n, Xc @ M.T + t), Xf @ M.T + t, rtol=0, atol=1e-12)


def _synthetic_level(n=4, seed=2):
    """Every cell active with a random SPD 9x9 tangent, every node carrying
    mass and free."""
    rng = np.random.default_rng(seed)
    Q = rng.normal(size=(n ** 3, 9, 9))
    A = np.einsum("cij,ckj->cik", Q, Q).reshape(n ** 3, 81)
    mc = np.ones(n ** 3)
    mi = rng.uniform(0.5, 1.5, (n + 1) ** 3)
    fixed = np.zeros((n + 1) ** 3, dtype=np.uint8)
    return MG._level(O.Grid(n, 1.0 / n), mc, mi, fixed, A)


def test_coarse_operator_keeps_the_energy_of_linear_fields():
    fine = _synthetic_level()
    coarse = MG.coarsen(fine)
    n = fine.grid.n
    rng = np.random.default_rng(3)
    Xc = (2.0 / n) * np.stack(np.meshgrid(*(np.arange(n // 2 + 1),) * 3, indexing="ij"), -1).reshape(-1, 3)
    for _ in range(3):
        M, t = rng.normal(size=(3, 3)), rng.normal(size=3)
        uc = Xc @ M.T + t
        uf = MG.prolong_field(n, uc)
        ef = float(np.sum(uf * fine.apply(uf)) - np.sum(fine.mi[:, None] * uf * uf))
        ec = float(np.sum(uc * coarse.apply(uc)) - np.sum(coarse.mi[:, None] * uc * uc))
        assert ef > 0
        assert abs(ec - ef) <= 1e-12 * ef
    # the coarse masses are P^T m, so the total mass is kept
    assert np.allclose(coarse.mi, _hat_matrix(n).T @ fine.mi, rtol=1e-15, atol=0)
    assert abs(coarse.mi.sum() - fine.mi.sum()) <= 1e-13 * fine.mi.sum()


def _dense(apply, nd):
    return np.stack([apply(e.reshape(-1, 3)).reshape(-1) for e in np.eye(nd)], axis=1)


def _small_levels(n=8, max_levels=2, seed=31, E=1e6):
    sc = scenes.small_block(n=n, lo=2, hi=n - 2, strain=0.05, model=scenes.FIXED_COROTATED,
                            E=E, seed=seed)
    ref = oracle_state(sc)
    A, _ = O.tangent(ref["grid"], ref["mats"], sc.dt, ref["Vck"], ref["S"], ref["vhat"], project=True)
    return MG.hierarchy(ref["grid"], ref["mc"], ref["mi"], ref["fixed"], A, max_levels=max_levels,
                        min_cells=2)


@pytest.mark.parametrize("nu", [1, 2])
def test_two_level_cycle_is_the_textbook_two_grid_operator(nu):
    levels = _small_levels()
    fine, coarse = levels
    n = fine.grid.n
    ndf, ndc = 3 * (n + 1) ** 3, 3 * (n // 2 + 1) ** 3
    Af = _dense(fine.apply, ndf)
    Ac = _dense(coarse.apply, ndc)
    ff, fc = fine.free.reshape(-1), coarse.free.reshape(-1)
    # masked trilinear prolongation from the hat functions
    P = np.kron(_hat_matrix(n), np.eye(3)) * ff[:, None] * fc[None, :]
    W = np.diag(np.where(ff, fine.omega / np.where(ff, fine.D.reshape(-1), 1.0), 0.0))
    Acp = np.zeros_like(Ac)
    Acp[np.ix_(fc, fc)] = np.linalg.inv(Ac[np.ix_(fc, fc)])
    I = np.eye(ndf)
    S = W.copy()                       # nu sweeps from zero: S_{k+1} = S_k + W (I - A S_k)
    for _ in range(nu - 1):
        S = S + W @ (I - Af @ S)
    E = np.linalg.matrix_power(I - W @ Af, nu)
    B_ref = E @ (S + P @ Acp @ P.T @ (I - Af @ S)) + S

    def exact(bc):
        return (Acp @ bc.reshape(-1)).reshape(-1, 3)

    B = _dense(lambda e: MG.vcycle(levels, e, nu=nu, coarse_solve=exact), ndf)
    sub = np.ix_(ff, ff)
    assert np.max(np.abs(B[sub] - B_ref[sub])) <= 1e-12 * np.max(np.abs(B_ref[sub]))
    assert np.all(B[~ff] == 0.0) and np.all(B[:, ~ff] == 0.0)


def test_vcycle_is_symmetric_positive_definite_and_omega_contracts():
    levels = _small_levels(n=16, max_levels=3)
    assert [lv.grid.n for lv in levels] == [16, 8, 4]
    rng = np.random.default_rng(7)
    fr = levels[0].free
    for _ in range(3):
        x = rng.normal(size=fr.shape) * fr
        y = rng.normal(size=fr.shape) * fr
        bx, by = MG.vcycle(levels, x, nu=2), MG.vcycle(levels, y, nu=2)
        assert abs(np.sum(bx * y) - np.sum(x * by)) <= 1e-12 * np.linalg.norm(bx) * np.linalg.norm(y)
        assert np.sum(bx * x) > 0.0
    # the power-iteration estimate against the dense spectrum of D^-1/2 A D^-1/2
    lv = levels[1]
    n1 = 3 * (lv.grid.n + 1) ** 3
    f = lv.free.reshape(-1)
    A = _dense(lv.apply, n1)[np.ix_(f, f)]
    s = 1.0 / np.sqrt(lv.D.reshape(-1)[f])
    lam_true = np.linalg.eigvalsh(s[:, None] * A * s[None, :])[-1]
    lam_est = MG.lambda_max_estimate(lv, 10)
    assert 0.8 * lam_true <= lam_est <= lam_true * (1 + 1e-12)
    assert lv.omega * lam_true < 2.0


def test_mg_pcg_solves_the_newton_system():
    levels = _small_levels(n=8, max_levels=2)
    fine = levels[0]
    rng = np.random.default_rng(9)
    fr = fine.free
    b = rng.normal(size=fr.shape) * fr
    nd = 3 * (fine.grid.n + 1) ** 3
    f = fr.reshape(-1)
    A = _dense(fine.apply, nd)[np.ix_(f, f)]
    xd = np.linalg.solve(A, b.reshape(-1)[f])
    for nu in (1, 2):
        x, it, rel = MG.pcg(levels, b, 1e-11, nu=nu)
        assert rel <= 1e-10
        assert np.linalg.norm(x.reshape(-1)[f] - xd) <= 1e-9 * np.linalg.norm(xd)


def test_mg_pcg_needs_fewer_iterations_than_jacobi_on_a_stiff_block():
    # stiffness-to-mass ratio dt^2 E / (rho dx^2) = 100: the smooth modes
    # Jacobi leaves behind are what the coarse level removes
    levels = _small_levels(n=8, max_levels=2, E=1.6e9)
    fr = levels[0].free
    b = np.random.default_rng(10).normal(size=fr.shape) * fr
    _, it_mg, rel = MG.pcg(levels, b, 1e-8, nu=2)
    _, it_j, _ = MG.pcg(levels, b, 1e-8, precond="jacobi")
    assert rel <= 1e-8
    assert it_mg < 0.8 * it_j


def test_power_start_generator_is_splitmix64():
    # SplitMix64 seeded with 0 (state advanced by the golden gamma before the
    # finaliser): its first outputs, as the generator's published reference
    # implementation prints them
    out = MG.splitmix64(np.arange(3, dtype=np.uint64))
    assert [int(v) for v in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
