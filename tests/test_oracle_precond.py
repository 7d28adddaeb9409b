"""Pins of the preconditioner oracle (oracle/precond.py) and of the oracle's
Jacobi diagonal: the diagonal against e_i^T H e_i from the oracle's own
Hessian-vector product, zero network weights against Jacobi (z = r / D),
and the features' invariances."""
import numpy as np

from oracle import oracle as O
from oracle import precond as PC
from oracle import unet as U
from paper_2602_07853_amd import scenes
import pytest

from tests.parity_util import oracle_state, slip_walls


def _system(kind="block"):
    """A strained block in sticky walls, or (``slip``) the block whose
    boundary nodes carry every combination of fixed components."""
    if kind == "slip":
        sc = slip_walls()
    else:
        sc = scenes.small_block(n=8, lo=2, hi=6, strain=0.05, model=scenes.FIXED_COROTATED, seed=31)
    ref = oracle_state(sc)
    A, _ = O.tangent(ref["grid"], ref["mats"], sc.dt, ref["Vck"], ref["S"], ref["vhat"], project=True)
    D = O.jacobi_diag(ref["grid"], ref["mc"], ref["mi"], ref["fixed"], A)
    return sc, ref, A, D


def test_jacobi_diag_is_the_diagonal_of_H():
    sc, ref, A, D = _system()
    free = np.flatnonzero((ref["mi"] > 0) & (ref["fixed"] == 0))
    assert len(free) > 10
    rng = np.random.default_rng(3)
    for node in rng.choice(free, 6, replace=False):
        for a in range(3):
            e = np.zeros_like(ref["vhat"])
            e[node, a] = 1.0
            He = O.hv(ref["grid"], ref["mc"], ref["mi"], ref["fixed"], A, e)
            assert abs(He[node, a] - D[node, a]) <= 1e-12 * abs(D[node, a])
    fixed_or_empty = (ref["mi"] == 0) | (ref["fixed"] > 0)
    assert np.all(D[fixed_or_empty] == 0.0) and np.all(D[~fixed_or_empty] > 0.0)


@pytest.mark.parametrize("kind", ["block", "slip"])
def test_zero_weights_give_jacobi(kind):
    sc, ref, A, D = _system(kind)
    rng = np.random.default_rng(4)
    r = rng.normal(size=D.shape) * (D > 0)
    params = np.zeros(U.param_layout()[1])
    z = PC.apply(params, sc.n, r, D)
    fr = D > 0
    assert np.allclose(z[fr], r[fr] / D[fr], rtol=1e-15, atol=0.0)
    assert np.all(z[~fr] == 0.0)


@pytest.mark.parametrize("kind", ["block", "slip"])
def test_features_are_scale_invariant_and_masked(kind):
    sc, ref, A, D = _system(kind)
    rng = np.random.default_rng(5)
    r = rng.normal(size=D.shape) * (D > 0)
    f1 = PC.features(sc.n, r, D)
    f2 = PC.features(sc.n, 37.5 * r, D)
    assert np.allclose(f1, f2, rtol=1e-13, atol=1e-15)
    n1 = sc.n + 1
    b = PC.box_dims(sc.n)[0]
    assert f1.shape == (b, b, b, U.IN_CH)
    assert np.all(f1[n1:] == 0) and np.all(f1[:, n1:] == 0) and np.all(f1[:, :, n1:] == 0)
    dof = (D > 0).reshape(n1, n1, n1, 3)
    nodes = dof.any(axis=3)
    if kind == "slip":   # partly fixed nodes are present
        assert np.any(nodes & ~dof.all(axis=3))
    assert np.array_equal(f1[:n1, :n1, :n1, 4] == 1.0, nodes)
    # fixed components read 0; the scaled residual has unit mean square over the free DOFs
    assert np.all(f1[:n1, :n1, :n1, :3][~dof] == 0.0)
    assert np.isclose(np.mean(f1[:n1, :n1, :n1, :3][dof] ** 2), 1.0)
    assert np.all(f1[..., 5:] == 0)


@pytest.mark.parametrize("kind", ["block", "slip"])
def test_preconditioned_residual_is_equivariant_in_scale(kind):
    """z(alpha r) = alpha z(r): the network sees a normalised residual; z
    is 0 on the fixed components."""
    sc, ref, A, D = _system(kind)
    rng = np.random.default_rng(6)
    r = rng.normal(size=D.shape) * (D > 0)
    params = U.init_params(seed=7, scale=0.5)
    z1 = PC.apply(params, sc.n, r, D)
    z2 = PC.apply(params, sc.n, 1e3 * r, D)
    assert np.allclose(z2, 1e3 * z1, rtol=1e-10, atol=1e-300)
    assert np.all(z1[~(D > 0)] == 0.0)
    assert not np.allclose(z1, np.where(D > 0, r / np.where(D > 0, D, 1.0), 0.0))
