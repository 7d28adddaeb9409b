"""Pins of the training path of the learned preconditioner in the oracle
(oracle/precond.py): the energy-norm loss and its gradients, Adam, and the
training-pair target, checked against properties fixed by the mathematics
rather than against the formulas themselves:

  * L is quadratic in z, so central differences are exact up to rounding;
  * L is minimised by z = H^{-1} r (solved here with SciPy's CG on the
    oracle's own product), with the closed-form value -r^T H^{-1} r / (2 r^T D^{-1} r),
    and L(z) - L(H^{-1} r) = |z - H^{-1} r|_H^2 / (2 r^T D^{-1} r);
  * Adam's first step moves every parameter by lr against the sign of its
    gradient, a constant gradient keeps doing so, and a second step with a
    new gradient matches moments worked out by hand as fractions;
  * a pair target fed through the preconditioner map gives z = x* - x_k
    exactly, i.e. the loss minimiser.
"""
import numpy as np
import scipy.sparse.linalg as spla

from oracle import oracle as O
from oracle import precond as PC
from paper_2602_07853_amd import scenes
from tests.parity_util import oracle_state


def _system(seed=31, E=1e7):
    # E = 1e7 makes the elastic part of H comparable to the mass part, so
    # that a few CG iterations leave a residual far from converged
    sc = scenes.small_block(n=8, lo=2, hi=6, strain=0.05, model=scenes.FIXED_COROTATED, seed=seed, E=E)
    ref = oracle_state(sc)
    g = ref["grid"]
    A, _ = O.tangent(g, ref["mats"], sc.dt, ref["Vck"], ref["S"], ref["vhat"], project=True)
    D = O.jacobi_diag(g, ref["mc"], ref["mi"], ref["fixed"], A)

    def H(u):
        return O.hv(g, ref["mc"], ref["mi"], ref["fixed"], A, u)
    return sc, D, H


def _solve(H, D, r, tol=1e-14):
    """x = H^{-1} r on the free DOFs with SciPy's CG (Jacobi preconditioned)."""
    fr = PC._free(D)   # [nodes, 3]: the free DOFs
    n = int(fr.sum())

    def mv(y):
        u = np.zeros(D.shape)
        u[fr] = y
        return H(u)[fr]
    op = spla.LinearOperator((n, n), matvec=mv)
    pre = spla.LinearOperator((n, n), matvec=lambda y: y / D[fr])
    sol, info = spla.cg(op, r[fr], rtol=tol, atol=0.0, maxiter=20000, M=pre)
    assert info == 0
    x = np.zeros(D.shape)
    x[fr] = sol
    return x


def test_energy_loss_gradients_by_central_differences():
    sc, D, H = _system()
    rng = np.random.default_rng(1)
    fr = D > 0
    r = rng.normal(size=D.shape) * fr
    z = rng.normal(size=D.shape) * fr / np.where(fr, D, 1.0)
    g = PC.energy_loss_grad_z(r, H(z), D)
    for k in range(3):
        u = rng.normal(size=D.shape) * fr
        h = 1e-3 * np.linalg.norm(z) / np.linalg.norm(u)
        lp = PC.energy_loss(z + h * u, r, H(z + h * u), D)
        lm = PC.energy_loss(z - h * u, r, H(z - h * u), D)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - np.sum(g * u)) <= 1e-9 * (abs(fd) + abs(lp) + abs(lm))
    # through the preconditioner map z(o) = r / D + s o / sqrt(D)
    s = PC.scale(r, D)
    o = rng.normal(size=D.shape) * fr

    def z_of(o):
        zz = np.zeros_like(r)
        zz[fr] = r[fr] / D[fr] + s * o[fr] / np.sqrt(D[fr])
        return zz
    go = PC.energy_loss_grad_o(r, H(z_of(o)), D)
    u = rng.normal(size=D.shape) * fr
    h = 1e-3
    lp = PC.energy_loss(z_of(o + h * u), r, H(z_of(o + h * u)), D)
    lm = PC.energy_loss(z_of(o - h * u), r, H(z_of(o - h * u)), D)
    fd = (lp - lm) / (2 * h)
    assert abs(fd - np.sum(go * u)) <= 1e-9 * (abs(fd) + abs(lp) + abs(lm))
    # entries off the free DOFs carry no gradient
    assert np.all(go[~fr] == 0.0) and np.all(g[~fr] == 0.0)


def test_energy_loss_minimiser_and_excess():
    sc, D, H = _system(seed=32)
    rng = np.random.default_rng(2)
    fr = D > 0
    r = rng.normal(size=D.shape) * fr
    zs = _solve(H, D, r)
    den = np.sum(r[fr] ** 2 / D[fr])
    lmin = PC.energy_loss(zs, r, H(zs), D)
    assert np.isclose(lmin, -0.5 * np.sum(r * zs) / den, rtol=1e-10)
    assert np.abs(PC.energy_loss_grad_z(r, H(zs), D)).max() <= 1e-10 * np.abs(r).max() / den
    for k in range(3):
        z = zs + rng.normal(size=D.shape) * fr * 1e-3 * np.abs(zs).max()
        e = z - zs
        excess = 0.5 * np.sum(e * H(e)) / den
        assert excess > 0.0
        assert np.isclose(PC.energy_loss(z, r, H(z), D) - lmin, excess, rtol=1e-7)
    # Jacobi (z = r / D) lies above the minimum
    zj = np.where(fr, r / np.where(fr, D, 1.0), 0.0)
    assert PC.energy_loss(zj, r, H(zj), D) > lmin


def test_adam_first_steps_by_hand():
    p0 = np.array([0.3, -1.0, 2.0])
    g1 = np.array([1.0, -2.0, 0.5])
    g2 = np.array([0.5, 0.5, -1.0])
    lr, eps = 0.1, 1e-8
    m0 = np.zeros(3)
    p1, m1, v1 = PC.adam(p0, g1, m0, m0, 1, lr)
    # step 1: bias-corrected moments are g and g^2, so the step is lr g / (|g| + eps)
    assert np.allclose(p1, p0 - lr * np.sign(g1) * np.abs(g1) / (np.abs(g1) + eps), rtol=0, atol=1e-15)
    # a constant gradient keeps the same step at t = 2 (moments stay g, g^2)
    pc, _, _ = PC.adam(p1, g1, m1, v1, 2, lr)
    assert np.allclose(pc - p1, p1 - p0, rtol=0, atol=1e-12)
    # step 2 with g2, moments worked by hand:
    #   m2 = 0.09 g1 + 0.1 g2 = (0.14, -0.13, -0.055);  mhat = m2 / 0.19
    #   v2 = 0.000999 g1^2 + 0.001 g2^2 = (0.001249, 0.004246, 0.00124975);
    #   vhat = v2 / 0.001999
    mhat = np.array([14.0 / 19.0, -13.0 / 19.0, -11.0 / 38.0])
    vhat = np.array([1249.0 / 1999.0, 4246.0 / 1999.0, 4999.0 / 7996.0])
    p2, m2, v2 = PC.adam(p1, g2, m1, v1, 2, lr)
    assert np.allclose(m2, [0.14, -0.13, -0.055], rtol=1e-14)
    assert np.allclose(v2, [0.001249, 0.004246, 0.00124975], rtol=1e-12)
    assert np.allclose(p2, p1 - lr * mhat / (np.sqrt(vhat) + eps), rtol=1e-13)


def test_pair_target_gives_the_minimiser():
    """Take a few Jacobi-PCG iterates x_k of H x = b; the target at x_k fed
    through the map of the preconditioner gives z = x* - x_k = H^{-1} r_k,
    whose energy-norm loss is the minimum."""
    sc, D, H = _system(seed=33)
    rng = np.random.default_rng(3)
    fr = D > 0
    b = rng.normal(size=D.shape) * fr
    xstar = _solve(H, D, b)
    # a plain Jacobi-PCG iterate after k steps
    x = np.zeros_like(b)
    r = b.copy()
    zz = np.where(fr, r / np.where(fr, D, 1.0), 0.0)
    p = zz.copy()
    rz = np.sum(r * zz)
    for k in range(3):
        q = H(p)
        a = rz / np.sum(p * q)
        x, r = x + a * p, r - a * q
        zz = np.where(fr, r / np.where(fr, D, 1.0), 0.0)
        rz, rz_old = np.sum(r * zz), rz
        p = zz + (rz / rz_old) * p
    r_true = b - H(x)
    assert np.linalg.norm(r_true - r) <= 1e-12 * np.linalg.norm(b)
    t = PC.pair_target(r, x, xstar, D)
    s = PC.scale(r, D)
    z = np.zeros_like(r)
    z[fr] = r[fr] / D[fr] + s * t[fr] / np.sqrt(D[fr])
    assert np.linalg.norm(z - (xstar - x)) <= 1e-13 * np.linalg.norm(xstar)
    lmin = -0.5 * np.sum(r * _solve(H, D, r)) / np.sum(r[fr] ** 2 / D[fr])
    assert np.isclose(PC.energy_loss(z, r, H(z), D), lmin, rtol=1e-9)
    assert np.all(t[~fr] == 0.0)
    # scale invariance: the target of (alpha r, alpha (x* - x)) is the same
    t2 = PC.pair_target(7.0 * r, 7.0 * x, 7.0 * xstar, D)
    assert np.linalg.norm(t2 - t) <= 1e-11 * np.linalg.norm(t)
