"""FP64 oracle of the learned preconditioner's input features and output
map — TEST INFRASTRUCTURE ONLY (tests, smoke, bench CPU-baseline leg).

The network runs on a dense box over all grid nodes of an N^3-cell grid:
voxel (i, j, k) is node (i, j, k), each axis padded from N + 1 up to a
multiple of 8 (padding voxels are zero).  With D the Jacobi diagonal of the
Newton matrix (zero off the free DOFs: massless nodes and the velocity
components a boundary condition fixes) and r a residual:

  s^2     = sum over free DOFs of r^2 / D, divided by the number of free DOFs
  x[v]    = (r_v / (s sqrt(D_v)) on its free components, 0 on the fixed ones
             (3 channels), log(mean of D_v over its free components / Dref),
             1, 11 zero channels) on nodes with a free DOF, 0 elsewhere;
             Dref = mean of that per-node mean over those nodes
  z_v     = r_v / D_v + s o_v / sqrt(D_v) on free DOFs, 0 elsewhere,

o = channels 0-2 of the network output (oracle/unet.py).  Zero weights give
o = 0, i.e. Jacobi.
"""
from __future__ import annotations

import numpy as np

from oracle import unet as U


def box_dims(n: int):
    b = ((n + 1 + 7) // 8) * 8
    return (b, b, b)


def _free(D):
    """[nodes, 3] bool: the free DOFs (D > 0)."""
    return np.asarray(D) > 0.0


def scale(r, D):
    fr = _free(D)
    s2 = np.sum(r[fr] ** 2 / D[fr])
    return np.sqrt(max(s2 / max(int(fr.sum()), 1), 1e-300))


def features(n: int, r, D):
    """Network input [X, Y, Z, 16] for node vector r [(n+1)^3, 3]."""
    fr = _free(D)
    nodes = fr.any(axis=1)
    sc = scale(r, D)
    Dsafe = np.where(fr, D, 1.0)
    dmean = np.where(nodes, np.sum(np.where(fr, D, 0.0), axis=1) / np.maximum(fr.sum(axis=1), 1), 1.0)
    dref = dmean[nodes].mean() if nodes.any() else 1.0
    f = np.zeros(((n + 1) ** 3, U.IN_CH))
    f[:, 0:3] = np.where(fr, r / (sc * np.sqrt(Dsafe)), 0.0)
    f[nodes, 3] = np.log(dmean[nodes] / dref)
    f[nodes, 4] = 1.0
    X = box_dims(n)
    box = np.zeros(X + (U.IN_CH,))
    box[:n + 1, :n + 1, :n + 1] = f.reshape(n + 1, n + 1, n + 1, U.IN_CH)
    return box


def apply(params, n: int, r, D, rnd=U._ident):
    """z = r / D + s o / sqrt(D) on free DOFs (``rnd`` as in unet.forward,
    also applied to the stored network input)."""
    x = rnd(features(n, r, D))
    return map_output(n, r, D, U.forward(params, x, rnd=rnd))


def map_output(n: int, r, D, o_box):
    """z = r / D + s o / sqrt(D) on free DOFs, o = channels 0-2 of the
    network output box o_box [X, Y, Z, >= 3] at the grid's nodes."""
    fr = _free(D)
    sc = scale(r, D)
    o = np.asarray(o_box)[:n + 1, :n + 1, :n + 1, :3].reshape(-1, 3)
    z = np.zeros_like(r)
    z[fr] = r[fr] / D[fr] + sc * o[fr] / np.sqrt(D[fr])
    return z


# ---------------------------------------------------------------- training
# The learned preconditioner is trained with two losses.  Both are written
# here from their definitions (FP64, no blocking or reordering):
#
#  * the energy-norm loss of a preconditioned residual z for the residual r
#    of the Newton system H x = b,
#        L(z) = (z^T H z / 2 - z^T r) / (r^T D^{-1} r),
#    which is minimised by z = H^{-1} r (L(z) - L(H^{-1} r) is half the
#    squared H-norm of z - H^{-1} r, over r^T D^{-1} r), and
#  * the pair loss of oracle/unet.py (masked relative L2) against the pair
#    target below.
#
# Parameters are updated by Adam (Kingma and Ba, 2015): with gradient g at
# step t (t = 1, 2, ...),
#    m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
#    p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).


def rdr(r, D):
    """r^T D^{-1} r over the free DOFs (D > 0)."""
    fr = _free(D)
    return float(np.sum(r[fr] ** 2 / D[fr]))


def energy_loss(z, r, Hz, D):
    """L(z) = (z^T H z / 2 - z^T r) / (r^T D^{-1} r) over the free DOFs, with
    Hz = H z given."""
    fr = _free(D)
    den = rdr(r, D)
    if den <= 0.0:
        return 0.0
    return (0.5 * float(np.sum(z[fr] * Hz[fr])) - float(np.sum(z[fr] * r[fr]))) / den


def energy_loss_grad_z(r, Hz, D):
    """dL/dz = (H z - r) / (r^T D^{-1} r) on free DOFs, 0 elsewhere (H is
    symmetric)."""
    fr = _free(D)
    den = rdr(r, D)
    g = np.zeros_like(r)
    if den > 0.0:
        g[fr] = (Hz[fr] - r[fr]) / den
    return g


def energy_loss_grad_o(r, Hz, D):
    """dL/do for the map z = r / D + s o / sqrt(D) of :func:`apply`:
    s (H z - r) / (sqrt(D) r^T D^{-1} r) on free DOFs."""
    fr = _free(D)
    g = energy_loss_grad_z(r, Hz, D)
    out = np.zeros_like(r)
    out[fr] = scale(r, D) * g[fr] / np.sqrt(D[fr])
    return out


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step at step number t >= 1; returns (p, m, v) updated."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def pair_target(r, x, xstar, D):
    """Target of a training pair taken at a CG iterate x with residual r of
    H x = b, x* the solution: the network output o for which the map of
    :func:`apply` gives z = x* - x (= H^{-1} r), i.e.
    o = sqrt(D) (x* - x - r / D) / s on free DOFs, 0 elsewhere."""
    fr = _free(D)
    t = np.zeros_like(r)
    t[fr] = np.sqrt(D[fr]) * (xstar[fr] - x[fr] - r[fr] / D[fr]) / scale(r, D)
    return t
