"""FP64 oracle of the learned preconditioner's input features and output
map — TEST INFRASTRUCTURE ONLY (tests, smoke, bench CPU-baseline leg).

The network runs on a dense box over all grid nodes of an N^3-cell grid:
voxel (i, j, k) is node (i, j, k), each axis padded from N + 1 up to a
multiple of 8 (padding voxels are zero).  With D the Jacobi diagonal of the
Newton matrix (zero off the free DOFs) and r a residual:

  s^2     = sum over free DOFs of r^2 / D, divided by the number of free DOFs
  x[v]    = (r_v / (s sqrt(D_v)) (3 channels), log(mean_a D_v,a / Dref), 1,
             11 zero channels) on free nodes, 0 elsewhere; Dref = mean over
             free nodes of mean_a D_v,a
  z_v     = r_v / D_v + s o_v / sqrt(D_v) on free nodes, 0 elsewhere,

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
    return np.all(D > 0.0, axis=1)


def scale(r, D):
    fr = _free(D)
    s2 = np.sum(r[fr] ** 2 / D[fr])
    return np.sqrt(max(s2 / (3.0 * max(int(fr.sum()), 1)), 1e-300))


def features(n: int, r, D):
    """Network input [X, Y, Z, 16] for node vector r [(n+1)^3, 3]."""
    fr = _free(D)
    sc = scale(r, D)
    dmean = np.where(fr, D.mean(axis=1), 1.0)
    dref = dmean[fr].mean() if fr.any() else 1.0
    f = np.zeros(((n + 1) ** 3, U.IN_CH))
    f[fr, 0:3] = r[fr] / (sc * np.sqrt(D[fr]))
    f[fr, 3] = np.log(dmean[fr] / dref)
    f[fr, 4] = 1.0
    X = box_dims(n)
    box = np.zeros(X + (U.IN_CH,))
    box[:n + 1, :n + 1, :n + 1] = f.reshape(n + 1, n + 1, n + 1, U.IN_CH)
    return box


def apply(params, n: int, r, D, rnd=U._ident):
    """z = r / D + s o / sqrt(D) on free nodes (``rnd`` as in unet.forward,
    also applied to the stored network input)."""
    fr = _free(D)
    sc = scale(r, D)
    x = rnd(features(n, r, D))
    o = U.forward(params, x, rnd=rnd)[:n + 1, :n + 1, :n + 1, :3].reshape(-1, 3)
    z = np.zeros_like(r)
    z[fr] = r[fr] / D[fr] + sc * o[fr] / np.sqrt(D[fr])
    return z
