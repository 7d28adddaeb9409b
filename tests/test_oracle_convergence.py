"""Pins of the oracle's transfers against the error bounds of the kinematic
transfer analysis (App. A, "Error Bounds"): the two-hop weights
T_ip = sum_c w_cp w_ic of the linear particle -> centre -> node path against
the quadratic B-spline (B2) weights beta_ip of APIC.

* The oracle's unload node velocity is, by construction, the two-hop P2G
  average v_i^(2hop) = sum_p alpha_p v_p(i) / sum_p alpha_p with
  alpha_p = m_p T_ip and v_p(i) = v_p + G_p (x_i - x_p); it is compared with
  that formula evaluated by brute force over particles.
* The oracle's load (N2C then C2P) gives v_p^(2hop) = sum_i T_ip v_i.
* Both T and beta are partitions of unity with linear reproduction, and
  beta_ip <= 1.5^d T_ip (the paper's comparison of the two kernels).
* On a smooth velocity field, |v^(2hop) - v^(beta)| stays below the
  theorems' bounds C(d) |H_v| dx^2 (P2G, C(d) = (1 + 1.5^d) 1.5^2 d) and
  1.5^2 d |H_v| dx^2 (G2P), and falls by about 4 when dx halves (second
  order).

The B2 weights are written here from their definition (tensor product of
the quadratic B-spline N(t) = 3/4 - t^2 for |t| < 1/2, (3/2 - |t|)^2 / 2 for
1/2 <= |t| < 3/2, 0 beyond); nothing of the oracle is reused for them."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2602_07853_amd import scenes

K = 2.0 * np.pi * 0.8   # wave number of the smooth field (per metre)


def field(x):
    """Smooth velocity field, its gradient G_ab = dv_a/dx_b and a bound on
    its componentwise Hessian (max over components of the max |d2 v_a|)."""
    sx, sy, sz = np.sin(K * x[:, 0]), np.sin(K * x[:, 1]), np.sin(K * x[:, 2])
    cx, cy, cz = np.cos(K * x[:, 0]), np.cos(K * x[:, 1]), np.cos(K * x[:, 2])
    v = np.stack([sy * cz, sz * cx, sx * cy], axis=1) * 0.3
    G = np.zeros((len(x), 3, 3))
    G[:, 0, 1] = 0.3 * K * cy * cz
    G[:, 0, 2] = -0.3 * K * sy * sz
    G[:, 1, 2] = 0.3 * K * cz * cx
    G[:, 1, 0] = -0.3 * K * sz * sx
    G[:, 2, 0] = 0.3 * K * cx * cy
    G[:, 2, 1] = -0.3 * K * sx * sy
    hess_bound = 0.3 * K * K  # each second derivative of a product of two unit trig factors
    return v, G.reshape(-1, 9), hess_bound


def b2(t):
    a = np.abs(t)
    return np.where(a < 0.5, 0.75 - a * a, np.where(a < 1.5, 0.5 * (1.5 - a) ** 2, 0.0))


def b2_weights(x, dx):
    """Nodes and tensor-product B2 weights of each particle (4 candidates per
    axis, zero weights included): ids [n, 64, 3], w [n, 64]."""
    base = np.floor(x / dx).astype(int) - 1
    offs = np.array([(a, b, c) for a in range(4) for b in range(4) for c in range(4)])
    ids = base[:, None, :] + offs[None, :, :]
    w = np.prod(b2((x[:, None, :] - ids * dx) / dx), axis=2)
    return ids, w


def twohop_weights(x, dx):
    """Nodes and two-hop weights T_ip = sum_c w_cp w_ic: the 2x2x2 dual-grid
    centres c around x_p with trilinear hat weights, and the 8 corners of
    each with w_ic = 1/8.  ids [n, 64, 3] (repeated nodes allowed), w [n, 64]."""
    xi = x / dx - 0.5
    b = np.floor(xi).astype(int)
    f = xi - b
    ids, ws = [], []
    for dc in [(a, bb, c) for a in range(2) for bb in range(2) for c in range(2)]:
        dc = np.array(dc)
        wc = np.prod(np.where(dc[None, :] == 1, f, 1.0 - f), axis=1)
        cell = b + dc
        for dn in [(a, bb, c) for a in range(2) for bb in range(2) for c in range(2)]:
            ids.append(cell + np.array(dn))
            ws.append(wc / 8.0)
    return np.stack(ids, 1), np.stack(ws, 1)


def scene(n, lo_frac=0.25, hi_frac=0.75, seed=5):
    dx = 1.0 / n
    lo, hi = int(n * lo_frac), int(n * hi_frac)
    cells = scenes.box_cells((lo, lo, lo), (hi, hi, hi))
    rng = np.random.Generator(np.random.PCG64(seed))
    x = scenes.fill_cells(cells, dx, 2, rng)
    mats = [scenes.material(scenes.NEOHOOKEAN, 1e5, 0.3)]
    p = scenes.make_particles(x, np.zeros(len(x), np.int32), mats, dx, 8)
    v, G, hb = field(x)
    p["v"], p["G"] = v, G
    omats = [O.Material(m["model"], m["E"], m["nu"], m["plastic"], m["yield_stress"], m["friction_deg"])
             for m in mats]
    return dx, lo, hi, p, omats, hb


def node_ids(n, ids):
    m = n + 1
    return (ids[..., 0] * m + ids[..., 1]) * m + ids[..., 2]


def test_weights_partition_of_unity_and_kernel_comparison():
    rng = np.random.default_rng(1)
    dx = 1.0 / 16
    x = rng.uniform(0.3, 0.7, size=(500, 3))
    for ids, w in (twohop_weights(x, dx), b2_weights(x, dx)):
        assert np.allclose(w.sum(1), 1.0, atol=1e-14)
        xr = np.einsum("pk,pkd->pd", w, ids * dx)
        assert np.allclose(xr, x, atol=1e-14)
    idt, wt = twohop_weights(x, dx)
    idb, wb = b2_weights(x, dx)
    # beta_ip <= 1.5^3 T_ip node by node
    for p in range(len(x)):
        T = {}
        for k in range(64):
            key = tuple(idt[p, k])
            T[key] = T.get(key, 0.0) + wt[p, k]
        for k in range(64):
            if wb[p, k] > 0.0:
                assert wb[p, k] <= 1.5 ** 3 * T.get(tuple(idb[p, k]), 0.0) * (1 + 1e-12)


def p2g_errors(n):
    dx, lo, hi, p, mats, hb = scene(n)
    g = O.Grid(n, dx)
    u = O.unload(g, p, mats)
    assert u["rc"] == 0
    x, m, v, G = p["x"], p["m"], p["v"], p["G"].reshape(-1, 3, 3)
    nn = (n + 1) ** 3

    def average(ids, w):
        nid = node_ids(n, ids)
        xi = ids * dx
        vpi = v[:, None, :] + np.einsum("pab,pkb->pka", G, xi - x[:, None, :])
        num = np.zeros((nn, 3))
        den = np.zeros(nn)
        np.add.at(num, nid.ravel(), (m[:, None] * w)[..., None].reshape(-1, 1) * vpi.reshape(-1, 3))
        np.add.at(den, nid.ravel(), (m[:, None] * w).ravel())
        return num, den

    num_t, den_t = average(*twohop_weights(x, dx))
    num_b, den_b = average(*b2_weights(x, dx))
    # interior nodes: every particle within the B2 support (1.5 dx) lies in the filled box
    ii = np.arange(n + 1)
    inner = (ii >= lo + 2) & (ii <= hi - 2)
    mask = (inner[:, None, None] & inner[None, :, None] & inner[None, None, :]).ravel()
    v2 = num_t[mask] / den_t[mask][:, None]
    vb = num_b[mask] / den_b[mask][:, None]
    # the oracle's unload node velocity is the two-hop average
    assert np.allclose(u["vi"][mask], v2, rtol=0, atol=1e-13)
    assert np.allclose(u["mi"][mask], den_t[mask], rtol=1e-13)
    return np.max(np.linalg.norm(v2 - vb, axis=1)), hb, dx


def test_p2g_two_hop_vs_b2_second_order():
    errs = []
    for n in (16, 32, 64):
        e, hb, dx = p2g_errors(n)
        bound = (1 + 1.5 ** 3) * 1.5 ** 2 * 3 * hb * dx * dx
        print(f"[P15] P2G n={n}: max |v_2hop - v_B2| = {e:.3e}, bound {bound:.3e}")
        assert e <= bound
        errs.append(e)
    for a, b in zip(errs, errs[1:]):
        assert 3.0 <= a / b <= 5.0, errs


def g2p_errors(n):
    dx, lo, hi, p, mats, hb = scene(n)
    g = O.Grid(n, dx)
    u = O.unload(g, p, mats)
    ii = np.arange(n + 1) * dx
    X = np.stack(np.meshgrid(ii, ii, ii, indexing="ij"), -1).reshape(-1, 3)
    vnode, _, _ = field(X)
    vnode = np.where(u["mi"][:, None] > 0, vnode, 0.0)
    out = O.load(g, 0.0, u["mc"], vnode, p, mats)
    assert out["rc"] == 0
    x = p["x"]
    idb, wb = b2_weights(x, dx)
    vb = np.einsum("pk,pka->pa", wb, vnode[node_ids(n, idb)])
    # particles whose B2 support lies in the nodes carrying velocity
    inside = np.all((x >= (lo + 2) * dx) & (x <= (hi - 2) * dx), axis=1)
    # the oracle's load velocity is the two-hop average of the node values
    idt, wt = twohop_weights(x, dx)
    vt = np.einsum("pk,pka->pa", wt, vnode[node_ids(n, idt)])
    assert np.allclose(out["v"], vt, rtol=0, atol=1e-13)
    return np.max(np.linalg.norm(out["v"][inside] - vb[inside], axis=1)), hb, dx


def test_g2p_two_hop_vs_b2_second_order():
    errs = []
    for n in (16, 32, 64):
        e, hb, dx = g2p_errors(n)
        bound = 1.5 ** 2 * 3 * hb * dx * dx
        print(f"[P15] G2P n={n}: max |v_2hop - v_B2| = {e:.3e}, bound {bound:.3e}")
        assert e <= bound
        errs.append(e)
    for a, b in zip(errs, errs[1:]):
        assert 3.0 <= a / b <= 5.0, errs
