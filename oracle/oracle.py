"""NumPy/ctypes front end of the FP64 CPU oracle — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product path (the HIP library under
``paper_2602_07853_amd``) never imports it.

The C++ library (``oracle/liboracle.so``) holds every formula; this file only
marshals NumPy arrays.  Grid layout: dense ``N^3`` cells and ``(N+1)^3``
nodes, index ``(i*M + j)*M + k`` with ``M = N`` (cells) or ``N+1`` (nodes),
origin 0, spacing ``dx``.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

NEOHOOKEAN, FIXED_COROTATED, HENCKY, WATER = 0, 1, 2, 3
PLASTIC_NONE, PLASTIC_VON_MISES, PLASTIC_DRUCKER_PRAGER = 0, 1, 2
BC_STICKY_BOX, BC_MOVING_BOX, BC_SLIP_PLANE = 0, 1, 2

OK, ERR_ARG, ERR_DOMAIN, ERR_NOT_CONVERGED, ERR_LINESEARCH, ERR_OUTSIDE = 0, -1, -2, -3, -4, -5


class _Material(C.Structure):
    _fields_ = [("model", C.c_int32), ("plastic", C.c_int32), ("mu", C.c_double),
                ("lam", C.c_double), ("yield_stress", C.c_double), ("friction_deg", C.c_double)]


class _Grid(C.Structure):
    _fields_ = [("n", C.c_int32), ("dx", C.c_double)]


class _BC(C.Structure):
    _fields_ = [("kind", C.c_int32), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("velocity", C.c_double * 3)]


class _Opts(C.Structure):
    _fields_ = [("newton_rtol", C.c_double), ("pcg_rtol", C.c_double), ("armijo_c", C.c_double),
                ("max_newton", C.c_int32), ("max_pcg", C.c_int32), ("max_ls", C.c_int32),
                ("fixed_point_plasticity", C.c_int32), ("vbd_sweeps", C.c_int32),
                ("block_jacobi", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("pcg_iters_total", C.c_int32),
                ("ls_halvings", C.c_int32), ("g0_norm", C.c_double), ("g_norm", C.c_double),
                ("energy", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError("oracle library missing: run __graft_entry__.build() first")
        _lib = C.CDLL(_LIB_PATH)
        _lib.or_psi.restype = C.c_double
    return _lib


def lame(E: float, nu: float):
    """Lame parameters from Young's modulus and Poisson ratio."""
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam


@dataclass
class Material:
    model: int
    E: float
    nu: float
    plastic: int = PLASTIC_NONE
    yield_stress: float = 0.0
    friction_deg: float = 0.0

    def c(self) -> _Material:
        # J-based water (Sec. 3, Water): E is the bulk modulus kappa, carried
        # in the lambda slot; the table of the paper's examples likewise lists
        # E in place of kappa for water
        mu, lam = (0.0, self.E) if self.model == WATER else lame(self.E, self.nu)
        return _Material(self.model, self.plastic, mu, lam, self.yield_stress, self.friction_deg)


@dataclass
class BC:
    kind: int
    lo: tuple
    hi: tuple
    velocity: tuple = (0.0, 0.0, 0.0)

    def c(self) -> _BC:
        return _BC(self.kind, (C.c_double * 3)(*self.lo), (C.c_double * 3)(*self.hi),
                   (C.c_double * 3)(*self.velocity))


@dataclass
class SolverOpts:
    newton_rtol: float = 1e-8
    pcg_rtol: float = 1e-8
    armijo_c: float = 1e-4
    max_newton: int = 50
    max_pcg: int = 20000
    max_ls: int = 40
    fixed_point_plasticity: int = 0
    vbd_sweeps: int = 0
    block_jacobi: int = 0

    def c(self) -> _Opts:
        return _Opts(self.newton_rtol, self.pcg_rtol, self.armijo_c, self.max_newton,
                     self.max_pcg, self.max_ls, self.fixed_point_plasticity, self.vbd_sweeps,
                     self.block_jacobi)


def _p(a: np.ndarray, ctype=C.c_double):
    return a.ctypes.data_as(C.POINTER(ctype))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _mats(mats):
    arr = (_Material * len(mats))(*[m.c() for m in mats])
    return arr


# ---------------------------------------------------------------- per point
def psi(mat: Material, F):
    return lib().or_psi(C.byref(mat.c()), _p(_f64(F)))


def piola(mat: Material, F):
    P = np.zeros(9)
    rc = lib().or_piola(C.byref(mat.c()), _p(_f64(F)), _p(P))
    return P.reshape(3, 3), rc


def tau(mat: Material, F):
    T = np.zeros(9)
    rc = lib().or_tau(C.byref(mat.c()), _p(_f64(F)), _p(T))
    return T.reshape(3, 3), rc


def dpdf(mat: Material, F):
    A = np.zeros(81)
    rc = lib().or_dpdf(C.byref(mat.c()), _p(_f64(F)), _p(A))
    return A.reshape(9, 9), rc


def stretch(mat: Material, tau_):
    S = np.zeros(9)
    rc = lib().or_stretch(C.byref(mat.c()), _p(_f64(tau_)), _p(S))
    return S.reshape(3, 3), rc


def svd3(F):
    U, s, V = np.zeros(9), np.zeros(3), np.zeros(9)
    lib().or_svd3(_p(_f64(F)), _p(U), _p(s), _p(V))
    return U.reshape(3, 3), s, V.reshape(3, 3)


def sym_eigen(A):
    A = _f64(A)
    n = A.shape[0]
    w, Q = np.zeros(n), np.zeros(n * n)
    lib().or_sym_eigen(n, _p(A), _p(w), _p(Q))
    return w, Q.reshape(n, n)


def project_psd(A):
    A = _f64(A).copy()
    lib().or_project_psd(A.shape[0], _p(A))
    return A


def cardano_largest(p, q):
    m = C.c_double()
    lib().or_cardano_largest(C.c_double(p), C.c_double(q), C.byref(m))
    return m.value


def plastic_project(mat: Material, F):
    F = _f64(F).reshape(9).copy()
    acc = C.c_double(0.0)
    rc = lib().or_plastic_project(C.byref(mat.c()), _p(F), C.byref(acc))
    return F.reshape(3, 3), acc.value, rc


# ---------------------------------------------------------------- grid stages
@dataclass
class Grid:
    n: int
    dx: float

    def c(self):
        return _Grid(self.n, self.dx)

    @property
    def ncell(self):
        return self.n ** 3

    @property
    def nnode(self):
        return (self.n + 1) ** 3


def unload(grid: Grid, parts: dict, mats):
    """Alg. 2.  ``parts`` holds x, v, G, F, m, V, mat arrays (particle-major)."""
    nc, nn, K = grid.ncell, grid.nnode, len(mats)
    out = dict(mc=np.zeros(nc), vc=np.zeros((nc, 3)), Gc=np.zeros((nc, 9)),
               Vck=np.zeros((K, nc)), tauck=np.zeros((K, nc, 9)), mi=np.zeros(nn),
               vi=np.zeros((nn, 3)))
    x, v, G, F = (_f64(parts[k]) for k in ("x", "v", "G", "F"))
    m, V = _f64(parts["m"]), _f64(parts["V"])
    mat = np.ascontiguousarray(parts["mat"], dtype=np.int32)
    rc = lib().or_unload(C.byref(grid.c()), C.c_int64(len(m)), _p(x), _p(v), _p(G), _p(F), _p(m),
                         _p(V), _p(mat, C.c_int32), K, _mats(mats), _p(out["mc"]), _p(out["vc"]),
                         _p(out["Gc"]), _p(out["Vck"]), _p(out["tauck"]), _p(out["mi"]),
                         _p(out["vi"]))
    out["rc"] = rc
    return out


def node_bcs(grid: Grid, mi, bcs, time=0.0):
    """Dirichlet sets: fixed [nnode] uint8 with bit a set when velocity
    component a is prescribed, vfix [nnode, 3] the prescribed values."""
    nn = grid.nnode
    fixed = np.zeros(nn, dtype=np.uint8)
    vfix = np.zeros((nn, 3))
    arr = (_BC * max(len(bcs), 1))(*[b.c() for b in bcs])
    rc = lib().or_node_bcs(C.byref(grid.c()), _p(_f64(mi)), len(bcs), arr, C.c_double(time),
                           _p(fixed, C.c_uint8), _p(vfix))
    if rc != OK:
        raise ValueError(f"or_node_bcs: invalid boundary condition (rc {rc})")
    return fixed, vfix


def fixed_components(fixed):
    """[nnode, 3] bool: component a of the node is prescribed."""
    return ((np.asarray(fixed, dtype=np.uint8)[:, None] >> np.arange(3, dtype=np.uint8)) & 1).astype(bool)


def reconstruct(grid: Grid, mats, Vck, tauck):
    S = np.zeros((len(mats), grid.ncell, 9))
    rc = lib().or_reconstruct(C.byref(grid.c()), len(mats), _mats(mats), _p(_f64(Vck)),
                              _p(_f64(tauck)), _p(S))
    return S, rc


def energy_grad(grid: Grid, mats, dt, mi, vhat, fixed, Vck, Sck, v):
    E = C.c_double()
    g = np.zeros((grid.nnode, 3))
    rc = lib().or_energy_grad(C.byref(grid.c()), len(mats), _mats(mats), C.c_double(dt),
                              _p(_f64(mi)), _p(_f64(vhat)),
                              _p(np.ascontiguousarray(fixed, dtype=np.uint8), C.c_uint8),
                              _p(_f64(Vck)), _p(_f64(Sck)), _p(_f64(v)), C.byref(E), _p(g))
    return E.value, g, rc


def tangent(grid: Grid, mats, dt, Vck, Sck, v, project=True):
    A = np.zeros((grid.ncell, 81))
    rc = lib().or_tangent(C.byref(grid.c()), len(mats), _mats(mats), C.c_double(dt),
                          _p(_f64(Vck)), _p(_f64(Sck)), _p(_f64(v)), int(project), _p(A))
    return A, rc


def hv(grid: Grid, mc, mi, fixed, Abar, u):
    Hu = np.zeros((grid.nnode, 3))
    lib().or_hv(C.byref(grid.c()), _p(_f64(mc)), _p(_f64(mi)),
                _p(np.ascontiguousarray(fixed, dtype=np.uint8), C.c_uint8), _p(_f64(Abar)),
                _p(_f64(u)), _p(Hu))
    return Hu


def jacobi_diag(grid: Grid, mc, mi, fixed, Abar):
    """Diagonal of the Newton matrix H on free DOFs (0 elsewhere), [nnode, 3]."""
    D = np.zeros((grid.nnode, 3))
    lib().or_jacobi_diag(C.byref(grid.c()), _p(_f64(mc)), _p(_f64(mi)),
                         _p(np.ascontiguousarray(fixed, dtype=np.uint8), C.c_uint8), _p(_f64(Abar)),
                         _p(D))
    return D


def block_jacobi(grid: Grid, mc, mi, fixed, Abar):
    """Inverted 3x3 node blocks of the Newton matrix H on free nodes (0
    elsewhere), [nnode, 3, 3]."""
    B = np.zeros((grid.nnode, 3, 3))
    rc = lib().or_block_jacobi(C.byref(grid.c()), _p(_f64(mc)), _p(_f64(mi)),
                               _p(np.ascontiguousarray(fixed, dtype=np.uint8), C.c_uint8), _p(_f64(Abar)),
                               _p(B))
    return B, rc


def plastic_base(grid: Grid, mats, dt, Vck, S0, v):
    """Fixed-point plasticity base at node velocity v (Sec. 7, Fixed-Point
    Plasticity): the return-mapped (I + dt G_c(v)) S0, mapped back by
    (I + dt G_c(v))^{-1}, where a plastic centre yields; S0 elsewhere."""
    Se = np.zeros((len(mats), grid.ncell, 9))
    rc = lib().or_plastic_base(C.byref(grid.c()), len(mats), _mats(mats), C.c_double(dt),
                               _p(_f64(Vck)), _p(_f64(S0)), _p(_f64(v)), _p(Se))
    return Se, rc


def explicit_force(grid: Grid, Vck, tauck):
    f = np.zeros((grid.nnode, 3))
    K = np.asarray(Vck).shape[0]
    lib().or_explicit_force(C.byref(grid.c()), K, _p(_f64(Vck)), _p(_f64(tauck)), _p(f))
    return f


def solve(grid: Grid, mats, dt, mc, mi, vhat, fixed, Vck, Sck, opts: SolverOpts):
    v = np.zeros((grid.nnode, 3))
    st = _Stats()
    rc = lib().or_solve(C.byref(grid.c()), len(mats), _mats(mats), C.c_double(dt), _p(_f64(mc)),
                        _p(_f64(mi)), _p(_f64(vhat)),
                        _p(np.ascontiguousarray(fixed, dtype=np.uint8), C.c_uint8),
                        _p(_f64(Vck)), _p(_f64(Sck)), C.byref(opts.c()), _p(v), C.byref(st))
    stats = {k: getattr(st, k) for k, _ in _Stats._fields_}
    return v, stats, rc


def node_to_centre(grid: Grid, mc, vnode):
    vc, Gc = np.zeros((grid.ncell, 3)), np.zeros((grid.ncell, 9))
    lib().or_node_to_centre(C.byref(grid.c()), _p(_f64(mc)), _p(_f64(vnode)), _p(vc), _p(Gc))
    return vc, Gc


def load(grid: Grid, dt, mc, vnode, parts: dict, mats):
    """Alg. 4.  Returns a new particle dict (input untouched)."""
    out = {k: np.array(v, dtype=np.float64 if k != "mat" else np.int32, copy=True)
           for k, v in parts.items()}
    if "eps" not in out:
        out["eps"] = np.zeros(len(out["m"]))
    mat = np.ascontiguousarray(out["mat"], dtype=np.int32)
    rc = lib().or_load(C.byref(grid.c()), C.c_double(dt), _p(_f64(mc)), _p(_f64(vnode)),
                       C.c_int64(len(out["m"])), _p(mat, C.c_int32), _mats(mats), _p(out["x"]),
                       _p(out["v"]), _p(out["G"]), _p(out["F"]), _p(out["eps"]))
    out["rc"] = rc
    return out


def step(grid: Grid, mats, dt, gravity, bcs, time, opts: SolverOpts, parts: dict):
    """Alg. 1 on a copy of ``parts``; returns (new parts, solver stats, node velocity, rc)."""
    out = {k: np.array(v, dtype=np.float64 if k != "mat" else np.int32, copy=True)
           for k, v in parts.items()}
    if "eps" not in out:
        out["eps"] = np.zeros(len(out["m"]))
    st = _Stats()
    vnode = np.zeros((grid.nnode, 3))
    arr = (_BC * max(len(bcs), 1))(*[b.c() for b in bcs])
    grav = (C.c_double * 3)(*gravity)
    rc = lib().or_step(C.byref(grid.c()), len(mats), _mats(mats), C.c_double(dt), grav, len(bcs),
                       arr, C.c_double(time), C.byref(opts.c()), C.c_int64(len(out["m"])),
                       _p(out["x"]), _p(out["v"]), _p(out["G"]), _p(out["F"]), _p(_f64(out["m"])),
                       _p(_f64(out["V"])), _p(np.ascontiguousarray(out["mat"], dtype=np.int32),
                                              C.c_int32),
                       _p(out["eps"]), C.byref(st), _p(vnode))
    stats = {k: getattr(st, k) for k, _ in _Stats._fields_}
    return out, stats, vnode, rc


def load_flip(grid: Grid, dt, mc, vnode, vnode_old, parts: dict, mats, flip):
    """Load with the FLIP/PIC transfer (Sec. 3, Degradation to FLIP/PIC).
    Returns a new particle dict (input untouched)."""
    out = {k: np.array(v, dtype=np.float64 if k != "mat" else np.int32, copy=True)
           for k, v in parts.items()}
    if "eps" not in out:
        out["eps"] = np.zeros(len(out["m"]))
    mat = np.ascontiguousarray(out["mat"], dtype=np.int32)
    rc = lib().or_load_flip(C.byref(grid.c()), C.c_double(dt), _p(_f64(mc)), _p(_f64(vnode)),
                            _p(_f64(vnode_old)), C.c_double(flip), C.c_int64(len(out["m"])),
                            _p(mat, C.c_int32), _mats(mats), _p(out["x"]), _p(out["v"]),
                            _p(out["G"]), _p(out["F"]), _p(out["eps"]))
    out["rc"] = rc
    return out


def step_flip(grid: Grid, mats, dt, gravity, bcs, time, parts: dict, flip, opts=None):
    """One step with the FLIP/PIC transfer (Sec. 3, Degradation to FLIP/PIC),
    composed from the pinned stages: the unload without the affine terms (the
    particles' G does not enter the grid, so centre and node velocities are
    plain weighted averages), the Dirichlet sets and vhat of Alg. 1, then the
    implicit solve (``opts``) or, with ``opts`` None, the explicit update of
    Eq. explicitforce, and the FLIP/PIC load with the unloaded node velocity
    as v^n.  Returns (new parts, node velocity, rc)."""
    p0 = dict(parts)
    p0["G"] = np.zeros_like(np.asarray(parts["G"], dtype=np.float64))
    u = unload(grid, p0, mats)
    if u["rc"] not in (OK, ERR_DOMAIN):
        return None, None, u["rc"]
    fixed, vfix = node_bcs(grid, u["mi"], bcs, time)
    act = u["mi"] > 0
    fx = fixed_components(fixed)
    free = act[:, None] & ~fx
    vhat = np.where(fx, vfix,
                    np.where(act[:, None], u["vi"] + dt * np.asarray(gravity, dtype=np.float64), 0.0))
    if opts is None:
        f = explicit_force(grid, u["Vck"], u["tauck"])
        vnew = vhat.copy()
        mi3 = np.broadcast_to(u["mi"][:, None], f.shape)
        vnew[free] += dt * f[free] / mi3[free]
    else:
        S, rc = reconstruct(grid, mats, u["Vck"], u["tauck"])
        if rc not in (OK, ERR_DOMAIN):
            return None, None, rc
        vnew, _, rc = solve(grid, mats, dt, u["mc"], u["mi"], vhat, fixed, u["Vck"], S, opts)
        if rc != OK:
            return None, None, rc
    out = load_flip(grid, dt, u["mc"], vnew, u["vi"], parts, mats, flip)
    return out, vnew, out["rc"]


def step_explicit(grid: Grid, mats, dt, gravity, bcs, time, parts: dict):
    """Explicit branch of the Integrate algorithm (Sec. 4 opening, Eq.
    explicitforce) between unload and load, on a copy of ``parts``; returns
    (new parts, node velocity, rc)."""
    out = {k: np.array(v, dtype=np.float64 if k != "mat" else np.int32, copy=True)
           for k, v in parts.items()}
    if "eps" not in out:
        out["eps"] = np.zeros(len(out["m"]))
    vnode = np.zeros((grid.nnode, 3))
    arr = (_BC * max(len(bcs), 1))(*[b.c() for b in bcs])
    grav = (C.c_double * 3)(*gravity)
    rc = lib().or_step_explicit(C.byref(grid.c()), len(mats), _mats(mats), C.c_double(dt), grav,
                                len(bcs), arr, C.c_double(time), C.c_int64(len(out["m"])),
                                _p(out["x"]), _p(out["v"]), _p(out["G"]), _p(out["F"]),
                                _p(_f64(out["m"])), _p(_f64(out["V"])),
                                _p(np.ascontiguousarray(out["mat"], dtype=np.int32), C.c_int32),
                                _p(out["eps"]), _p(vnode))
    return out, vnode, rc


# ---------------------------------------------------------------- scene glue
def materials_of(scene):
    return [Material(m["model"], m["E"], m["nu"], m["plastic"], m["yield_stress"],
                     m["friction_deg"]) for m in scene.materials]


def bcs_of(scene):
    return [BC(b["kind"], tuple(b["lo"]), tuple(b["hi"]), tuple(b["velocity"])) for b in scene.bcs]


def grid_of(scene):
    return Grid(scene.n, scene.dx)
