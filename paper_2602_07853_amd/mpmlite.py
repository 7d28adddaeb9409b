"""Thin ctypes binding of ``libmpmlite.so`` (the C-ABI in ``include/mpmlite.h``).

Argument marshalling only: every step of the implicit path runs in the HIP
kernels of the library.  PyTorch provides device memory and the stream.
There is no CPU fallback: constructing a :class:`Context` without the built
library or without a GPU raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpmlite.so")

F32, F64 = 0, 1
PRECOND_JACOBI, PRECOND_BLOCK_JACOBI, PRECOND_LEARNED, PRECOND_MULTIGRID = 0, 1, 2, 3
MG_MAX_LEVELS = 6
TRANSFER_APIC, TRANSFER_FLIP_PIC = 0, 1
PLASTICITY_AFTER_SOLVE, PLASTICITY_FIXED_POINT = 0, 1
NEOHOOKEAN, FIXED_COROTATED, HENCKY = 0, 1, 2
BC_STICKY_BOX, BC_MOVING_BOX, BC_SLIP_PLANE = 0, 1, 2

STATUS = {0: "OK", -1: "INVALID_ARG", -2: "HIP", -3: "OOM", -4: "NOT_CONVERGED",
          -5: "LINESEARCH", -6: "NONFINITE", -7: "DOMAIN", -8: "STATE"}

FIELDS = dict(mass_c=(0, "cell", 1), vel_c=(1, "cell", 3), grad_c=(2, "cell", 9),
              vol_ck=(3, "cellk", 1), tau_ck=(4, "cellk", 9), s_ck=(5, "cellk", 9),
              abar=(6, "cell", 81), mass_i=(7, "node", 1), vel_i=(8, "node", 3),
              vhat=(9, "node", 3), fixed=(10, "node", 1), v=(11, "node", 3), diag=(12, "node", 3),
              block_diag=(13, "node", 9))


class MplError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mpmlite {STATUS.get(status, status)} ({status}): {msg}")
        self.status = status


class _Grid(C.Structure):
    _fields_ = [("dx", C.c_double), ("origin", C.c_double * 3), ("dims", C.c_int32 * 3)]


class _Material(C.Structure):
    _fields_ = [("model", C.c_int32), ("plastic", C.c_int32), ("E", C.c_double), ("nu", C.c_double),
                ("rho", C.c_double), ("yield_stress", C.c_double), ("friction_deg", C.c_double)]


class _Opts(C.Structure):
    _fields_ = [("hv_precision", C.c_int32), ("precond", C.c_int32), ("newton_rtol", C.c_double),
                ("pcg_rtol", C.c_double), ("max_newton", C.c_int32), ("max_pcg", C.c_int32),
                ("max_ls", C.c_int32), ("armijo_c", C.c_double), ("pcg_check_every", C.c_int32),
                ("time_kernels", C.c_int32), ("warm_start", C.c_int32), ("transfer", C.c_int32),
                ("flip_ratio", C.c_double), ("plasticity", C.c_int32), ("plastic_anderson", C.c_int32),
                ("newton_forcing", C.c_double),
                ("vbd_sweeps", C.c_int32), ("mg_levels", C.c_int32), ("mg_smooth", C.c_int32),
                ("mg_coarse_sweeps", C.c_int32), ("mg_omega", C.c_double)]


class _Particles(C.Structure):
    _fields_ = [("n", C.c_int64), ("dtype", C.c_int32), ("x", C.c_void_p), ("v", C.c_void_p), ("F", C.c_void_p),
                ("G", C.c_void_p), ("m", C.c_void_p), ("V0", C.c_void_p), ("plastic", C.c_void_p),
                ("mat", C.c_void_p)]


class _BC(C.Structure):
    _fields_ = [("kind", C.c_int32), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("velocity", C.c_double * 3)]


class _Stats(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("pcg_iters", C.c_int32), ("ls_halvings", C.c_int32),
                ("fallbacks", C.c_int32), ("active_cells", C.c_int32), ("active_nodes", C.c_int32),
                ("free_dofs", C.c_int32), ("cell_blocks", C.c_int32), ("node_blocks", C.c_int32),
                ("g0_norm", C.c_double), ("g_norm", C.c_double), ("energy", C.c_double),
                ("hv_ms_total", C.c_double), ("hv_calls", C.c_int32), ("ms_unload", C.c_double),
                ("ms_reconstruct", C.c_double), ("ms_newton", C.c_double), ("ms_load", C.c_double),
                ("domain_events", C.c_int32), ("tangent_entries", C.c_int32),
                ("hv_model_bytes", C.c_double), ("pcg_per_newton", C.c_int32 * 8),
                ("graph_replays", C.c_int32), ("upd_calls", C.c_int32), ("upd_ms_total", C.c_double),
                ("upd_model_bytes", C.c_double), ("tangent_cells", C.c_int32), ("factored_cells", C.c_int32)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)


class _Allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", C.c_void_p)]


class TorchAllocator:
    """Device-memory callbacks backed by PyTorch's caching allocator, so that
    PyTorch owns the library's grid scratch (it shows in
    ``torch.cuda.memory_allocated``)."""

    def __init__(self, device, stream):
        self.device = device
        self.stream = stream
        self.live = {}

        def alloc(user, nbytes, hip_stream):
            try:
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            except Exception:
                return None
            self.live[ptr] = int(nbytes)
            return ptr

        def free(user, ptr, nbytes, hip_stream):
            if ptr in self.live:
                del self.live[ptr]
                try:
                    torch.cuda.caching_allocator_delete(ptr)
                except Exception:
                    pass

        self._alloc = _ALLOC_FN(alloc)
        self._free = _FREE_FN(free)
        self.c = _Allocator(self._alloc, self._free, None)

    @property
    def bytes_live(self) -> int:
        return sum(self.live.values())


_lib = None


def _stats_dict(st) -> dict:
    out = {}
    for k, _ in _Stats._fields_:
        v = getattr(st, k)
        out[k] = list(v) if k == "pcg_per_newton" else v
    return out


def library():
    """Load the in-tree HIP library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        lib = C.CDLL(LIB_PATH)
        lib.mpl_version.restype = C.c_char_p
        lib.mpl_last_error.restype = C.c_char_p
        lib.mpl_last_error.argtypes = [C.c_void_p]
        lib.mpl_destroy.argtypes = [C.c_void_p]
        _lib = lib
    return _lib


def _dptr(t: torch.Tensor, dtype) -> int:
    if t.numel() == 0:
        return 0
    if not t.is_cuda:
        raise ValueError("mpmlite needs device tensors")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} tensor, got {t.dtype}")
    return t.data_ptr()


def _particles(p: dict) -> _Particles:
    n = p["x"].shape[0]
    for k, shape in (("x", (n, 3)), ("v", (n, 3)), ("F", (n, 9)), ("G", (n, 9)), ("m", (n,)),
                     ("V", (n,)), ("mat", (n,))):
        if tuple(p[k].shape) != shape:
            raise ValueError(f"particle field {k} has shape {tuple(p[k].shape)}, want {shape}")
    pl = p.get("plastic")
    dt = p["x"].dtype
    if dt not in (torch.float64, torch.float32):
        raise ValueError(f"particle arrays must be float64 or float32, got {dt}")
    return _Particles(n, F64 if dt == torch.float64 else F32,
                      _dptr(p["x"], dt), _dptr(p["v"], dt),
                      _dptr(p["F"], dt), _dptr(p["G"], dt),
                      _dptr(p["m"], dt), _dptr(p["V"], dt),
                      _dptr(pl, dt) if pl is not None else None,
                      _dptr(p["mat"], torch.int32))


def _bcs(bcs):
    arr = (_BC * max(len(bcs), 1))()
    for i, b in enumerate(bcs):
        arr[i] = _BC(int(b["kind"]), (C.c_double * 3)(*b["lo"]), (C.c_double * 3)(*b["hi"]),
                     (C.c_double * 3)(*b.get("velocity", (0.0, 0.0, 0.0))))
    return arr


def particles_to_device(parts: dict, device="cuda", dtype=torch.float64) -> dict:
    """Copy a NumPy particle dict (x, v, G, F, m, V, mat[, eps]) to device
    tensors of ``dtype`` (float64, or float32 staged to FP64 by the library)."""
    out = {}
    for k in ("x", "v", "G", "F", "m", "V"):
        out[k] = torch.as_tensor(parts[k], dtype=torch.float64).to(dtype).contiguous().to(device)
    out["mat"] = torch.as_tensor(parts["mat"], dtype=torch.int32).contiguous().to(device)
    eps = parts.get("eps", parts.get("plastic"))
    n = out["x"].shape[0]
    out["plastic"] = (torch.as_tensor(eps, dtype=torch.float64) if eps is not None
                      else torch.zeros(n, dtype=torch.float64)).to(dtype).contiguous().to(device)
    return out


def default_opts(**kw) -> dict:
    o = dict(hv_precision=F32, precond=PRECOND_JACOBI, newton_rtol=1e-6, pcg_rtol=1e-6,
             max_newton=50, max_pcg=20000, max_ls=40, armijo_c=1e-4, pcg_check_every=16,
             time_kernels=0, warm_start=0, transfer=TRANSFER_APIC, flip_ratio=0.0,
             plasticity=PLASTICITY_AFTER_SOLVE, plastic_anderson=0, newton_forcing=0.0, vbd_sweeps=0,
             mg_levels=0, mg_smooth=0, mg_coarse_sweeps=0, mg_omega=0.0)
    o.update(kw)
    return o


class Context:
    """One simulation grid (dims multiples of 4) with its materials and solver options."""

    def __init__(self, dims, dx, materials, opts=None, origin=(0.0, 0.0, 0.0), stream=None,
                 torch_allocator=True):
        if not torch.cuda.is_available():
            raise RuntimeError("mpmlite runs on the GPU only; no device is visible")
        lib = library()
        self._lib = lib
        self.dims = tuple(int(d) for d in dims)
        self.dx = float(dx)
        self.nmat = len(materials)
        g = _Grid(self.dx, (C.c_double * 3)(*origin), (C.c_int32 * 3)(*self.dims))
        mats = (_Material * len(materials))()
        for i, m in enumerate(materials):
            mats[i] = _Material(int(m["model"]), int(m.get("plastic", 0)), float(m["E"]),
                                float(m["nu"]), float(m.get("rho", 1000.0)),
                                float(m.get("yield_stress", 0.0)), float(m.get("friction_deg", 0.0)))
        self.opts = default_opts(**(opts or {}))
        o = self._copts()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        ctx = C.c_void_p()
        # grid scratch from PyTorch's caching allocator (or hipMalloc in the library)
        self.allocator = TorchAllocator(torch.cuda.current_device(), self.stream) if torch_allocator else None
        st = lib.mpl_create_with_allocator(C.byref(g), mats, len(materials), C.byref(o),
                                           C.c_void_p(self.stream.cuda_stream),
                                           C.byref(self.allocator.c) if self.allocator else None,
                                           C.byref(ctx))
        if st != 0:
            raise MplError(st, "mpl_create failed")
        self._ctx = ctx

    def _copts(self):
        # every struct field by name, so an added option cannot arrive as zero
        o = self.opts
        return _Opts(**{name: (int(o[name]) if ctype is C.c_int32 else float(o[name]))
                        for name, ctype in _Opts._fields_})

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.mpl_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st != 0:
            msg = self._lib.mpl_last_error(self._ctx)
            raise MplError(st, f"{what}: {msg.decode() if msg else ''}")

    def set_opts(self, **kw):
        self.opts.update(kw)
        self._check(self._lib.mpl_set_opts(self._ctx, C.byref(self._copts())), "mpl_set_opts")

    # ------------------------------------------------------------ full step
    def step(self, parts_in: dict, parts_out: dict, dt, gravity=(0.0, 0.0, 0.0), bcs=(), time=0.0):
        pi, po = _particles(parts_in), _particles(parts_out)
        st = _Stats()
        rc = self._lib.mpl_step(self._ctx, C.byref(pi), C.byref(po), C.c_double(dt),
                                (C.c_double * 3)(*gravity), _bcs(list(bcs)), len(bcs),
                                C.c_double(time), C.byref(st))
        stats = _stats_dict(st)
        self._check(rc, "mpl_step")
        return stats

    def step_explicit(self, parts_in: dict, parts_out: dict, dt, gravity=(0.0, 0.0, 0.0), bcs=(),
                      time=0.0):
        pi, po = _particles(parts_in), _particles(parts_out)
        st = _Stats()
        rc = self._lib.mpl_step_explicit(self._ctx, C.byref(pi), C.byref(po), C.c_double(dt),
                                         (C.c_double * 3)(*gravity), _bcs(list(bcs)), len(bcs),
                                         C.c_double(time), C.byref(st))
        stats = _stats_dict(st)
        self._check(rc, "mpl_step_explicit")
        return stats

    # ------------------------------------------------------------ sub-steps
    def unload(self, parts: dict, dt, gravity=(0.0, 0.0, 0.0), bcs=(), time=0.0):
        pi = _particles(parts)
        self._parts_ref = parts
        self._check(self._lib.mpl_unload(self._ctx, C.byref(pi), C.c_double(dt),
                                         (C.c_double * 3)(*gravity), _bcs(list(bcs)), len(bcs),
                                         C.c_double(time)), "mpl_unload")

    def reconstruct(self):
        self._check(self._lib.mpl_reconstruct_stretch(self._ctx), "mpl_reconstruct_stretch")

    def _check_node_vec(self, t: torch.Tensor, name: str):
        n1 = [d + 1 for d in self.dims]
        want = (n1[0] * n1[1] * n1[2], 3)
        if tuple(t.shape) != want:
            raise ValueError(f"{name} has shape {tuple(t.shape)}, want {want} (dense node vector)")
        return t

    @staticmethod
    def _check_box(t: torch.Tensor, name: str, channels, like=None):
        shape = tuple(t.shape)
        if like is not None:
            want = tuple(like.shape[:3]) + ((channels,) if channels else ())
        else:
            want = shape[:3] + ((channels,) if channels else ())
        if shape != want or len(shape[:3]) != 3:
            raise ValueError(f"{name} has shape {shape}, want {want} ([X, Y, Z(, C)] box)")
        return t

    def _node_vec(self, dtype=torch.float64):
        n1 = [d + 1 for d in self.dims]
        return torch.zeros((n1[0] * n1[1] * n1[2], 3), dtype=dtype, device="cuda")

    def energy_grad(self, v=None, want_grad=True):
        E = C.c_double()
        g = self._node_vec() if want_grad else None
        vp = C.c_void_p(_dptr(self._check_node_vec(v, "v"), torch.float64)) if v is not None else None
        self._check(self._lib.mpl_energy_grad(self._ctx, vp, C.byref(E),
                                              C.c_void_p(g.data_ptr()) if g is not None else None),
                    "mpl_energy_grad")
        return E.value, g

    def build_tangent(self, v=None, precision=F32):
        vp = C.c_void_p(_dptr(self._check_node_vec(v, "v"), torch.float64)) if v is not None else None
        self._check(self._lib.mpl_build_tangent(self._ctx, vp, int(precision)), "mpl_build_tangent")

    def hv(self, u: torch.Tensor, precision=F32):
        dt = torch.float32 if precision == F32 else torch.float64
        out = self._node_vec(dt)
        self._check(self._lib.mpl_hv(self._ctx, C.c_void_p(_dptr(self._check_node_vec(u, "u"), dt)), C.c_void_p(out.data_ptr()),
                                     int(precision)), "mpl_hv")
        return out

    def hv_noalloc(self, u: torch.Tensor, out: torch.Tensor, precision=F32):
        """Allocation-free Hu (mpl_hv_noalloc) into the caller's dense tensor ``out``;
        enqueued on the context's stream, not synchronised."""
        dt = torch.float32 if precision == F32 else torch.float64
        self._check_node_vec(out, "out")
        self._check(self._lib.mpl_hv_noalloc(self._ctx, C.c_void_p(_dptr(self._check_node_vec(u, "u"), dt)),
                                             C.c_void_p(_dptr(out, dt)), int(precision)),
                    "mpl_hv_noalloc")
        return out

    def pcg(self, b: torch.Tensor):
        x = self._node_vec()
        it = C.c_int32()
        rel = C.c_double()
        self._check(self._lib.mpl_pcg(self._ctx, C.c_void_p(_dptr(self._check_node_vec(b, "b"), torch.float64)),
                                      C.c_void_p(x.data_ptr()), C.byref(it), C.byref(rel)), "mpl_pcg")
        return x, it.value, rel.value

    def solve(self):
        v = self._node_vec()
        st = _Stats()
        rc = self._lib.mpl_solve(self._ctx, C.c_void_p(v.data_ptr()), C.byref(st))
        stats = _stats_dict(st)
        self._check(rc, "mpl_solve")
        return v, stats

    def integrate_explicit(self, want_force=False):
        v = self._node_vec()
        f = self._node_vec() if want_force else None
        self._check(self._lib.mpl_integrate_explicit(self._ctx, C.c_void_p(v.data_ptr()),
                                                     C.c_void_p(f.data_ptr()) if f is not None else None),
                    "mpl_integrate_explicit")
        return (v, f) if want_force else v

    def load(self, parts_in: dict, parts_out: dict, dt, v=None):
        vp = C.c_void_p(_dptr(self._check_node_vec(v, "v"), torch.float64)) if v is not None else None
        self._check(self._lib.mpl_load(self._ctx, vp, C.byref(_particles(parts_in)),
                                       C.byref(_particles(parts_out)), C.c_double(dt)), "mpl_load")

    def export(self, name: str) -> torch.Tensor:
        fid, kind, comps = FIELDS[name]
        nx, ny, nz = self.dims
        if kind == "node":
            shape = ((nx + 1) * (ny + 1) * (nz + 1), comps)
        elif kind == "cell":
            shape = (nx * ny * nz, comps)
        else:
            shape = (self.nmat, nx * ny * nz, comps)
        out = torch.zeros(shape, dtype=torch.float64, device="cuda")
        self._check(self._lib.mpl_export_field(self._ctx, int(fid), C.c_void_p(out.data_ptr())),
                    "mpl_export_field")
        return out

    # ------------------------------------------------------------ multigrid
    def mg_apply(self, r: torch.Tensor):
        """One V-cycle z = B r (dense FP64 node vectors) with the current
        tangent; returns (z, level count, per-level damping)."""
        z = torch.zeros_like(self._check_node_vec(r, "r"))
        nl = C.c_int32()
        om = (C.c_double * MG_MAX_LEVELS)()
        self._check(self._lib.mpl_mg_apply(self._ctx, C.c_void_p(_dptr(r, torch.float64)),
                                           C.c_void_p(z.data_ptr()), C.byref(nl), om), "mpl_mg_apply")
        return z, nl.value, [om[i] for i in range(nl.value)]

    def mg_export(self, level: int, field: str) -> torch.Tensor:
        """Dense FP64 export of multigrid level ``level`` >= 1: ``mass``,
        ``fixed``, ``abar`` (cells x 81) or ``diag`` (nodes x 3)."""
        code, kind, comps = dict(mass=(0, "node", 1), fixed=(1, "node", 1), abar=(2, "cell", 81),
                                 diag=(3, "node", 3))[field]
        d = [n >> level for n in self.dims]
        rows = (d[0] + 1) * (d[1] + 1) * (d[2] + 1) if kind == "node" else d[0] * d[1] * d[2]
        out = torch.zeros((rows, comps), dtype=torch.float64, device="cuda")
        self._check(self._lib.mpl_mg_export(self._ctx, C.c_int32(level), C.c_int32(code),
                                            C.c_void_p(out.data_ptr())), "mpl_mg_export")
        return out if comps > 1 else out[:, 0]

    # ------------------------------------------------------------ learned preconditioner
    def precond_param_count(self) -> int:
        n = C.c_int64()
        self._check(self._lib.mpl_precond_param_count(self._ctx, C.byref(n)), "mpl_precond_param_count")
        return n.value

    def precond_set_weights(self, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        self._check(self._lib.mpl_precond_set_weights(self._ctx, p.ctypes.data_as(C.c_void_p),
                                                      C.c_int64(p.size)), "mpl_precond_set_weights")

    def precond_get_weights(self):
        import numpy as np
        p = np.zeros(self.precond_param_count(), dtype=np.float32)
        self._check(self._lib.mpl_precond_get_weights(self._ctx, p.ctypes.data_as(C.c_void_p),
                                                      C.c_int64(p.size)), "mpl_precond_get_weights")
        return p

    def nn_forward(self, x: torch.Tensor):
        """Network forward on a dense box x [X, Y, Z, 16] (FP32 device)."""
        self._check_box(x, "x", 16)
        dims = (C.c_int32 * 3)(*x.shape[:3])
        y = torch.zeros_like(x)
        self._check(self._lib.mpl_nn_forward(self._ctx, C.c_void_p(_dptr(x, torch.float32)), dims,
                                             C.c_void_p(y.data_ptr())), "mpl_nn_forward")
        return y

    def nn_backward(self, x: torch.Tensor, dy: torch.Tensor):
        """Parameter gradient of <dy, network(x)> (FP32 device, flat)."""
        self._check_box(x, "x", 16)
        self._check_box(dy, "dy", 16, like=x)
        dims = (C.c_int32 * 3)(*x.shape[:3])
        g = torch.zeros(self.precond_param_count(), dtype=torch.float32, device="cuda")
        self._check(self._lib.mpl_nn_backward(self._ctx, C.c_void_p(_dptr(x, torch.float32)), dims,
                                              C.c_void_p(_dptr(dy, torch.float32)),
                                              C.c_void_p(g.data_ptr())), "mpl_nn_backward")
        return g

    def nn_layer_grad(self, layer: int, x: torch.Tensor, dy: torch.Tensor, box):
        """One network layer on caller tensors (mpl_nn_layer_grad): x [in voxels, Ci],
        dy [out voxels, Co] (FP32 device); returns (y, dx, dparams)."""
        dims = (C.c_int32 * 3)(*box)
        y = torch.zeros_like(dy)
        dx = torch.zeros_like(x)
        n = self._layer_param_counts()[layer]
        dp = torch.zeros(n, dtype=torch.float32, device="cuda")
        self._check(self._lib.mpl_nn_layer_grad(self._ctx, C.c_int32(layer), C.c_void_p(_dptr(x, torch.float32)),
                                                dims, C.c_void_p(_dptr(dy, torch.float32)),
                                                C.c_void_p(y.data_ptr()), C.c_void_p(dx.data_ptr()),
                                                C.c_void_p(dp.data_ptr())), "mpl_nn_layer_grad")
        return y, dx, dp

    @staticmethod
    def _layer_param_counts():
        # (k, Ci, Co) of the 21 layers in execution order (include/mpmlite.h)
        spec = [(3, 16, 16), (3, 16, 16), (2, 16, 32), (3, 32, 32), (3, 32, 32), (2, 32, 64),
                (3, 64, 64), (3, 64, 64), (2, 64, 128), (3, 128, 128), (3, 128, 128), (2, 128, 64),
                (3, 128, 64), (3, 64, 64), (2, 64, 32), (3, 64, 32), (3, 32, 32), (2, 32, 16),
                (3, 32, 16), (3, 16, 16), (1, 16, 16)]
        return [k ** 3 * ci * co + co for k, ci, co in spec]

    def precond_train_step(self, x, t, mask, lr, grads_out: torch.Tensor = None):
        """One Adam step on the pair loss; returns the loss before the step.
        grads_out (FP32 CUDA, precond_param_count values) receives the
        parameter gradient the step applies."""
        self._check_box(x, "x", 16)
        self._check_box(t, "t", 3, like=x)
        self._check_box(mask, "mask", None, like=x)
        if grads_out is not None and (grads_out.dtype != torch.float32 or not grads_out.is_cuda
                                      or not grads_out.is_contiguous()
                                      or grads_out.numel() != self.precond_param_count()):
            raise ValueError("grads_out: contiguous FP32 CUDA tensor of precond_param_count() values")
        dims = (C.c_int32 * 3)(*x.shape[:3])
        loss = C.c_float()
        self._check(self._lib.mpl_precond_train_step(
            self._ctx, C.c_void_p(_dptr(x, torch.float32)), C.c_void_p(_dptr(t, torch.float32)),
            C.c_void_p(_dptr(mask, torch.float32)), dims, C.c_float(lr), C.byref(loss),
            C.c_void_p(grads_out.data_ptr() if grads_out is not None else None)),
            "mpl_precond_train_step")
        return loss.value

    def precond_apply(self, r: torch.Tensor) -> torch.Tensor:
        """z = learned preconditioner applied to the dense node vector r."""
        z = self._node_vec()
        self._check(self._lib.mpl_precond_apply(self._ctx, C.c_void_p(_dptr(self._check_node_vec(r, "r"), torch.float64)),
                                                C.c_void_p(z.data_ptr())), "mpl_precond_apply")
        return z

    def precond_reserve(self, capacity: int):
        self._check(self._lib.mpl_precond_reserve(self._ctx, C.c_int32(capacity)), "mpl_precond_reserve")

    def precond_collect(self, every: int, rtol: float = 1e-10):
        self._check(self._lib.mpl_precond_collect(self._ctx, C.c_int32(every), C.c_double(rtol)),
                    "mpl_precond_collect")

    def precond_sample_count(self) -> int:
        n = C.c_int32()
        self._check(self._lib.mpl_precond_sample_count(self._ctx, C.byref(n)), "mpl_precond_sample_count")
        return n.value

    def precond_train(self, n_steps: int, lr: float, seed: int = 0):
        import numpy as np
        losses = np.zeros(max(n_steps, 1), dtype=np.float32)
        self._check(self._lib.mpl_precond_train(self._ctx, C.c_int32(n_steps), C.c_float(lr),
                                                C.c_uint32(seed), losses.ctypes.data_as(C.c_void_p)),
                    "mpl_precond_train")
        return losses[:n_steps]

    def box_dims(self):
        """Dims of the network box over the grid's nodes (each axis padded to a multiple of 8)."""
        return tuple(((d + 1 + 7) // 8) * 8 for d in self.dims)

    def precond_energy_loss(self, r: torch.Tensor, o_box: torch.Tensor = None):
        """(L(z), Jacobi loss, dL/do) of the energy-norm loss on residual r, with the
        network output o_box [X, Y, Z, 16] given or (None) computed from r."""
        loss, ref = C.c_double(), C.c_double()
        g = self._node_vec()
        op = None
        if o_box is not None:
            if tuple(o_box.shape) != self.box_dims() + (16,):
                raise ValueError(f"o_box has shape {tuple(o_box.shape)}, want {self.box_dims() + (16,)}")
            op = C.c_void_p(_dptr(o_box, torch.float32))
        self._check(self._lib.mpl_precond_energy_loss(
            self._ctx, C.c_void_p(_dptr(self._check_node_vec(r, "r"), torch.float64)), op,
            C.byref(loss), C.byref(ref), C.c_void_p(g.data_ptr())), "mpl_precond_energy_loss")
        return loss.value, ref.value, g

    def precond_adam_step(self, grad: torch.Tensor, lr: float):
        if tuple(grad.shape) != (self.precond_param_count(),):
            raise ValueError("grad must hold one value per network parameter")
        self._check(self._lib.mpl_precond_adam_step(self._ctx, C.c_void_p(_dptr(grad, torch.float32)),
                                                    C.c_float(lr)), "mpl_precond_adam_step")

    def precond_record_pair(self, r: torch.Tensor, x: torch.Tensor, xstar: torch.Tensor):
        ptrs = [C.c_void_p(_dptr(self._check_node_vec(t, n), torch.float64))
                for t, n in ((r, "r"), (x, "x"), (xstar, "xstar"))]
        self._check(self._lib.mpl_precond_record_pair(self._ctx, *ptrs), "mpl_precond_record_pair")

    def precond_get_sample(self, i: int):
        """(features [X, Y, Z, 16], target [X, Y, Z, 3], mask [X, Y, Z]) of stored pair i."""
        X = self.box_dims()
        f = torch.zeros(X + (16,), dtype=torch.float32, device="cuda")
        t = torch.zeros(X + (3,), dtype=torch.float32, device="cuda")
        m = torch.zeros(X, dtype=torch.float32, device="cuda")
        self._check(self._lib.mpl_precond_get_sample(self._ctx, C.c_int32(i), C.c_void_p(f.data_ptr()),
                                                     C.c_void_p(t.data_ptr()), C.c_void_p(m.data_ptr())),
                    "mpl_precond_get_sample")
        return f, t, m

    def precond_online(self, every: int, steps: int = 1, lr: float = 1e-3):
        self._check(self._lib.mpl_precond_online(self._ctx, C.c_int32(every), C.c_int32(steps),
                                                 C.c_float(lr)), "mpl_precond_online")

    def precond_online_stats(self):
        """(training steps so far, mean network loss, mean Jacobi loss) since the last call."""
        n = C.c_int64()
        loss = C.c_double()
        ref = C.c_double()
        self._check(self._lib.mpl_precond_online_stats(self._ctx, C.byref(n), C.byref(loss), C.byref(ref)),
                    "mpl_precond_online_stats")
        return n.value, loss.value, ref.value
