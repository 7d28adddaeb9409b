"""Benchmark: implicit MPM Lite steps per second on one MI355X.

Workload (default): the stiff plastic solid on a 128^3 grid, ~1M active cells,
~8M particles, fixed-corotated E=7e7 nu=0.3 with von Mises yield 1e5, a
sticky floor and a plate pressing at 0.2 m/s, dt=1e-3; every step is a full
Unload -> stretch reconstruction -> Newton-PCG (Jacobi, FP32 Hessian-vector
products, FP64 reductions) to relative residual 1e-6 -> Load.

Prints ONE JSON line (see the fields below).  ``roofline`` describes the
kernel with the most time per step, the single-reduction CG update
(``k_cg_step``): algorithmic bytes per launch (60 B per free DOF) divided by
its average duration, timed with HIP events on the library's stream over the
timed steps; ``hv_kernel`` gives the same for the fused Hessian-vector
product (180 B per tangent-carrying cell + 28 B per active node).  Both also
carry the library's own count of the bytes its kernels must move (the
factored tangent reads 25 values per cell).  ``traffic`` is the HBM bytes per
launch measured by rocprofv3 counters (profiles/cg_traffic.json), when those
were taken with the current library.  ``cpu_baseline`` times the FP64 CPU
oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=3, choices=[1, 2, 3, 5])
    ap.add_argument("--precision", choices=["f32", "f64"], default="f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision-check", action="store_true",
                    help="skip the final-error check of one step against the FP64 GPU variant")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "cg_traffic.json"))
    ap.add_argument("--ppc-axis", type=int, default=None,
                    help="particles per cell along each axis (default: the config's, 2 = 8 PPC)")
    ap.add_argument("--check-every", type=int, default=16,
                    help="CG iterations per graph chunk between convergence polls")
    ap.add_argument("--time-kernels", type=int, default=2, choices=[0, 1, 2],
                    help="HIP events around Hv launches: 1 every launch, 2 the middle product of "
                         "every CG chunk, 0 none (no roofline figure)")
    ap.add_argument("--warm-start", type=int, default=4, choices=[0, 1, 2, 3, 4],
                    help="start each Newton iteration's CG from the previous step's direction "
                         "(2, 3: extrapolated linearly / quadratically from the last steps; 4: the "
                         "energy-norm best combination of the last three)")
    ap.add_argument("--explicit-steps", type=int, default=200,
                    help="timed steps of the explicit leg (jelly-falling workload, 256^3); 0 = skip")
    ap.add_argument("--plasticity", choices=["after_solve", "fixed_point"], default="after_solve",
                    help="plastic projection on the particles after the solve, or in addition the "
                         "fixed point inside Newton")
    ap.add_argument("--plastic-anderson", type=int, default=0,
                    help="Anderson depth of the fixed-point plasticity iteration (0 = plain)")
    ap.add_argument("--vbd-steps", type=int, default=10,
                    help="timed steps of the VBD-vs-Newton-PCG leg (two-material bar, 64^3); 0 = skip")
    ap.add_argument("--vbd-sweeps", type=int, default=4)
    ap.add_argument("--bj-steps", type=int, default=5,
                    help="timed steps of the block-Jacobi leg, after 3 untimed ones (0 = skip the leg)")
    ap.add_argument("--mg-steps", type=int, default=5,
                    help="timed steps of the multigrid-preconditioned CG leg (0: skip)")
    ap.add_argument("--mg-levels", type=int, default=0, help="V-cycle levels (0: the library's 4)")
    ap.add_argument("--mg-smooth", type=int, default=0, help="sweeps per side (0: the library's 2)")
    ap.add_argument("--newton-forcing", type=float, default=0.0,
                    help="inexact Newton forcing term for the main run (0: every CG to 1e-6)")
    ap.add_argument("--inexact-forcing", type=float, default=0.1,
                    help="forcing term of the inexact-Newton leg (0 = skip the leg)")
    ap.add_argument("--learned-steps", type=int, default=2,
                    help="timed steps of the learned-preconditioner leg (0 = skip the leg)")
    ap.add_argument("--learned-train-steps", type=int, default=2,
                    help="untimed Jacobi steps with online network training before that leg")
    return ap.parse_args()


def make_scene(cfg, ppc_axis=None):
    from paper_2602_07853_amd import scenes
    if ppc_axis is not None:
        if cfg not in (2, 3, 5):
            raise SystemExit("--ppc-axis applies to configs 2, 3 and 5")
        return scenes.CONFIGS[cfg](ppc_axis=ppc_axis)
    return scenes.CONFIGS[cfg]()


def workload_name(sc):
    return (f"{sc.name}: {sc.n}^3 grid, {sc.occupied_cells} occupied cells, "
            f"{sc.n_particles} particles, dt={sc.dt}, Newton + Jacobi PCG to rel. resid 1e-6")


_ORACLE_STEP = r"""
import json, sys, time
sys.path.insert(0, sys.argv[1])
from oracle import oracle as O
from paper_2602_07853_amd import scenes
sc = scenes.CONFIGS[int(sys.argv[2])]()
g, mats, bcs = O.grid_of(sc), O.materials_of(sc), O.bcs_of(sc)
t0 = time.perf_counter()
po, st, v, rc = O.step(g, mats, sc.dt, sc.gravity, bcs, 0.0, O.SolverOpts(1e-6, 1e-6), sc.particles)
print(json.dumps({"s": time.perf_counter() - t0, "rc": rc, "newton": st["newton_iters"],
                  "pcg": st["pcg_iters_total"], "particles": sc.n_particles}))
"""


def cpu_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def oracle_full_step(cfg, threads):
    """One whole oracle step (Alg. 1, Newton + Jacobi PCG to 1e-6, FP64) of
    config ``cfg`` from its initial state, in a child process with
    ``threads`` OpenMP threads; wall seconds and the oracle's own counts."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    out = subprocess.run([sys.executable, "-c", _ORACLE_STEP, ROOT, str(cfg)], env=env,
                         capture_output=True, text=True, timeout=900, check=True)
    return json.loads(out.stdout.strip().splitlines()[-1])


def cpu_baseline(sc, cold_counts):
    """The FP64 oracle on the host cores.

    Measured: (1) one whole oracle step of the 64^3 fixed-corotated workload
    (885k particles, Newton + Jacobi PCG to 1e-6) on one thread and on all
    threads; (2) a bounded sample of the 128^3 workload at its initial
    state: the oracle's unload, reconstruction and load, and its own
    Newton-PCG solver stopped after one Newton iteration with its CG capped
    at 10 and at 40 iterations, which gives the cost of one CG iteration
    (product and vector operations) and of the rest of a Newton iteration
    (energy, gradient, tangent, line search).  The 128^3 steps/s (``value``)
    extrapolates the sample to a whole step with the Newton and CG counts of
    this run's first step, which starts CG from zero like the oracle."""
    from oracle import oracle as O
    model, ncpu = cpu_info()
    threads = int(os.environ.get("OMP_NUM_THREADS", ncpu))
    full = {"threads_1": oracle_full_step(2, 1), f"threads_{threads}": oracle_full_step(2, threads)}
    g, mats, bcs = O.grid_of(sc), O.materials_of(sc), O.bcs_of(sc)
    t = {}

    def timed(name, fn):
        t0 = time.perf_counter()
        out = fn()
        t[name] = time.perf_counter() - t0
        return out

    u = timed("unload", lambda: O.unload(g, sc.particles, mats))
    fixed, vfix = O.node_bcs(g, u["mi"], bcs, 0.0)
    act = u["mi"] > 0
    vhat = np.where(O.fixed_components(fixed), vfix,
                    np.where(act[:, None], u["vi"] + sc.dt * np.asarray(sc.gravity), 0))
    S, _ = timed("reconstruct", lambda: O.reconstruct(g, mats, u["Vck"], u["tauck"]))
    for K in (10, 40):
        timed(f"solve_{K}", lambda: O.solve(g, mats, sc.dt, u["mc"], u["mi"], vhat, fixed, u["Vck"], S,
                                            O.SolverOpts(1e-6, 1e-6, max_newton=1, max_pcg=K)))
    timed("load", lambda: O.load(g, sc.dt, u["mc"], vhat, sc.particles, mats))
    per_cg = (t["solve_40"] - t["solve_10"]) / 30.0
    per_newton = max(t["solve_10"] - 10 * per_cg, 0.0)
    newton, pcg = cold_counts
    step_s = t["unload"] + t["reconstruct"] + t["load"] + newton * per_newton + pcg * per_cg
    cpu_s = sum(t.values()) + sum(v["s"] for v in full.values())
    sample = (f"{cpu_s:.1f}s of CPU work. Measured: whole oracle steps of the 64^3 workload "
              f"(1 thread {full['threads_1']['s']:.1f}s, {threads} threads "
              f"{full[f'threads_{threads}']['s']:.1f}s); at 128^3 the oracle's unload "
              f"{t['unload']:.2f}s, reconstruction {t['reconstruct']:.2f}s, load {t['load']:.2f}s, and "
              f"its own solver for one Newton iteration: {per_cg * 1e3:.1f} ms per CG iteration "
              f"(product + vector ops), {per_newton:.2f}s for the rest of the iteration. The 128^3 "
              f"figure extrapolates these to a whole step with the counts of this run's first step "
              f"(CG from zero, as in the oracle): {newton} Newton, {pcg} CG iterations")
    return {"value": 1.0 / step_s, "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": sample, "cpu_model": model, "nproc": ncpu,
            "method": "128^3 value extrapolated from a measured sample; 64^3 steps measured whole",
            "oracle_step_s_128": round(step_s, 2),
            "oracle_full_step_64": full}


def step_error(sc, parts, ctx, t):
    """Error of one step of `ctx` (its current options) from state `parts`
    against the FP64 GPU variant of the same step converged to 1e-10."""
    import torch
    from paper_2602_07853_amd import mpmlite
    src = {k: v.clone() for k, v in parts.items()}
    tight = mpmlite.Context((sc.n,) * 3, sc.dx, sc.materials,
                            opts=dict(hv_precision=mpmlite.F64, newton_rtol=1e-10, pcg_rtol=1e-10))
    ref = {k: v.clone() for k, v in src.items()}
    tight.step(src, ref, sc.dt, sc.gravity, sc.bcs, t)
    out = {k: v.clone() for k, v in src.items()}
    ctx.step(src, out, sc.dt, sc.gravity, sc.bcs, t)
    torch.cuda.synchronize()
    del tight

    def rel(a, b):
        return float((a - b).norm() / b.norm().clamp_min(1e-300))
    res = {"x": rel(out["x"], ref["x"]), "dx": rel(out["x"] - src["x"], ref["x"] - src["x"]),
           "v": rel(out["v"], ref["v"]), "F": rel(out["F"], ref["F"]), "G": rel(out["G"], ref["G"])}
    return {k: float(f"{v:.3e}") for k, v in res.items()}


def precision_check(sc, parts, ctx, t):
    """Final error of one production step (FP32 products, tolerances 1e-6)
    from the current state, against the FP64 GPU variant of the same step
    converged to 1e-10 (the variant the parity tests hold to the oracle
    within 1e-10); the FP64 variant at the production tolerances is given
    too, to separate the tolerance from the precision."""
    import torch
    from paper_2602_07853_amd import mpmlite
    src = {k: v.clone() for k, v in parts.items()}
    runs = {}
    tight = mpmlite.Context((sc.n,) * 3, sc.dx, sc.materials,
                            opts=dict(hv_precision=mpmlite.F64, newton_rtol=1e-10, pcg_rtol=1e-10))
    same = mpmlite.Context((sc.n,) * 3, sc.dx, sc.materials,
                           opts=dict(hv_precision=mpmlite.F64, newton_rtol=1e-6, pcg_rtol=1e-6))
    for name, c in (("f32", ctx), ("f64_tight", tight), ("f64", same)):
        out = {k: v.clone() for k, v in src.items()}
        c.step(src, out, sc.dt, sc.gravity, sc.bcs, t)
        runs[name] = out
    torch.cuda.synchronize()

    def rel(a, b):
        return float((a - b).norm() / b.norm().clamp_min(1e-300))

    ref = runs["f64_tight"]
    res = {}
    for name in ("f32", "f64"):
        r = runs[name]
        res[name] = {"x": rel(r["x"], ref["x"]), "dx": rel(r["x"] - src["x"], ref["x"] - src["x"]),
                     "v": rel(r["v"], ref["v"]), "F": rel(r["F"], ref["F"]), "G": rel(r["G"], ref["G"])}
        res[name] = {k: float(f"{v:.3e}") for k, v in res[name].items()}
    del tight, same
    return {"reference": "FP64 GPU variant, Newton and CG to 1e-10 (held to the oracle within 1e-10 by the parity tests)",
            "step": "one step from the state after the timed steps", "production_f32": res["f32"],
            "f64_same_tolerances": res["f64"]}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path is not sharded "
              f"across GPUs.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2602_07853_amd import mpmlite

    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU")
    torch.cuda.set_device(0)
    sc = make_scene(args.config, args.ppc_axis)
    prec = mpmlite.F32 if args.precision == "f32" else mpmlite.F64
    ctx = mpmlite.Context((sc.n,) * 3, sc.dx, sc.materials,
                          opts=dict(hv_precision=prec, newton_rtol=1e-6, pcg_rtol=1e-6,
                                    pcg_check_every=args.check_every, time_kernels=args.time_kernels,
                                    warm_start=args.warm_start, newton_forcing=args.newton_forcing,
                                    plasticity=(mpmlite.PLASTICITY_FIXED_POINT if args.plasticity == "fixed_point"
                                                else mpmlite.PLASTICITY_AFTER_SOLVE),
                                    plastic_anderson=args.plastic_anderson))
    parts = mpmlite.particles_to_device(sc.particles)
    print(f"[bench] {workload_name(sc)}", file=sys.stderr, flush=True)
    step_idx = 0

    def one_step():
        nonlocal step_idx
        st = ctx.step(parts, parts, sc.dt, sc.gravity, sc.bcs, step_idx * sc.dt)
        step_idx += 1
        return st

    parts0 = {k: v.clone() for k, v in parts.items()} if args.learned_steps > 0 else None
    traj = {}   # trajectory step -> (CG iterations, host-timed ms of the step's stages)
    first = None
    for w in range(args.warmup):
        st = one_step()
        traj[w] = (st["pcg_iters"], st["ms_unload"] + st["ms_newton"] + st["ms_load"])
        if first is None:
            first = (st["newton_iters"], st["pcg_iters"])
        print(f"[bench] warmup {w} {json.dumps(st)}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    hv_ms, hv_calls, newton, pcg, ls = 0.0, 0, 0, 0, 0
    up_ms, up_calls, up_bytes = 0.0, 0, 0.0
    cells = nodes = 0
    hv_bytes = 0.0
    tan_entries = 0
    t0 = time.perf_counter()
    for k in range(args.steps):
        st = one_step()
        traj[args.warmup + k] = (st["pcg_iters"], st["ms_unload"] + st["ms_newton"] + st["ms_load"])
        if first is None:
            first = (st["newton_iters"], st["pcg_iters"])
        hv_ms += st["hv_ms_total"]
        hv_calls += st["hv_calls"]
        up_ms += st["upd_ms_total"]
        up_calls += st["upd_calls"]
        up_bytes = st["upd_model_bytes"]
        newton += st["newton_iters"]
        pcg += st["pcg_iters"]
        ls += st["ls_halvings"]
        cells, nodes = st["active_cells"], st["active_nodes"]
        hv_bytes, tan_entries = st["hv_model_bytes"], st["tangent_entries"]
        print(f"[bench] step {k} newton {st['newton_iters']} pcg {st['pcg_iters']} "
              f"({'/'.join(str(x) for x in st['pcg_per_newton'][:st['newton_iters']])}) "
              f"ls {st['ls_halvings']} g {st['g_norm']:.3e}/{st['g0_norm']:.3e} "
              f"ms unload {st['ms_unload']:.1f} newton {st['ms_newton']:.1f} load {st['ms_load']:.1f}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    steps_per_s = args.steps / elapsed
    # Algorithmic bytes per launch, from the per-unit figures of the design
    # notes' roofline table (FP32 products):
    #   CG update (a9): 60 B per free DOF -- r and x in FP64, p, q and the
    #     Jacobi diagonal in FP32, each read or written once;
    #   Hessian-vector product (a8): 180 B per tangent-carrying cell (45 FP32
    #     values of the symmetric 9x9 tangent) + 28 B per active node (u read,
    #     Hu written, m read).
    # The library's own count of what its kernels must move (the factored
    # tangent reads 25 values per cell) is given beside them.
    free_dofs = st["free_dofs"]
    elem = 4 if prec == mpmlite.F32 else 8
    n_tan = st["tangent_cells"]
    hv_alg = (45 * elem * n_tan + 7 * elem * nodes)
    up_alg = 15 * elem * free_dofs
    hv_avg_ms = hv_ms / max(hv_calls, 1)
    up_avg_ms = up_ms / max(up_calls, 1)
    traffic = {}
    if os.path.exists(args.traffic_json):
        try:
            tj = json.load(open(args.traffic_json)).get(sc.name, {})
            if tj.get("kernel_version") == ctx_version():
                traffic = {"hv": tj.get("bytes_per_hv"), "update": tj.get("bytes_per_update")}
        except Exception:
            traffic = {}
    copy_gbs = copy_bandwidth()

    def gbs(nbytes, ms):
        return nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0

    up_gbs = gbs(up_alg, up_avg_ms)
    roof = {"bound": "hbm", "achieved": round(up_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(up_gbs / HBM_PEAK_GBS, 4), "traffic": traffic.get("update"),
            "kernel": "k_cg_step (single-reduction CG update with the product-piece gather; the "
                      "kernel with the most time per step)",
            "bytes_per_launch": up_alg, "bytes_model": "60 B per free DOF (FP32 products)",
            "free_dofs": free_dofs, "avg_ms": round(up_avg_ms, 5), "launches": up_calls,
            "design_bytes_per_launch": up_bytes,
            "design_frac": round(gbs(up_bytes, up_avg_ms) / HBM_PEAK_GBS, 4),
            "achievable_copy_gbs": copy_gbs}
    hv_gbs = gbs(hv_alg, hv_avg_ms)
    hv_line = {"kernel": "k_hv_fused (matrix-free Hessian-vector product)", "bound": "hbm",
               "achieved": round(hv_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(hv_gbs / HBM_PEAK_GBS, 4), "traffic": traffic.get("hv"),
               "bytes_per_launch": hv_alg,
               "bytes_model": "180 B per tangent-carrying cell + 28 B per active node (FP32)",
               "tangent_cells": n_tan, "active_nodes": nodes,
               "avg_ms": round(hv_avg_ms, 5), "launches": hv_calls,
               "design_bytes_per_launch": hv_bytes, "factored_cells": st["factored_cells"],
               "design_frac": round(gbs(hv_bytes, hv_avg_ms) / HBM_PEAK_GBS, 4)}
    counts = (newton / args.steps, pcg / args.steps, ls / args.steps)
    final_error = None
    if not args.no_precision_check:
        final_error = precision_check(sc, parts, ctx, step_idx * sc.dt)
        print(f"[bench] final error {json.dumps(final_error)}", file=sys.stderr, flush=True)
    inexact = None
    if args.inexact_forcing > 0.0 and args.newton_forcing == 0.0:
        inexact = inexact_leg(sc, args, steps_per_s, traj, prec)
    block_jacobi = None
    if args.bj_steps > 0:
        block_jacobi = precond_leg(ctx, sc, args, steps_per_s, counts, traj, mpmlite.PRECOND_BLOCK_JACOBI,
                                   "block-Jacobi", args.bj_steps)
    multigrid = None
    if args.mg_steps > 0:
        mg_opts = dict(mg_levels=args.mg_levels, mg_smooth=args.mg_smooth)
        multigrid = precond_leg(ctx, sc, args, steps_per_s, counts, traj, mpmlite.PRECOND_MULTIGRID,
                                "multigrid", args.mg_steps, extra_opts=mg_opts)
        multigrid["options"] = {"levels": args.mg_levels or 4, "smooth": args.mg_smooth or 2,
                                "coarse_sweeps": 4, "omega_lambda": 1.6}
    learned = None
    if args.learned_steps > 0:
        learned = learned_leg(ctx, sc, parts0, args, steps_per_s, counts, traj)
    explicit = None
    if args.explicit_steps > 0:
        explicit = explicit_leg(args.explicit_steps)
    vbd = None
    if args.vbd_steps > 0:
        vbd = vbd_leg(args.vbd_steps, args.vbd_sweeps)
    base = None
    if not args.no_cpu_baseline and args.config in (1, 2, 3):
        base = cpu_baseline(sc, first)
    line = {
        "metric": "implicit steps/s @1M cells to resid 1e-6, learned vs plain PCG; Hv HBM GB/s",
        "value": round(steps_per_s, 4),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec == mpmlite.F32 else "f64",
        "data": "synthetic",
        "config": {"workload": workload_name(sc), "preconditioner": "jacobi",
                   "newton_forcing": args.newton_forcing,
                   "active_cells": cells, "active_nodes": nodes,
                   "newton_per_step": round(counts[0], 3), "pcg_per_step": round(counts[1], 2),
                   "hv_precision": args.precision, "plasticity": args.plasticity,
                   "plastic_anderson": args.plastic_anderson},
        "roofline": roof,
        "hv_kernel": hv_line,
        "final_error": final_error,
        "cpu_baseline": base,
        "inexact_newton": inexact,
        "block_jacobi": block_jacobi,
        "multigrid": multigrid,
        "learned": learned,
        "explicit": explicit,
        "vbd": vbd,
    }
    print(json.dumps(line), flush=True)


def inexact_leg(sc, args, plain_steps_per_s, traj, prec):
    """The same workload from its initial state with inexact Newton
    (Eisenstat-Walker forcing terms, eta_0 = --inexact-forcing): the early
    Newton systems are solved loosely, Newton still stops at 1e-6.  The same
    trajectory steps as the main run are timed (warm starts as in the main
    run), then one more step is compared with the FP64 variant converged to
    1e-10 like the main run's final error."""
    import torch
    from paper_2602_07853_amd import mpmlite
    ctx = mpmlite.Context((sc.n,) * 3, sc.dx, sc.materials,
                          opts=dict(hv_precision=prec, newton_rtol=1e-6, pcg_rtol=1e-6,
                                    pcg_check_every=args.check_every, warm_start=args.warm_start,
                                    newton_forcing=args.inexact_forcing))
    parts = mpmlite.particles_to_device(sc.particles)
    newton = pcg = 0
    host_ms = 0.0
    t = 0.0
    el = 0.0
    for k in range(args.warmup + args.steps):
        if k == args.warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        st = ctx.step(parts, parts, sc.dt, sc.gravity, sc.bcs, t)
        t += sc.dt
        if k >= args.warmup:
            newton += st["newton_iters"]
            pcg += st["pcg_iters"]
            host_ms += st["ms_unload"] + st["ms_newton"] + st["ms_load"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    n = args.steps
    sps = n / el
    jp = sum(traj[i][0] for i in range(args.warmup, args.warmup + n)) / n
    err = None if args.no_precision_check else step_error(sc, parts, ctx, t)
    out = {"newton_forcing": args.inexact_forcing, "steps_per_s": round(sps, 4), "steps": n,
           "ms_per_step": round(1e3 * el / n, 3), "newton_per_step": round(newton / n, 3),
           "pcg_per_step": round(pcg / n, 2), "vs_exact_newton": round(sps / plain_steps_per_s, 4),
           "exact_pcg_per_step": round(jp, 2), "trajectory_steps": [args.warmup, args.warmup + n - 1],
           "final_error": err}
    print(f"[bench] inexact Newton leg {json.dumps(out)}", file=sys.stderr, flush=True)
    del ctx, parts
    return out


def precond_leg(ctx, sc, args, plain_steps_per_s, plain_counts, traj, precond, label, nsteps, untimed=3,
                extra_opts=None):
    """The same workload from its initial state with another preconditioner
    (3x3 nodal block-Jacobi in the same single-reduction CG, or the
    multigrid V-cycle in Hestenes-Stiefel PCG), with the same warm start:
    ``untimed`` steps (the warm start's history fills up), then ``nsteps``
    timed steps.  The CG count falls along the trajectory, so the comparison
    with Jacobi is also made over the same trajectory steps of the main run
    (host stage timers on both sides)."""
    import torch
    from paper_2602_07853_amd import mpmlite
    parts = mpmlite.particles_to_device(sc.particles)
    # the leg's CG starts build their history from its own steps, as the main run's did
    ctx.set_opts(warm_start=0)
    ctx.set_opts(time_kernels=0, precond=precond, warm_start=args.warm_start, **(extra_opts or {}))
    t = 0.0
    for k in range(untimed):
        ctx.step(parts, parts, sc.dt, sc.gravity, sc.bcs, t)
        t += sc.dt
    torch.cuda.synchronize()
    newton = pcg = 0
    host_ms = 0.0
    t0 = time.perf_counter()
    for k in range(nsteps):
        st = ctx.step(parts, parts, sc.dt, sc.gravity, sc.bcs, t)
        t += sc.dt
        newton += st["newton_iters"]
        pcg += st["pcg_iters"]
        host_ms += st["ms_unload"] + st["ms_newton"] + st["ms_load"]
        print(f"[bench] {label} step {k}: newton {st['newton_iters']} pcg {st['pcg_iters']} "
              f"ms {st['ms_unload'] + st['ms_newton'] + st['ms_load']:.1f}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.set_opts(precond=mpmlite.PRECOND_JACOBI)
    n = nsteps
    sps = n / el
    out = {"steps_per_s": round(sps, 4), "steps": n, "untimed_steps": untimed,
           "ms_per_step": round(1e3 * el / n, 3), "newton_per_step": round(newton / n, 3),
           "pcg_per_step": round(pcg / n, 2), "vs_jacobi": round(sps / plain_steps_per_s, 4),
           "jacobi_pcg_per_step": round(plain_counts[1], 2), "same_steps": None}
    window = range(untimed, untimed + n)
    if not all(i in traj for i in window):
        raise RuntimeError(f"{label} window {window.start}..{window.stop - 1} lies outside the "
                           f"main run's {len(traj)} recorded steps; raise --steps or lower its step count")
    jp = sum(traj[i][0] for i in window) / n
    jm = sum(traj[i][1] for i in window) / n
    bm = host_ms / n
    key = label.lower().replace("-", "_")
    out["same_steps"] = {"trajectory_steps": [window.start, window.stop - 1],
                         "jacobi_pcg_per_step": round(jp, 2), f"{key}_pcg_per_step": round(pcg / n, 2),
                         "jacobi_host_ms": round(jm, 2), f"{key}_host_ms": round(bm, 2),
                         "speed_vs_jacobi": round(jm / bm, 4)}
    return out


def learned_leg(ctx, sc, parts, args, plain_steps_per_s, plain_counts, traj):
    """The same workload from its initial state with the learned preconditioner
    (flexible CG, Jacobi fallback): the network starts as the zero map (i.e.
    Jacobi), is trained online on the energy-norm loss during
    ``learned_train_steps`` untimed Jacobi steps, then ``learned_steps`` steps
    are timed with the learned preconditioner and no training.  They are
    compared with the main Jacobi run over the same trajectory steps (host
    stage timers on both sides); both start each CG from the same kind of
    warm start (the main run's option)."""
    import torch
    from paper_2602_07853_amd import precond_train
    ctx.precond_set_weights(precond_train.init_weights(0))
    # the leg's CG starts build their history from its own steps, as the main run's did
    ctx.set_opts(warm_start=0)
    ctx.set_opts(time_kernels=0, precond=0, warm_start=args.warm_start)
    ctx.precond_online(64, 1, 1e-3)
    t = 0.0
    for k in range(args.learned_train_steps):
        st = ctx.step(parts, parts, sc.dt, sc.gravity, sc.bcs, t)
        t += sc.dt
        n, loss, ref = ctx.precond_online_stats()
        print(f"[bench] learned-leg training step {k}: pcg {st['pcg_iters']} train steps {n} "
              f"mean loss {loss:.4f} (Jacobi {ref:.4f})", file=sys.stderr, flush=True)
    ctx.precond_online(0, 0, 0.0)
    ctx.set_opts(precond=2)
    torch.cuda.synchronize()
    newton = pcg = fb = 0
    host_ms = 0.0
    t0 = time.perf_counter()
    for k in range(args.learned_steps):
        st = ctx.step(parts, parts, sc.dt, sc.gravity, sc.bcs, t)
        t += sc.dt
        newton += st["newton_iters"]
        pcg += st["pcg_iters"]
        fb += st["fallbacks"]
        host_ms += st["ms_unload"] + st["ms_newton"] + st["ms_load"]
        print(f"[bench] learned step {k}: newton {st['newton_iters']} pcg {st['pcg_iters']} "
              f"fallbacks {st['fallbacks']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # one more learned step from the state reached, against the FP64 reference
    err = None if args.no_precision_check else step_error(sc, parts, ctx, t)
    ctx.set_opts(precond=0)
    net = network_rate(ctx, sc)
    n = args.learned_steps
    sps = n / el
    window = range(args.learned_train_steps, args.learned_train_steps + n)
    if not all(i in traj for i in window):
        raise RuntimeError(f"learned window {window.start}..{window.stop - 1} lies outside the main "
                           f"run's {len(traj)} recorded steps; raise --steps or --warmup")
    jp = sum(traj[i][0] for i in window) / n
    jm = sum(traj[i][1] for i in window) / n
    return {"steps_per_s": round(sps, 4), "steps": n, "ms_per_step": round(1e3 * el / n, 3),
            "newton_per_step": round(newton / n, 3), "pcg_per_step": round(pcg / n, 2),
            "fallbacks_per_step": round(fb / n, 3),
            "vs_plain": round(sps / plain_steps_per_s, 4),
            "same_steps": {"trajectory_steps": [window.start, window.stop - 1],
                           "jacobi_pcg_per_step": round(jp, 2), "learned_pcg_per_step": round(pcg / n, 2),
                           "jacobi_host_ms": round(jm, 2), "learned_host_ms": round(host_ms / n, 2),
                           "speed_vs_jacobi": round(jm / (host_ms / n), 4),
                           "note": f"both CG solvers start from warm_start={args.warm_start}"},
            "network": net,
            "final_error": err,
            "plain_pcg_per_step": round(plain_counts[1], 2),
            "training": f"online, energy-norm loss, {args.learned_train_steps} untimed Jacobi steps "
                        "from the workload's initial state, 1 Adam step per 64 CG iterations"}


def explicit_leg(nsteps, warmup=3):
    """The explicit branch of Integrate on the jelly-falling workload (256^3,
    about 1.1M particles, dt = 6e-5): unload, nodal force and update, load per
    step, timed on the wall clock between two synchronisations.  The stage
    split comes from the library's host timers."""
    import torch
    from paper_2602_07853_amd import mpmlite, scenes
    sc = scenes.jelly_falling()
    ctx = mpmlite.Context((sc.n,) * 3, sc.dx, sc.materials, opts=dict(hv_precision=mpmlite.F64))
    parts = mpmlite.particles_to_device(sc.particles)
    t = 0.0
    for _ in range(warmup):
        ctx.step_explicit(parts, parts, sc.dt, sc.gravity, sc.bcs, t)
        t += sc.dt
    torch.cuda.synchronize()
    ms = {"unload": 0.0, "integrate": 0.0, "load": 0.0}
    t0 = time.perf_counter()
    for _ in range(nsteps):
        st = ctx.step_explicit(parts, parts, sc.dt, sc.gravity, sc.bcs, t)
        t += sc.dt
        ms["unload"] += st["ms_unload"]
        ms["integrate"] += st["ms_newton"]
        ms["load"] += st["ms_load"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    line = {"workload": f"{sc.name}: {sc.n}^3 grid, dx=1/{sc.n}, {sc.n_particles} particles "
                        f"(8 ppc, {sc.occupied_cells} occupied cells), StVK-Hencky E=5e3 nu=0.4, "
                        f"dt={sc.dt:g}, gravity, two cubes falling onto a slab",
            "steps_per_s": round(nsteps / el, 2), "steps": nsteps,
            "ms_per_step": round(1e3 * el / nsteps, 4),
            "particles_per_s": round(sc.n_particles * nsteps / el, 1),
            "active_cells": st["active_cells"], "active_nodes": st["active_nodes"],
            "ms_stage": {k: round(v / nsteps, 4) for k, v in ms.items()}}
    print(f"[bench] explicit leg {json.dumps(line)}", file=sys.stderr, flush=True)
    del ctx, parts
    return line


def vbd_leg(nsteps, sweeps, warmup=1):
    """Vertex block descent against Newton-PCG on the same potential (the
    paper's VBD comparison, a soft-stiff-soft bar): each solver advances the
    bar from its initial state; steps/s, and the gradient reduction each
    reaches per step (Newton-PCG to 1e-6, VBD after a fixed sweep count)."""
    import torch
    from paper_2602_07853_amd import mpmlite, scenes
    sc = scenes.two_material_bar()
    out = {"workload": f"{sc.name}: {sc.n}^3 grid, {sc.n_particles} particles, split NH E=1e4/1e5/1e4, "
                       f"dt={sc.dt:g}, one end held, the other dragged at 0.5 m/s"}
    for name, opts in (("newton_pcg", dict(newton_rtol=1e-6, pcg_rtol=1e-6, warm_start=4)),
                       ("vbd", dict(vbd_sweeps=sweeps))):
        ctx = mpmlite.Context((sc.n,) * 3, sc.dx, sc.materials,
                              opts=dict(hv_precision=mpmlite.F64 if name == "vbd" else mpmlite.F32, **opts))
        parts = mpmlite.particles_to_device(sc.particles)
        t = 0.0
        for _ in range(warmup):
            ctx.step(parts, parts, sc.dt, sc.gravity, sc.bcs, t)
            t += sc.dt
        torch.cuda.synchronize()
        red = []
        t0 = time.perf_counter()
        for _ in range(nsteps):
            st = ctx.step(parts, parts, sc.dt, sc.gravity, sc.bcs, t)
            t += sc.dt
            red.append(st["g_norm"] / max(st["g0_norm"], 1e-300))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[name] = {"steps_per_s": round(nsteps / el, 2), "ms_per_step": round(1e3 * el / nsteps, 3),
                     "iters_per_step": round(st["newton_iters"], 2), "pcg_per_step": st["pcg_iters"],
                     "max_grad_reduction": float(f"{max(red):.3e}")}
        if name == "vbd":
            out[name]["sweeps"] = sweeps
        del ctx, parts
    out["vbd_vs_newton_pcg"] = round(out["vbd"]["steps_per_s"] / out["newton_pcg"]["steps_per_s"], 3)
    print(f"[bench] vbd leg {json.dumps(out)}", file=sys.stderr, flush=True)
    return out


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Read + write GB/s of a plain 1 GiB device-to-device copy (context for the
    roofline: what a streaming kernel reaches on this GPU)."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return round(2 * nbytes / (ms * 1e-3) / 1e9, 1)


def network_rate(ctx, sc, reps=5):
    """Time the network forward on the solver's box (all grid nodes, padded
    to multiples of 8) with events on the library's stream: dense MAC FLOPs
    per application / average time, against the BF16 dense MFMA peak."""
    import torch
    from paper_2602_07853_amd import precond_train
    b = ((sc.n + 1 + 7) // 8) * 8
    x = torch.randn((b, b, b, 16), dtype=torch.float32, device="cuda")
    x[..., 5:] = 0
    ctx.nn_forward(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ctx.nn_forward(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    flops = precond_train.forward_flops((b, b, b))
    return {"box": [b, b, b], "ms_per_forward": round(ms, 3), "gflop_per_forward": round(flops / 1e9, 1),
            "tflops": round(flops / (ms * 1e-3) / 1e12, 1), "peak_tflops": 2500.0,
            "frac": round(flops / (ms * 1e-3) / 2.5e15, 4),
            "note": "dense box, through the C-ABI forward entry point (includes its fp32->bf16 input and "
                    "bf16->fp32 output conversions, ~0.17 ms; the solver path stages bf16 directly)"}


def ctx_version():
    from paper_2602_07853_amd import mpmlite
    return mpmlite.library().mpl_version().decode()


if __name__ == "__main__":
    main()
