"""Training driver of the learned preconditioner (the network and its
training run in the library: pair collection during Newton solves, BF16
MFMA forward/backward, Adam on FP32 master weights; this module only
sequences the calls and stores the weights).

    python -m paper_2602_07853_amd.precond_train --config 3 --out weights.npy
    python -m paper_2602_07853_amd.precond_train --configs 2,3 --eval-steps 5 --out weights.npy

collects (residual, error) pairs from the Jacobi-PCG solves of the first
``--collect-steps`` implicit steps of the scene (or of several scenes, the
corpus of the learned-preconditioner configuration: pairs from the 64^3 and
128^3 workloads) and trains on them; ``--eval-steps`` then times Jacobi PCG
and the learned preconditioner over the same trajectory steps.
"""
from __future__ import annotations

import argparse
import sys
import time

import numpy as np

# (name, kernel taps, in channels, out channels) in execution order; the
# flat parameter vector holds W[tap][in][out] then bias[out] per layer.
CH = (16, 32, 64, 128)
LAYERS = [("enc0a", 27, 16, 16), ("enc0b", 27, 16, 16), ("down0", 8, 16, 32),
          ("enc1a", 27, 32, 32), ("enc1b", 27, 32, 32), ("down1", 8, 32, 64),
          ("enc2a", 27, 64, 64), ("enc2b", 27, 64, 64), ("down2", 8, 64, 128),
          ("bota", 27, 128, 128), ("botb", 27, 128, 128), ("up2", 8, 128, 64),
          ("dec2a", 27, 128, 64), ("dec2b", 27, 64, 64), ("up1", 8, 64, 32),
          ("dec1a", 27, 64, 32), ("dec1b", 27, 32, 32), ("up0", 8, 32, 16),
          ("dec0a", 27, 32, 16), ("dec0b", 27, 16, 16), ("out", 1, 16, 16)]
UP = {"up2", "up1", "up0"}


# (input level, output level) of every layer; level L has box >> L voxels per axis
LEVEL = {"enc0a": (0, 0), "enc0b": (0, 0), "down0": (0, 1), "enc1a": (1, 1), "enc1b": (1, 1),
         "down1": (1, 2), "enc2a": (2, 2), "enc2b": (2, 2), "down2": (2, 3), "bota": (3, 3),
         "botb": (3, 3), "up2": (3, 2), "dec2a": (2, 2), "dec2b": (2, 2), "up1": (2, 1),
         "dec1a": (1, 1), "dec1b": (1, 1), "up0": (1, 0), "dec0a": (0, 0), "dec0b": (0, 0),
         "out": (0, 0)}


def forward_flops(box) -> float:
    """Multiply-add FLOPs (2 per MAC) of one forward pass on a dense box."""
    total = 0.0
    for name, t, ci, co in LAYERS:
        lin, lout = LEVEL[name]
        nout = (box[0] >> lout) * (box[1] >> lout) * (box[2] >> lout)
        # gather convolutions: taps x ci MACs per output channel and voxel;
        # transposed convolutions: ci MACs per output value (one tap each)
        total += 2.0 * co * (ci * nout if name in UP else t * ci * nout)
    return total


def param_count() -> int:
    return sum(t * ci * co + co for _, t, ci, co in LAYERS)


def init_weights(seed: int = 0, out_scale: float = 0.0) -> np.ndarray:
    """He-normal weights, zero biases; the output layer scaled by out_scale
    (0 = the network starts as the zero map, i.e. as Jacobi)."""
    rng = np.random.default_rng(seed)
    w = []
    for name, t, ci, co in LAYERS:
        fan_in = ci if name in UP else t * ci
        W = rng.normal(0.0, np.sqrt(2.0 / fan_in), t * ci * co)
        if name == "out":
            W *= out_scale
        w += [W, np.zeros(co)]
    return np.concatenate(w).astype(np.float32)


def save_weights(path: str, w: np.ndarray):
    np.save(path, np.asarray(w, dtype=np.float32), allow_pickle=False)


def load_weights(path: str) -> np.ndarray:
    w = np.load(path, allow_pickle=False)
    if w.dtype != np.float32 or w.ndim != 1 or w.size != param_count():
        raise ValueError(f"{path}: expected {param_count()} float32 parameters")
    return w


def collect(ctx, sc, parts, steps: int, every: int, capacity: int, t0: float = 0.0, log=print):
    """Run `steps` implicit steps of the scene from `parts` (advanced in
    place) with pair collection on; returns the number of stored pairs."""
    ctx.precond_reserve(capacity)
    ctx.precond_collect(every, 1e-10)
    try:
        for k in range(steps):
            st = ctx.step(parts, parts, sc.dt, sc.gravity, sc.bcs, t0 + k * sc.dt)
            log(f"[train] collect step {k}: newton {st['newton_iters']} pcg {st['pcg_iters']} "
                f"pairs {ctx.precond_sample_count()}")
    finally:
        ctx.precond_collect(0, 1e-10)
    return ctx.precond_sample_count()


def train(ctx, n_steps: int, lr: float, seed: int = 0, chunk: int = 50, log=print):
    """n_steps Adam steps on the stored pairs (learning rate halved for the
    last third); returns the per-step losses."""
    losses = []
    done = 0
    t = time.perf_counter()
    while done < n_steps:
        k = min(chunk, n_steps - done)
        rate = lr if done < 2 * n_steps // 3 else 0.5 * lr
        losses.append(ctx.precond_train(k, rate, seed=seed + done))
        done += k
        log(f"[train] {done}/{n_steps} steps, loss {losses[-1][-k:].mean():.4f} "
            f"({time.perf_counter() - t:.1f}s)")
    return np.concatenate(losses) if losses else np.zeros(0)


def evaluate(sc, weights, warmup: int, steps: int, log=print, warm_start: int = 4) -> dict:
    """Jacobi PCG against the learned preconditioner over the same trajectory
    steps of scene `sc`: `warmup` untimed Jacobi steps from the initial
    state, then `steps` timed steps with each preconditioner from that same
    state (the Jacobi CG with the given warm start, the flexible CG of the
    learned preconditioner from zero).  Returns CG iterations and ms per step."""
    import torch
    from paper_2602_07853_amd import mpmlite
    out = {}
    parts = mpmlite.particles_to_device(sc.particles)
    ctx = mpmlite.Context((sc.n,) * 3, sc.dx, sc.materials,
                          opts=dict(hv_precision=mpmlite.F32, newton_rtol=1e-6, pcg_rtol=1e-6,
                                    warm_start=warm_start))
    ctx.precond_set_weights(weights)
    for k in range(warmup):
        ctx.step(parts, parts, sc.dt, sc.gravity, sc.bcs, k * sc.dt)
    start = {k: v.clone() for k, v in parts.items()}
    for name, pre in (("jacobi", mpmlite.PRECOND_JACOBI), ("learned", mpmlite.PRECOND_LEARNED)):
        ctx.set_opts(precond=pre)
        p = {k: v.clone() for k, v in start.items()}
        pcg = newton = fb = 0
        torch.cuda.synchronize()
        t = time.perf_counter()
        for k in range(steps):
            st = ctx.step(p, p, sc.dt, sc.gravity, sc.bcs, (warmup + k) * sc.dt)
            pcg += st["pcg_iters"]
            newton += st["newton_iters"]
            fb += st["fallbacks"]
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / steps
        out[name] = dict(pcg_per_step=pcg / steps, newton_per_step=newton / steps,
                         fallbacks_per_step=fb / steps, ms_per_step=round(ms, 2))
        log(f"[train] eval {name}: {out[name]}")
    out["trajectory_steps"] = [warmup, warmup + steps - 1]
    out["learned_vs_jacobi_time"] = round(out["jacobi"]["ms_per_step"] / out["learned"]["ms_per_step"], 4)
    return out


def corpus(configs, collect_steps: int, every: int, capacity: int, train_steps: int, lr: float,
           seed: int, rounds: int, log=print):
    """Pairs from the Newton solves of several workloads (one context per
    grid, each holding its own pairs), trained in rounds: each round takes
    train_steps / rounds Adam steps on every workload's pairs in turn, the
    weights handed from context to context (each keeps its own Adam
    moments).  Returns (weights, pair counts, final losses)."""
    from paper_2602_07853_amd import mpmlite, scenes
    w = init_weights(seed)
    ctxs, counts = [], {}
    for cfg in configs:
        sc = scenes.CONFIGS[cfg]()
        ctx = mpmlite.Context((sc.n,) * 3, sc.dx, sc.materials,
                              opts=dict(hv_precision=mpmlite.F32, newton_rtol=1e-6, pcg_rtol=1e-6))
        ctx.precond_set_weights(w)
        parts = mpmlite.particles_to_device(sc.particles)
        counts[sc.name] = collect(ctx, sc, parts, collect_steps, every, capacity, log=log)
        del parts
        ctxs.append((sc.name, ctx))
    per = max(1, train_steps // (rounds * len(ctxs)))
    losses = {}
    for r in range(rounds):
        for name, ctx in ctxs:
            ctx.precond_set_weights(w)
            l = ctx.precond_train(per, lr if r < (2 * rounds) // 3 else 0.5 * lr, seed=seed + r)
            w = ctx.precond_get_weights()
            losses[name] = float(np.mean(l[-min(len(l), 10):]))
        log(f"[train] round {r + 1}/{rounds}: losses {losses}")
    for _, ctx in ctxs:
        ctx.close()
    return w, counts, losses


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--configs", default=None,
                    help="comma-separated workloads whose Newton solves give the pairs (e.g. 2,3); "
                         "trained in rounds, then evaluated on the last one")
    ap.add_argument("--collect-steps", type=int, default=3)
    ap.add_argument("--every", type=int, default=20)
    ap.add_argument("--capacity", type=int, default=120)
    ap.add_argument("--train-steps", type=int, default=1500)
    ap.add_argument("--rounds", type=int, default=10)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--eval-warmup", type=int, default=3)
    ap.add_argument("--eval-steps", type=int, default=0,
                    help="after training, time this many steps of the last workload with Jacobi and "
                         "with the learned preconditioner from the same state")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    import json
    from paper_2602_07853_amd import mpmlite, scenes
    log = lambda s: print(s, file=sys.stderr, flush=True)
    if a.configs:
        cfgs = [int(c) for c in a.configs.split(",")]
        w, counts, losses = corpus(cfgs, a.collect_steps, a.every, a.capacity, a.train_steps, a.lr,
                                   a.seed, a.rounds, log=log)
        save_weights(a.out, w)
        res = dict(pairs=counts, final_losses=losses, train_steps=a.train_steps, rounds=a.rounds)
        if a.eval_steps > 0:
            res["eval"] = evaluate(scenes.CONFIGS[cfgs[-1]](), w, a.eval_warmup, a.eval_steps, log=log)
        print(json.dumps(res), flush=True)
        return
    sc = scenes.CONFIGS[a.config]()
    ctx = mpmlite.Context((sc.n,) * 3, sc.dx, sc.materials,
                          opts=dict(hv_precision=mpmlite.F32, newton_rtol=1e-6, pcg_rtol=1e-6))
    ctx.precond_set_weights(init_weights(a.seed))
    parts = mpmlite.particles_to_device(sc.particles)
    n = collect(ctx, sc, parts, a.collect_steps, a.every, a.capacity, log=log)
    log(f"[train] {n} pairs")
    train(ctx, a.train_steps, a.lr, a.seed, log=log)
    save_weights(a.out, ctx.precond_get_weights())
    if a.eval_steps > 0:
        print(json.dumps(evaluate(sc, ctx.precond_get_weights(), a.eval_warmup, a.eval_steps, log=log)),
              flush=True)


if __name__ == "__main__":
    main()
