#!/usr/bin/env python3
"""Train the warm start's perceptron on the GPU and measure it on held-out
instances.

Data: the 80-instance family of `instances.learned_family` (grid and dense,
n = 20..30); idx < 64 train, idx >= 64 held out.  For each training
instance the library runs `--iters` plain F1 iterations with multiplier
tracking on (the transfers of the ascent rules are Lagrange multiplier
updates, Section 3.1 / Eq. ch4:proof:2), samples `--per-instance` orbits,
and gathers their features and their members' tracked z multipliers divided
by max|F| max|D| / (n - 2).  The perceptron (bf16 MFMA kernels, float32
Adam) fits the zero-sum projection of its outputs to those targets.

After fitting, a gain on the predicted multipliers is chosen on the last
`--calib` training instances (fewest iterations to the bound of
`--cold-iters` cold iterations) and saved with the weights.

Held-out measurement (time-to-bound): cold = `--cold-iters` F1 iterations
from Algorithm 1's start, wall time W and bound LB_cold; warm = the learned
S-form start (features + inference + z writer, all timed) followed by F1
iterations until the bound reaches LB_cold.  Reported per instance: warm
time to LB_cold, warm bound at time W, and the held-out fit (R^2).

Writes the weights (npz: W1 b1 W2 b2 W3 b3, float32) and a JSON report.
Every step runs in the HIP library; this script only moves tensors.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_1710_03732_amd import binding as B  # noqa: E402
from paper_1710_03732_amd import instances as I  # noqa: E402

WEIGHTS = os.path.join(HERE, "weights", "warm_mlp.npz")


def log(*a):
    print(f"[{time.strftime('%H:%M:%S')}]", *a, flush=True)


def init_params(seed: int) -> dict:
    """He-normal hidden layers, small output layer, zero biases."""
    rng = np.random.default_rng(seed)
    return {"W1": rng.standard_normal((256, 32)) * np.sqrt(2.0 / 28),
            "b1": np.zeros(256),
            "W2": rng.standard_normal((256, 256)) * np.sqrt(2.0 / 256),
            "b2": np.zeros(256),
            "W3": rng.standard_normal((6, 256)) * np.sqrt(1.0 / 256) * 0.1,
            "b3": np.zeros(6)}


def load_weights(path: str = WEIGHTS) -> dict:
    """W1..b3 and the calibrated multiplier gain (1.0 if the file has none)."""
    with np.load(path) as z:
        out = {k: z[k] for k in ("W1", "b1", "W2", "b2", "W3", "b3")}
        out["gain"] = float(z["gain"]) if "gain" in z.files else 1.0
    return out


def save_weights(mlp: "B.Mlp", path: str):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, gain=np.float64(mlp.gain), **B.unpack_mlp_params(mlp.params()))


GAINS = (1.0, 1.5, 2.0, 2.5, 3.0, 3.5)


def calibrate_gain(mlp, idx_list, cold_iters: int):
    """Multiplier gain of the warm start, chosen on training instances: the
    one whose warm run reaches the bound of `cold_iters` cold iterations in
    the fewest iterations (geometric mean over the instances; a run that
    never reaches it counts 2 * cold_iters).  Regression toward the mean
    shrinks the predicted multipliers, and the ascent profits from a
    stronger start than their least-squares scale."""
    scores = {g: [] for g in GAINS}
    for idx in idx_list:
        inst = I.learned_family(idx)
        F, D, Bm = inst.arrays()
        c = B.DualAscent(F, D, Bm)
        lbc = c.run(cold_iters)["lb"]
        c.close()
        h = B.DualAscent(F, D, Bm)
        y = h.orbit_outputs(mlp)
        scale = h.multiplier_scale()
        row = []
        for g in GAINS:
            h.warm_start_outputs(y, scale * g)
            h.run(cold_iters)
            tr = np.maximum.accumulate(h.trace())
            hit = np.nonzero(tr >= lbc)[0]
            k = int(hit[0]) + 1 if len(hit) else 2 * cold_iters
            scores[g].append(k)
            row.append(k)
        h.close()
        log(f"gain calibration {inst.name}: iterations to the cold bound {dict(zip(GAINS, row))}")
    gm = {g: float(np.exp(np.mean(np.log(v)))) for g, v in scores.items()}
    best = min(GAINS, key=lambda g: gm[g])
    log(f"gain {best} (geometric-mean iterations {gm})")
    return best, gm


def collect(idx_list, iters, per_instance, seed):
    """Features and targets of sampled orbits of each instance (device)."""
    import torch

    xs, ts, info = [], [], []
    for idx in idx_list:
        inst = I.learned_family(idx)
        F, D, Bm = inst.arrays()
        t0 = time.perf_counter()
        h = B.DualAscent(F, D, Bm)
        h.track()
        r = h.run(iters)
        scale = h.multiplier_scale()
        cnt = B.orbit_count(inst.n)
        g = torch.Generator().manual_seed(seed + idx)
        ids = torch.randint(0, cnt, (per_instance,), generator=g, dtype=torch.int64).to("cuda")
        xs.append(h.orbit_features(ids))
        ts.append(h.orbit_targets(ids, scale))
        h.close()
        info.append({"idx": idx, "name": inst.name, "n": inst.n, "lb": r["lb"], "ub": r["ub"],
                     "seconds": time.perf_counter() - t0})
        log(f"targets {inst.name}: {iters} tracked iterations, LB {r['lb']:.1f}, UB {r['ub']:.1f}, "
            f"{time.perf_counter() - t0:.2f} s")
    return torch.cat(xs), torch.cat(ts), info


def fit(X, T, epochs, batch, lr, seed, params=None):
    import torch

    mlp = B.Mlp(params or init_params(seed), max_batch=batch)
    N = X.shape[0]
    steps = max(1, N // batch)
    total = epochs * steps
    g = torch.Generator(device="cuda").manual_seed(seed)
    k = 0
    for ep in range(epochs):
        perm = torch.randperm(N, device="cuda", generator=g)
        acc, cnt = 0.0, 0
        for s in range(steps):
            idx = perm[s * batch:(s + 1) * batch]
            cur = lr * 0.5 * (1.0 + np.cos(np.pi * k / total))  # cosine decay
            loss = mlp.train_step(X[idx].contiguous(), T[idx].contiguous(), lr=max(cur, lr * 0.02))
            acc += loss
            cnt += 1
            k += 1
        log(f"epoch {ep + 1}/{epochs}: mean loss {acc / cnt:.5f}")
    return mlp


def r2(mlp, X, T, batch):
    import torch

    se, ss = 0.0, 0.0
    for s in range(0, X.shape[0], batch):
        y = mlp.forward(X[s:s + batch].contiguous())
        y = y - y.mean(dim=1, keepdim=True)
        t = T[s:s + batch]
        se += float(((y - t) ** 2).sum())
        ss += float((t ** 2).sum())
    return 1.0 - se / ss


def time_to_bound(inst, mlp, cold_iters: int):
    """Cold: cold_iters F1 iterations from Algorithm 1's start (wall time W,
    bound LB_cold).  Warm: the learned start plus the k F1 iterations it
    needs to reach LB_cold, k found by a first warm run and then timed as one
    call on a fresh handle (warm start included).  All runs are
    deterministic, so the timed run reaches the same bound."""
    import torch

    F, D, Bm = inst.arrays()
    cold = B.DualAscent(F, D, Bm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = cold.run(cold_iters)
    W = time.perf_counter() - t0
    cold_tr = cold.trace()
    lb_cold = r["lb"]
    cold.close()
    probe = B.DualAscent(F, D, Bm)
    st = probe.warm_start(mlp)
    tp = time.perf_counter()
    probe.run(cold_iters)
    per_iter = (time.perf_counter() - tp) / cold_iters
    warm_tr = probe.trace()
    probe.close()
    best = np.maximum.accumulate(warm_tr)
    hit = np.nonzero(best >= lb_cold)[0]
    reached = None
    if len(hit):
        k = int(hit[0]) + 1
        timed = B.DualAscent(F, D, Bm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        timed.warm_start(mlp)
        rr = timed.run(k)
        el = time.perf_counter() - t0
        timed.close()
        reached = {"seconds": el, "iterations": k, "lb": rr["lb"]}
    # bound the warm start holds at wall time W (iterations at the measured rate)
    k_W = int(max(0, min(len(best), (W - st["seconds"]) / per_iter)))
    return {"name": inst.name, "n": inst.n, "cold_iterations": len(cold_tr), "cold_seconds": W,
            "cold_lb": lb_cold, "cold_lb_t0": float(cold_tr[0]), "cold_ub": r["ub"],
            "warm_start_seconds": st["seconds"], "warm_start_ms_mlp": st["ms_mlp"],
            "warm_start_ms_write": st["ms_write"], "warm_lb_t0": float(warm_tr[0]),
            "warm_lb_after_cold_iterations": float(best[-1]),
            "warm_lb_at_W": float(best[k_W - 1]) if k_W > 0 else None,
            "warm_to_cold_lb": reached,
            "speedup": (W / reached["seconds"]) if reached else None}


def u_ablation(inst, mlp, tracked_iters: int, cold_iters: int):
    """How much could predicting the y-pair multipliers u add?  From the
    multipliers (v, u) that `tracked_iters` plain iterations with tracking
    reach (the training targets), restart once with (v, u) and once with
    (v, 0), and compare both with the learned start (predicted v, u = 0):
    bound at the restart, iterations and seconds to the bound of
    `cold_iters` cold iterations.  The tracked (v, u) is the best a
    predictor of both could hope to reproduce; the gap between its two
    restarts bounds what a u prediction can gain."""
    import torch

    F, D, Bm = inst.arrays()
    cold = B.DualAscent(F, D, Bm)
    lb_cold = cold.run(cold_iters)["lb"]
    cold.close()
    t = B.DualAscent(F, D, Bm)
    t.track()
    t.run(tracked_iters)
    v, u = t.multipliers()
    t.close()
    out = {"name": inst.name, "n": inst.n, "cold_iterations": cold_iters, "cold_lb": lb_cold,
           "tracked_iterations": tracked_iters,
           "u_rel_size": float(np.abs(u).sum() / max(1e-300, np.abs(v).sum()))}
    for label, uu in (("tracked_v_u", u), ("tracked_v_only", None), ("learned_v", None)):
        h = B.DualAscent(F, D, Bm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if label == "learned_v":
            h.warm_start(mlp)
        else:
            h.set_multipliers(v, uu)
        h.run(cold_iters)
        el = time.perf_counter() - t0
        tr = np.maximum.accumulate(h.trace())
        h.close()
        hit = np.nonzero(tr >= lb_cold)[0]
        k = int(hit[0]) + 1 if len(hit) else None
        out[label] = {"lb_t0": float(tr[0]), "lb_after": float(tr[-1]), "iterations_to_cold_lb": k,
                      "seconds_per_iteration": el / cold_iters,
                      "seconds_to_cold_lb_est": (el * k / cold_iters) if k else None}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--iters", type=int, default=500, help="tracked iterations per training instance")
    ap.add_argument("--per-instance", type=int, default=1 << 18)
    ap.add_argument("--train", type=int, default=64, help="training instances (idx < this)")
    ap.add_argument("--heldout", type=int, default=16, help="held-out instances (idx 64..)")
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cold-iters", type=int, default=100)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--report", default=None)
    ap.add_argument("--eval-only", action="store_true",
                    help="load --out instead of training; re-measure the held-out instances")
    ap.add_argument("--recalibrate", action="store_true",
                    help="with --eval-only: choose the gain again on the training instances and save it")
    ap.add_argument("--calib", type=int, default=16, help="training instances (the last ones) for the gain")
    ap.add_argument("--u-ablation", default=None,
                    help="instead of training: write the u ablation of the held-out instances to this JSON file")
    args = ap.parse_args(argv)

    import torch

    if not torch.cuda.is_available():
        print("train_warm.py: no GPU visible", file=sys.stderr)
        return 1
    t_all = time.perf_counter()
    if args.u_ablation:
        mlp = B.Mlp(load_weights(args.out), max_batch=args.batch)
        rows = []
        for idx in range(64, 64 + args.heldout):
            res = u_ablation(I.learned_family(idx), mlp, args.iters, args.cold_iters)
            rows.append(res)
            log(f"{res['name']}: |u|/|v| {res['u_rel_size']:.3f}; LB0 (v,u) {res['tracked_v_u']['lb_t0']:.1f} "
                f"(v,0) {res['tracked_v_only']['lb_t0']:.1f} learned {res['learned_v']['lb_t0']:.1f}; "
                f"iterations to the cold bound (v,u) {res['tracked_v_u']['iterations_to_cold_lb']} "
                f"(v,0) {res['tracked_v_only']['iterations_to_cold_lb']} "
                f"learned {res['learned_v']['iterations_to_cold_lb']}")
        with open(args.u_ablation, "w") as f:
            json.dump({"rows": rows, "args": vars(args), "seconds": time.perf_counter() - t_all}, f, indent=1)
        mlp.close()
        return 0
    calib = list(range(max(0, args.train - args.calib), args.train))
    gain_scores = None
    if args.eval_only:
        mlp = B.Mlp(load_weights(args.out), max_batch=args.batch)
        info, train_r2 = None, None
        log(f"weights <- {args.out} (gain {mlp.gain})")
        if args.recalibrate:
            mlp.gain, gain_scores = calibrate_gain(mlp, calib, args.cold_iters)
            save_weights(mlp, args.out)
            log(f"gain {mlp.gain} -> {args.out}")
    else:
        X, T, info = collect(range(args.train), args.iters, args.per_instance, args.seed)
        log(f"training set: {X.shape[0]} orbits from {len(info)} instances")
        mlp = fit(X, T, args.epochs, args.batch, args.lr, args.seed)
        train_r2 = r2(mlp, X, T, args.batch)
        del X, T
        mlp.gain, gain_scores = calibrate_gain(mlp, calib, args.cold_iters)
        save_weights(mlp, args.out)
        log(f"weights -> {args.out}; train R^2 {train_r2:.4f}; gain {mlp.gain}")
    held = list(range(64, 64 + args.heldout))
    Xh, Th, _ = collect(held, args.iters, 1 << 16, args.seed + 7)
    held_r2 = r2(mlp, Xh, Th, args.batch)
    del Xh, Th
    log(f"held-out R^2 {held_r2:.4f}")
    ttb = []
    for idx in held:
        res = time_to_bound(I.learned_family(idx), mlp, args.cold_iters)
        ttb.append(res)
        w = res["warm_to_cold_lb"]
        log(f"{res['name']}: cold {args.cold_iters} its {res['cold_seconds']:.3f} s LB {res['cold_lb']:.1f}; "
            f"warm LB0 {res['warm_lb_t0']:.1f} (cold LB0 {res['cold_lb_t0']:.1f}); "
            + (f"warm reaches it in {w['seconds']:.3f} s / {w['iterations']} its" if w else "warm does not reach it")
            + f"; warm LB after {args.cold_iters} its {res['warm_lb_after_cold_iterations']:.1f}")
    report = {"train": info, "train_r2": train_r2, "heldout_r2": held_r2, "gain": mlp.gain,
              "gain_calibration": gain_scores, "time_to_bound": ttb,
              "args": vars(args), "seconds": time.perf_counter() - t_all}
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)
    reached = [r["speedup"] for r in ttb if r["speedup"]]
    log(f"held-out: warm reached the cold bound on {len(reached)}/{len(ttb)} instances; "
        f"median speedup {np.median(reached) if reached else float('nan'):.2f}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
