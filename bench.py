#!/usr/bin/env python3
"""Benchmark: F1 RLT2 dual-ascent iterations/s and LAPs/s on one MI355X.

Workload (default): the n = 30 root dual ascent of a dense symmetric QAP,
F and D ~ U{0..99} with zero diagonals, seed 0 (synthetic stand-in for the
Taillard-a family); FULL scheme, all n^2 (n-1)^2 = 756,900 Z-LAPs of size 28,
900 Y-LAPs of size 29 and one X-LAP of size 30 per iteration, FP64.

A step is one dual-ascent iteration (ascent sweep over the 593.4 M-entry z
array, Z-, Y- and X-LAPs).  W warmup iterations (including iteration 0, whose
z level is zero) run first; the K timed iterations are bracketed by
torch.cuda.synchronize() and the library's kernels run on torch's current
stream, each phase between HIP events recorded on that stream.

Prints one JSON line.  `roofline` is for the kernel with the largest device
time; its `achieved` is algorithmic bytes per launch / average launch time.
`frac` is against the 8 TB/s peak and `frac_of_copy` against a plain 2 GiB
device copy measured in the same run (after the timed region).
`variants` runs the HALF scheme (Section 5: only the Z-LAPs of tiles with
i < j), the two-phase F2 and the slow S1 and S2 (Section 3.4) on the same workload
and times each to the F1 bound of 100 iterations; `variants.annealing` compares 300
iterations of F1 and F2 with and without Type 4 annealing steps.
`time_to_bound` compares 100 cold iterations with the learned warm start
(trained weights from train_warm.py) reaching the same bound; its
`mlp_roofline` gives the inference kernel's TFLOP/s against the bf16 MFMA
peak.  `bnb` times branch-and-bound at n = 14 and 18 (dense) and on a 4x4 grid
(n = 16) with and without symmetry elimination.  `graph_replay` times the
same iterations on the library's production path (one captured HIP graph
per iteration, no events between kernels).  `n42` runs the n = 42 root
bound: 100 plain iterations (per-phase times, HBM rates, the bound every 10
iterations) against the learned warm start.  `iteration_hbm` relates the
iteration time to the minimal schedule's bytes (three passes over z) and to
the implemented schedule's (four).  `cpu_baseline` times the CPU oracle
(all OpenMP threads, then one iteration on one thread) on a bounded sample
(about 10 s of iterations) of the same workload, names the host CPU, and
checks the oracle's bound against the GPU trace at the same iteration (the
run exits with status 3 when they differ by more than 1e-9 relative).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense bf16 MFMA


def algorithmic_bytes(n: int) -> dict:
    """Minimal HBM bytes per launch of each phase (FP64, compact layout)."""
    m = n - 2
    T = n * n * (n - 1) * (n - 1)
    V = T * m * m
    nn = n * n
    return {
        # reads the z array, writes its slacks pi_z back in place; Theta RMW
        "zlap": 8 * (2 * V + 2 * T),
        # reads pi_z and writes the new z array, reads pi_y, pi_x; the x/y
        # scaling reads pi_y and writes R_y
        "sweep": 8 * (2 * V + T + nn) + 8 * (2 * T + 2 * nn),
        # reads R_y and its partner entries, writes pi_y, updates R_x
        "ylap": 8 * (3 * T + 2 * nn),
        "xlap": 8 * (5 * nn),
    }


def minimal_iteration_bytes(n: int) -> int:
    """HBM bytes of one iteration under the minimal schedule: the Z-LAPs read
    the z array and write only their duals (u, v per tile and Theta), the
    sweep reads the z array and the duals, forms the slacks on the fly and
    writes the new z array: 8 (3 V + 2 T (2 m + 1)) plus the O(n^4) y and x
    arrays.  The implemented schedule moves more (the Z-LAPs write the slacks
    back in place and the sweep reads them: four passes over z, not three);
    both are reported."""
    m = n - 2
    T = n * n * (n - 1) * (n - 1)
    V = T * m * m
    return 8 * (3 * V + 2 * T * (2 * m + 1))


def cpu_model() -> str:
    """The host CPU's model name (first entry of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def algorithmic_bytes_half(n: int) -> dict:
    """The same under the HALF scheme: only the upper half of the z array
    (tiles with i < j) is read and written; pi_y of every tile still feeds
    the sweep."""
    m = n - 2
    T = n * n * (n - 1) * (n - 1)
    V = T * m * m
    nn = n * n
    full = algorithmic_bytes(n)
    return {"zlap": 8 * (V + T), "sweep": 8 * (V + T + nn) + 8 * (2 * T + 2 * nn),
            "ylap": full["ylap"], "xlap": full["xlap"]}


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for name in ("lap_scalar.hpp", "lap_wave.hpp", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_1710_03732_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str):
    """HBM traffic per launch of the dominant kernel from the committed
    rocprofv3 PMC summary (FETCH_SIZE / WRITE_SIZE scaled by the copy-kernel
    factor), or None when it was taken on another workload or the kernels
    changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha") != kernel_source_sha() or t.get("workload") != workload:
        return None
    k = t.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k.get("bytes_per_launch")


def cpu_baseline(inst, threads: int | None, gpu_trace, budget_s: float = 10.0):
    """The CPU oracle on the same workload: full F1 iterations (t >= 1: ascent
    sweep and all Z/Y/X LAPs) after iteration 0, on all threads until
    `budget_s` seconds have been timed (at least two iterations); then one
    iteration on a single thread and the next one on all threads again
    (neighbouring iterations take about the same number of Dijkstra steps).
    The oracle's results do not depend on the thread count, so its bound
    after those iterations is compared with the GPU's trace at the same
    iteration (bitwise, and within the 1e-9 relative tolerance)."""
    import numpy as np

    from oracle import oracle as O

    if threads:
        O.set_threads(threads)
    used = O.max_threads()
    F, D, B = inst.arrays()
    cpu = O.DualAscent(F, D, B)
    cpu.run(1)  # iteration 0 (z level zero), untimed
    done, el = 0, 0.0
    while done < 2 or el < budget_s:
        t0 = time.perf_counter()
        cpu.run(1)
        el += time.perf_counter() - t0
        done += 1
    O.set_threads(1)
    t0 = time.perf_counter()
    cpu.run(1)
    one = time.perf_counter() - t0
    O.set_threads(used)
    t0 = time.perf_counter()
    cpu.run(1)
    nxt = time.perf_counter() - t0
    O.set_threads(threads or used)
    total = done + 3  # iterations 0 .. done + 2
    lb = cpu.LB
    gpu_lb = float(gpu_trace[total - 1]) if len(gpu_trace) >= total else None
    parity = {"iterations": total, "oracle_lb": lb, "gpu_lb": gpu_lb,
              "bitwise": gpu_lb is not None and gpu_lb == lb,
              "within_1e-9": gpu_lb is not None and abs(gpu_lb - lb) <= 1e-9 * abs(lb),
              "oracle_trace_equal": gpu_lb is not None
              and bool(np.array_equal(np.asarray(gpu_trace[:total]), np.asarray(cpu.trace())))}
    return {"value": done / el, "unit": "iterations/s", "cores": used, "kind": "oracle",
            "sample": f"{done} full F1 iterations (t = 1..{done}: ascent sweep and all Z/Y/X LAPs) of the "
                      f"{inst.name} workload after iteration 0, {el:.2f} s on {used} threads; then iteration "
                      f"{done + 1} on one thread ({one:.2f} s) and iteration {done + 2} on {used} threads "
                      f"({nxt:.2f} s)",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "seconds": el, "iterations": done,
            "single_thread": {"iteration": done + 1, "seconds": one, "iterations_per_s": 1.0 / one,
                              "laps_per_s": (inst.n * inst.n * (inst.n - 1) ** 2 + inst.n ** 2 + 1) / one},
            "all_threads_next_iteration": {"iteration": done + 2, "seconds": nxt, "threads": used},
            "lb_after": lb, "gpu_parity": parity}


def mem_available_gb() -> float:
    """MemAvailable of /proc/meminfo in GB (0 if unreadable)."""
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemAvailable:"):
                    return int(line.split()[1]) * 1024 / 1e9
    except OSError:
        pass
    return 0.0


def oracle_sizes_leg():
    """The CPU oracle at the other sizes of the measurement plan, beside the
    GPU on the same iterations: the n = 15 grid (3x5, 200 iterations after
    iteration 0 on all threads, then 10 on one thread) and the n = 42 dense
    instance (2 iterations after iteration 0 on all threads; its dense z
    array takes 43.9 GB, so it runs only with at least 48 GB of host memory
    available).  The GPU runs the same iterations on graph replay; the bounds
    are compared bitwise."""
    import numpy as np

    from oracle import oracle as O
    from paper_1710_03732_amd import binding, instances as insts

    used = O.max_threads()
    out = {"cores": used, "cpu_model": cpu_model(), "nproc": os.cpu_count()}

    def one(inst, iters_all: int, iters_single: int):
        F, D, B = inst.arrays()
        nn = inst.n
        laps = nn * nn * (nn - 1) ** 2 + nn * nn + 1
        cpu = O.DualAscent(F, D, B)
        cpu.run(1)  # iteration 0, untimed
        t0 = time.perf_counter()
        cpu.run(iters_all)
        el = time.perf_counter() - t0
        res = {"n": nn, "instance": inst.name, "iterations": iters_all, "seconds": el,
               "iterations_per_s": iters_all / el, "laps_per_s": iters_all * laps / el, "threads": used}
        if iters_single:
            O.set_threads(1)
            t0 = time.perf_counter()
            cpu.run(iters_single)
            one_s = time.perf_counter() - t0
            O.set_threads(used)
            res["single_thread"] = {"iterations": iters_single, "seconds": one_s,
                                    "iterations_per_s": iters_single / one_s}
        total = 1 + iters_all + iters_single
        gpu = binding.DualAscent(F, D, B)
        gpu.run(1)
        t0 = time.perf_counter()
        gpu.run(total - 1)
        gel = time.perf_counter() - t0
        gt = gpu.trace()
        res["gpu"] = {"iterations": total - 1, "seconds": gel, "iterations_per_s": (total - 1) / gel}
        res["bound_after"] = cpu.LB
        res["gpu_trace_equal"] = bool(np.array_equal(np.asarray(gt[:total]), np.asarray(cpu.trace())))
        gpu.close()
        del cpu
        return res

    out["n15"] = one(insts.grid_n15(), 200, 10)
    avail = mem_available_gb()
    if avail >= 48.0:
        out["n42"] = one(insts.dense_instance(42, 0), 2, 0)
    else:
        out["n42"] = {"skipped": f"{avail:.1f} GB of host memory available, 48 GB needed"}
    return out


def warm_vs_cold(inst, cold_iters: int):
    """Time-to-bound: wall time of `cold_iters` cold F1 iterations (W, bound
    LB_cold) against the learned warm start (features, inference and z
    writer included) plus the F1 iterations it needs to reach LB_cold."""
    from paper_1710_03732_amd import binding, train_warm

    if not os.path.exists(train_warm.WEIGHTS):
        return {"skipped": "no trained weights (paper_1710_03732_amd/train_warm.py)"}
    mlp = binding.Mlp(train_warm.load_weights(), max_batch=256)
    res = train_warm.time_to_bound(inst, mlp, cold_iters)
    ms = res["warm_start_ms_mlp"]
    flops = 2.0 * binding.orbit_count(inst.n) * (32 * 256 + 256 * 256 + 256 * 6)
    res["mlp_roofline"] = {"bound": "mfma", "kernel": "k_orbit_mlp", "achieved": flops / (ms * 1e-3) / 1e12,
                           "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": flops / (ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS, "flops": flops,
                           "ms": ms}
    mlp.close()
    return res


def graph_replay_leg(inst, steps: int, warmup: int, timed_trace):
    """The library's production path: a handle on its own stream, whose
    iteration is one captured HIP graph replayed per iteration with no events
    between the kernels.  Same workload, warmup and step count as the timed
    run (which records events around every kernel); the bounds must agree
    bitwise."""
    import numpy as np
    import torch

    from paper_1710_03732_amd import binding

    F, D, B = inst.arrays()
    h = binding.DualAscent(F, D, B)
    if warmup > 0:
        h.run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = h.run(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    tr = h.trace()
    h.close()
    done = r["iterations_done"]
    n = inst.n
    laps = n * n * (n - 1) * (n - 1) + n * n + 1
    return {"iterations_per_s": done / el if done else None, "ms_per_step": 1e3 * el / done if done else None,
            "laps_per_s": laps * done / el if done else None, "iterations_done": done,
            "trace_equal_to_timed_run": bool(np.array_equal(tr, timed_trace))}


def n42_leg(cold_iters: int = 100, every: int = 10):
    """The n = 42 root bound (dense symmetric F, D ~ U{0..99}, seed 0; the
    z array is 37.96 GB): `cold_iters` plain iterations with events around
    every kernel (per-phase times, HBM rates against the minimal schedule's
    bytes and the implemented schedule's), then the learned warm start
    followed by the same number of iterations, and the wall time the warm
    start (features, inference and z writer included) needs to reach the
    plain bound.  Bounds every `every` iterations."""
    import numpy as np
    import torch

    from paper_1710_03732_amd import binding, instances as insts, train_warm

    inst = insts.dense_n42()
    F, D, B = inst.arrays()
    n = inst.n
    m = n - 2
    T = n * n * (n - 1) * (n - 1)
    ab = algorithmic_bytes(n)
    stream = torch.cuda.current_stream()
    h = binding.DualAscent(F, D, B, timing=1)
    h.set_stream(stream.cuda_stream)
    h.run(1)  # iteration 0 and the Z-LAP mapping's tuning, untimed
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = h.run(cold_iters - 1)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    cold_tr = h.trace()
    mapping = mapping_text(h)
    h.close()
    done = r["iterations_done"]
    phase_ms = {"sweep": r["ms_sweep"] / done, "zlap": r["ms_zlap"] / done,
                "ylap": r["ms_ylap"] / done, "xlap": r["ms_xlap"] / done}
    per_it = el / done
    out = {"workload": "dense_n42: QAP n=42 root dual ascent, dense symmetric F,D~U{0..99}, zero diagonals, "
                       "seed 0; F1 FULL",
           "z_laps_per_iter": T, "laps_per_iter": T + n * n + 1, "z_entries": T * m * m,
           "zlap_mapping": mapping,
           "cold": {"iterations": len(cold_tr), "timed_iterations": done, "iterations_per_s": done / el,
                    "ms_per_step": 1e3 * per_it, "laps_per_s": (T + n * n + 1) * done / el,
                    "phase_ms_per_iter": phase_ms,
                    "phase_gbs": {k: ab[k] / (phase_ms[k] * 1e-3) / 1e9 for k in ("zlap", "sweep")},
                    "dijkstra_steps_per_lap": r["dijkstra_steps"] / max(1, done * (T + n * n + 1)),
                    "zlap_dijkstra_steps_per_s": r["dijkstra_steps"] / max(1e-12, r["ms_zlap"] * 1e-3),
                    "iteration_hbm_minimal": {"bytes": minimal_iteration_bytes(n),
                                              "achieved_gbs": minimal_iteration_bytes(n) / per_it / 1e9,
                                              "frac": minimal_iteration_bytes(n) / per_it / 1e9 / HBM_PEAK_GBS},
                    "iteration_hbm_schedule": {"bytes": sum(ab.values()),
                                               "achieved_gbs": sum(ab.values()) / per_it / 1e9,
                                               "frac": sum(ab.values()) / per_it / 1e9 / HBM_PEAK_GBS},
                    "lb_every": {str(k): float(cold_tr[k - 1]) for k in range(every, len(cold_tr) + 1, every)},
                    "lb": float(cold_tr[-1])}}
    if not os.path.exists(train_warm.WEIGHTS):
        out["warm"] = {"skipped": "no trained weights"}
        return out
    # the cold side on the production path (graph replay), for the wall time
    # (the Z-LAP mapping chosen by the first handle is kept for the process)
    c = binding.DualAscent(F, D, B)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c.run(cold_iters)
    cold_s = time.perf_counter() - t0
    assert np.array_equal(c.trace(), cold_tr), "graph replay and timed run disagree"
    c.close()
    mlp = binding.Mlp(train_warm.load_weights(), max_batch=256)
    w = binding.DualAscent(F, D, B)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = w.warm_start(mlp)
    w.run(cold_iters)
    wel = time.perf_counter() - t0
    warm_tr = w.trace()
    w.close()
    best = np.maximum.accumulate(warm_tr)
    hit = np.nonzero(best >= cold_tr[-1])[0]
    reached = None
    if len(hit):
        k = int(hit[0]) + 1
        w = binding.DualAscent(F, D, B)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        w.warm_start(mlp)
        rr = w.run(k)
        kel = time.perf_counter() - t0
        w.close()
        reached = {"iterations": k, "seconds": kel, "lb": rr["lb"]}
    mlp.close()
    flops = 2.0 * binding.orbit_count(n) * (32 * 256 + 256 * 256 + 256 * 6)
    out["warm"] = {"iterations": len(warm_tr), "seconds_with_start": wel, "start_seconds": st["seconds"],
                   "ms_mlp": st["ms_mlp"], "ms_write": st["ms_write"],
                   "mlp_tflops": flops / (st["ms_mlp"] * 1e-3) / 1e12,
                   "lb_t0": float(warm_tr[0]),
                   "lb_every": {str(k): float(best[k - 1]) for k in range(every, len(best) + 1, every)},
                   "lb": float(best[-1]), "to_cold_lb": reached}
    out["time_to_cold_bound"] = {"cold_iterations": len(cold_tr), "cold_seconds": cold_s,
                                 "warm_seconds": reached["seconds"] if reached else None,
                                 "speedup": cold_s / reached["seconds"] if reached else None}
    return out


def variant_leg(inst, label: str, make_params, z_laps: int, ab: dict, steps: int, warmup: int,
                full_trace, cold_iters: int, stream):
    """One variant of the ascent on the same workload: iterations/s with the
    same warmup and step count, its per-phase HBM rates against its own
    algorithmic bytes, its bound against FULL F1's after as many iterations,
    and the wall time it needs to reach the F1 bound of `cold_iters`
    iterations (if it does within 3 x cold_iters) against F1's time for
    those iterations."""
    import torch

    from paper_1710_03732_amd import binding

    F, D, B = inst.arrays()
    n = inst.n
    h = binding.DualAscent(F, D, B, params=make_params(timing=1))
    h.set_stream(stream.cuda_stream)
    if warmup > 0:
        h.run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = h.run(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    done = r["iterations_done"]
    h.close()
    if done <= 0:
        return {"skipped": "bound proved optimal during warmup"}
    phase_ms = {"sweep": r["ms_sweep"] / done, "zlap": r["ms_zlap"] / done,
                "ylap": r["ms_ylap"] / done, "xlap": r["ms_xlap"] / done}
    out = {"iterations_per_s": done / el, "ms_per_step": 1e3 * el / done,
           "laps_per_s": r["laps"] / el, "z_laps_per_iter": z_laps,
           "phase_ms_per_iter": phase_ms,
           "phase_gbs": {k: ab[k] / (phase_ms[k] * 1e-3) / 1e9 for k in ("zlap", "sweep")},
           "lb_after": r["lb"], "lb_f1_after_same_iterations": full_trace[-1] if len(full_trace) else None}
    # time to F1's bound after cold_iters iterations (plain handles, graph replay)
    if len(full_trace) >= cold_iters:
        target = float(full_trace[cold_iters - 1])
        probe = binding.DualAscent(F, D, B, params=make_params())
        probe.run(3 * cold_iters)
        tr = probe.trace()
        probe.close()
        need = next((k + 1 for k, v in enumerate(tr) if v >= target), None)
        res = {"target_lb": target, "f1_iterations": cold_iters, f"{label}_iterations": need}
        timed = {}
        for who, prm, iters in (("f1", binding.default_params(), cold_iters), (label, make_params(), need)):
            if not iters:
                continue
            hd = binding.DualAscent(F, D, B, params=prm)  # own stream: graph replay
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hd.run(iters)  # returns after synchronising the handle's stream
            timed[who] = time.perf_counter() - t0
            hd.close()
        res["f1_seconds"] = timed["f1"]
        res[f"{label}_seconds"] = timed.get(label)
        res["speedup"] = timed["f1"] / timed[label] if label in timed else None
        out["time_to_f1_bound"] = res
    return out


def annealing_leg(inst, iters: int = 300, seed: int = 1):
    """Type 4 steps with Section 5's schedule (t0 = 4 % of the incumbent
    after two iterations, kappa_max 0.25, cooling 0.99 per 100 iterations)
    against plain runs: best bound after `iters` iterations and wall time,
    for F1 and for F2 (the paper's strongest combination)."""
    from paper_1710_03732_amd import binding

    F, D, B = inst.arrays()
    out = {"iterations": iters, "seed": seed}
    for label, kw in (("f1", {}), ("f2", {"two_phase": 1})):
        for sa in (False, True):
            h = binding.DualAscent(F, D, B, **kw)
            t0 = time.perf_counter()
            r = h.run(2)
            if sa:
                h.set_annealing(0.04 * r["ub"], seed=seed)
            r = h.run(iters - 2)
            el = time.perf_counter() - t0
            h.close()
            out[label + ("_sa" if sa else "")] = {"best_lb": r["best_lb"], "ub": r["ub"], "seconds": el,
                                                  "type4_steps": r["sa_steps"]}
    return out


def variant_legs(inst, steps: int, warmup: int, full_trace, cold_iters: int, stream):
    """HALF (Section 5: only the Z-LAPs of tiles with i < j) and the
    two-phase F2 (Section 3.4: solve, pool each orbit's slacks, solve)."""
    from paper_1710_03732_amd import binding

    n = inst.n
    T = n * n * (n - 1) * (n - 1)
    V = T * (n - 2) * (n - 2)
    f1 = algorithmic_bytes(n)
    f2_bytes = dict(f1, zlap=2 * f1["zlap"] + 8 * 2 * V)  # two solves and the pooling pass
    # S1's sweep also reads and writes the multipliers v; its reset writes the x/y costs
    s1_bytes = dict(f1, sweep=8 * (4 * V + T + n * n) + 8 * (T + 2 * n * n))
    return {
        "half": variant_leg(inst, "half", binding.half_params, T // 2, algorithmic_bytes_half(n), steps,
                            warmup, full_trace, cold_iters, stream),
        "f2": variant_leg(inst, "f2", lambda **kw: binding.default_params(two_phase=1, **kw), 2 * T, f2_bytes,
                          steps, warmup, full_trace, cold_iters, stream),
        "s1": variant_leg(inst, "s1", lambda **kw: binding.default_params(slow=1, **kw), T, s1_bytes,
                          steps, warmup, full_trace, cold_iters, stream),
        "s2": variant_leg(inst, "s2", lambda **kw: binding.default_params(slow=1, two_phase=1, **kw), 2 * T,
                          dict(s1_bytes, zlap=f2_bytes["zlap"] + 8 * 2 * V), steps, warmup, full_trace, cold_iters,
                          stream),
        "annealing": annealing_leg(inst),
    }


def bnb_leg():
    """Branch-and-bound: the n = 14 dense instance with forced branching (4
    iterations per node, batches of up to 256 nodes of mixed depth) and with
    the default settings (the root bound closes it), the n = 18 dense
    instance (seed 0) with the default settings, and a 4x4 grid instance
    (n = 16) with and without Section 4's symmetry elimination."""
    from paper_1710_03732_amd import binding, instances as insts

    out = {}
    runs = (("dense_n14_branching", insts.dense_n14(), dict(batch=256, node_iters=4, window=25)),
            ("dense_n14_default", insts.dense_n14(), {}),
            ("dense_n18_default", insts.dense_instance(18, 0), {}),
            ("grid4x4_n16_default", insts.grid_instance(16, 4, 4, 0.4, 1, 9, 1), {}),
            ("grid4x4_n16_symmetry", insts.grid_instance(16, 4, 4, 0.4, 1, 9, 1), dict(symmetry=1)))
    for label, inst, kw in runs:
        F, D, B = inst.arrays()
        h = binding.DualAscent(F, D, B)
        t0 = time.perf_counter()
        obj, perm, st = h.bnb_solve(**kw)
        el = time.perf_counter() - t0
        h.close()
        out[label] = {"optimum": obj, "seconds": el, "nodes": st["nodes"], "batches": st["batches"],
                      "da_iterations": st["da_iters"], "nodes_per_s": st["nodes"] / el,
                      "node_iterations_per_s": st["da_iters"] / el,
                      "node_iteration_bytes": st["node_bytes"],
                      "bytes_per_node_iteration": st["node_bytes"] / max(1, st["da_iters"]),
                      "algorithmic_gbs_over_wall_time": st["node_bytes"] / el / 1e9,
                      "symmetric_skipped": st["symmetric_skipped"], **kw}
    return out


def mapping_text(da) -> str:
    """The Z-LAP mapping the handle used and how it was chosen."""
    lanes, cols, us = da.zlap_mapping()
    what = {-1: "one LAP per wavefront", -2: "two LAPs per wavefront"}.get(lanes, f"{lanes}-lane groups x {cols} cols")
    if us >= 0:
        return f"{what} (autotuned: {us:.0f} us on the tuning batch)"
    return f"{what} ({'requested' if da.params.zlap_lanes else 'rule-based'})"


def measure_copy_gbs(nbytes: int = 1 << 31, reps: int = 5) -> float:
    """Read + write GB/s of a plain device copy of nbytes, best of reps
    after one warm-up: the practical bandwidth beside the 8 TB/s peak."""
    import torch

    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    best = None
    for rep in range(reps + 1):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        if rep > 0 and (best is None or ms < best):
            best = ms
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (best * 1e-3) / 1e9


def calibrate_copy(nbytes: int = 1 << 31):
    """A plain device copy of known size, for scaling PMC byte counters."""
    import torch

    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    return nbytes


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="dense_n30",
                    help="dense_n30 | grid_n30 | dense_n42 | grid_n15 | ...")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--zlap-lanes", type=int, default=0)
    ap.add_argument("--zlap-cols", type=int, default=0)
    ap.add_argument("--no-time-to-bound", action="store_true")
    ap.add_argument("--no-bnb", action="store_true", help="skip the branch-and-bound leg (n = 14 and 18)")
    ap.add_argument("--no-variants", action="store_true", help="skip the HALF and F2 legs")
    ap.add_argument("--no-n42", action="store_true", help="skip the n = 42 plain vs warm leg")
    ap.add_argument("--cold-iters", type=int, default=100,
                    help="cold iterations whose bound the learned warm start must reach")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 2 GiB device copy (PMC counter calibration)")
    ap.add_argument("--oracle-sizes", action="store_true",
                    help="also time the CPU oracle at n = 15 (200 iterations) and n = 42 (2 iterations)")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only (--gpus 1); sharding the dual ascent over "
              "several GPUs is not implemented", file=sys.stderr)
        return 2

    import torch

    from paper_1710_03732_amd import binding, instances

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    inst = instances.named(args.workload)
    F, D, B = inst.arrays()
    n = inst.n
    m = n - 2
    T = n * n * (n - 1) * (n - 1)
    V = T * m * m
    laps_per_iter = T + n * n + 1

    if args.calibrate_copy:
        calibrate_copy()

    stream = torch.cuda.current_stream()
    da = binding.DualAscent(F, D, B, timing=1, zlap_lanes=args.zlap_lanes,
                            zlap_cols=args.zlap_cols)
    da.set_stream(stream.cuda_stream)
    if args.warmup > 0:
        da.run(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = da.run(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    done = r["iterations_done"]
    if done <= 0:
        print("bench.py: the bound proved optimality during warmup; nothing timed",
              file=sys.stderr)
        return 1
    its = done / el
    phase_ms = {"sweep": r["ms_sweep"] / done, "zlap": r["ms_zlap"] / done,
                "ylap": r["ms_ylap"] / done, "xlap": r["ms_xlap"] / done}
    ab = algorithmic_bytes(n)
    dom = max(("zlap", "sweep"), key=lambda k: phase_ms[k])
    dom_s = phase_ms[dom] / 1e3
    achieved = ab[dom] / dom_s / 1e9
    traffic = load_traffic(dom, inst.name)
    iter_bytes = sum(ab.values())
    min_bytes = minimal_iteration_bytes(n)
    full_trace = da.trace()
    copy_gbs = measure_copy_gbs()  # after the timed region
    steps_per_zlap = r["dijkstra_steps"] / max(1, done * laps_per_iter)

    out = {
        "metric": "RLT2 dual-ascent iters/s + LAPs/s at n=30 FP64; time-to-bound warm vs cold",
        "value": its,
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / done,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{inst.name}: QAP n={n} root dual ascent, "
                        + ("dense symmetric F,D~U{0..99}, zero diagonals, seed 0"
                           if inst.name.startswith("dense") else "grid Manhattan D, sparse flows")
                        + "; F1 one-phase RLT2-DA, FULL scheme (all Z-LAPs)",
            "n": n,
            "z_laps_per_iter": T,
            "laps_per_iter": laps_per_iter,
            "z_entries": V,
            "zlap_mapping": mapping_text(da),
        },
        "laps_per_s": its * laps_per_iter,
        "iterations_done": done,
        "phase_ms_per_iter": phase_ms,
        "lb_after": r["lb"],
        "ub": r["ub"],
        "gap": r["gap"],
        "dijkstra_steps_per_lap": steps_per_zlap,
        "zlap_issue": {"dijkstra_steps_per_s": r["dijkstra_steps"] / max(1e-12, r["ms_zlap"] * 1e-3),
                       "z_laps_per_s": T * done / max(1e-12, r["ms_zlap"] * 1e-3),
                       "ms_per_launch": phase_ms["zlap"]},
        "iteration_hbm": {"minimal_schedule_bytes": min_bytes,
                          "minimal_achieved_gbs": min_bytes / (el / done) / 1e9,
                          "minimal_frac": min_bytes / (el / done) / 1e9 / HBM_PEAK_GBS,
                          "schedule_bytes": iter_bytes, "achieved_gbs": iter_bytes / (el / done) / 1e9,
                          "frac": iter_bytes / (el / done) / 1e9 / HBM_PEAK_GBS,
                          "copy_gbs": copy_gbs, "frac_of_copy": iter_bytes / (el / done) / 1e9 / copy_gbs,
                          "minimal_frac_of_copy": min_bytes / (el / done) / 1e9 / copy_gbs},
        "roofline": {"bound": "hbm", "kernel": {"zlap": "k_zlap", "sweep": "k_sweep+k_scale_xy"}[dom],
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": ab[dom],
                     "avg_launch_ms": phase_ms[dom], "frac_of_copy": achieved / copy_gbs},
        "graph_replay": None,
        "variants": None,
        "bnb": None,
        "time_to_bound": None,
        "n42": None,
        "cpu_baseline": None,
        "oracle_sizes": None,
    }
    da.close()
    out["graph_replay"] = graph_replay_leg(inst, args.steps, args.warmup, full_trace)
    if not args.no_variants:
        out["variants"] = variant_legs(inst, args.steps, args.warmup, full_trace, args.cold_iters, stream)
    if not args.no_bnb and inst.name == "dense_n30":
        out["bnb"] = bnb_leg()
    if not args.no_time_to_bound:
        from paper_1710_03732_amd import instances as insts

        ttb = {inst.name: warm_vs_cold(inst, args.cold_iters)}
        if inst.name == "dense_n30":  # the headline's second instance
            ttb["grid_n30"] = warm_vs_cold(insts.grid_n30(), args.cold_iters)
        out["time_to_bound"] = ttb
    if not args.no_n42 and inst.name == "dense_n30":
        out["n42"] = n42_leg(args.cold_iters)
    if not args.no_cpu_baseline:
        torch.cuda.synchronize()
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_threads or None, full_trace)
    if args.oracle_sizes:
        out["oracle_sizes"] = oracle_sizes_leg()
    print(json.dumps(out), flush=True)
    par = (out["cpu_baseline"] or {}).get("gpu_parity")
    if par is not None and par["gpu_lb"] is not None and not par["within_1e-9"]:
        print(f"bench.py: the GPU bound {par['gpu_lb']!r} differs from the oracle's {par['oracle_lb']!r} "
              f"after {par['iterations']} iterations", file=sys.stderr)
        return 3
    return 0


if __name__ == "__main__":
    sys.exit(main())
