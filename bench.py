"""Throughput of the ORCA step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one pass of the whole path over every agent: binning, neighbour
gather, half-planes and 2D LP, fallback, Euler update and goal steering.
Default workload: 1,048,576 agents uniform at 2 agents/m^2 (K = 16,
neighbor_dist = 3 m), inputs resident on the GPU before timing starts.

Prints one JSON line with the throughput (agent-steps/s), the roofline of the
dominant stage (per-stage times from HIP events recorded on the library's
stream) and the CPU reference's rate on a bounded sample of the same state.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "agent-steps/s at 1M agents (plain vs batched vs fwd+adjoint, 1e-4 m/s)"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6

# Algorithmic bytes per agent of each stage (every array touched once; the
# neighbours' re-reads are cache traffic, not counted).  K = neighbour cap.
#   binning:    bbox 8 + key pass 28 + scatter 60          = 96 per agent, + 12 per cell
#   neighbours: own row 28 + list 4K + count 4              = 32 + 4K
#   lp2d:       own row 36 + list 4K + goal 8 + outputs 24  = 68 + 4K
#   fallback:   the same for each fallback agent, + list 4  = 72 + 4K
def stage_bytes(stage: int, n: int, k: int, cells: int, n_fallback: float) -> float:
    if stage == 0:
        return 96.0 * n + 12.0 * cells
    if stage == 1:
        return (32.0 + 4.0 * k) * n
    if stage == 2:
        return (68.0 + 4.0 * k) * n
    return (72.0 + 4.0 * k) * n_fallback


def make_workload(name: str):
    from paper_1908_10107_amd import scenes
    if name == "dense_uniform":
        return scenes.dense_uniform()
    if name == "uniform_rsa":
        return scenes.uniform_rsa()
    if name == "ring":
        return scenes.ring()
    if name == "batched":
        return scenes.batched()
    raise SystemExit("unknown workload %s" % name)


def cpu_baseline(w, sample: int):
    """The reference's rate on one step of ``sample`` agents of the same state."""
    import oracle
    rng = np.random.default_rng(0)
    agents = np.sort(rng.choice(w.n, size=min(sample, w.n), replace=False))
    t0 = time.perf_counter()
    oracle.velocities(w.pos, w.vel, w.pref_vel, w.offsets, w.params, goals=w.goals,
                      agents=agents, neighbor_mode=1)
    dt = time.perf_counter() - t0
    return dict(value=len(agents) / dt, unit="agent-steps/s", cores=oracle.threads(),
                kind="oracle",
                sample="one step of %d of the %d agents from the initial state (binning of all "
                       "agents included), %.1f s" % (len(agents), w.n, dt))


def batched_forms(steps: int, no_autotune: bool):
    """512 independent scenes: one graph-replayed launch sequence per step over
    all scenes, against stepping each scene with its own plain orca_step."""
    import torch
    from paper_1908_10107_amd import orca, scenes
    w = scenes.batched()
    kmax = max(p.max_neighbors for p in w.params)
    d = orca.to_device(w)
    ctx = orca.Context(max_agents=w.n, max_scenes=w.n_scenes, k_max=kmax)
    tuned = None
    if not no_autotune:
        ctx.build_grid(w.offsets, w.params, d["pos"])
        tuned = ctx.autotune(d["pos"], d["vel"], d["pref_vel"], goals=d["goals"], reps=2)
    ctx.step_graph(w.offsets, w.params, d["pos"], d["vel"], d["pref_vel"], goals=d["goals"],
                   n_steps=3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step_graph(w.offsets, w.params, d["pos"], d["vel"], d["pref_vel"], goals=d["goals"],
                   n_steps=steps)
    torch.cuda.synchronize()
    gw = time.perf_counter() - t0
    ctx.close()
    # per-scene plain forward, one context per scene (no re-uploads between calls)
    per = []
    for s in range(w.n_scenes):
        one = w.subset_scenes([s])
        c = orca.Context(max_agents=max(one.n, 1), max_scenes=1, k_max=kmax)
        per.append((one, c, orca.to_device(one)))
    for one, c, t in per:
        c.step(one.offsets, one.params, t["pos"], t["vel"], t["pref_vel"], goals=t["goals"])
    torch.cuda.synchronize()
    ps = max(2, steps // 4)
    t0 = time.perf_counter()
    for _ in range(ps):
        for one, c, t in per:
            c.step(one.offsets, one.params, t["pos"], t["vel"], t["pref_vel"], goals=t["goals"])
    torch.cuda.synchronize()
    pw = time.perf_counter() - t0
    for _, c, _ in per:
        c.close()
    bg = w.n * steps / gw
    bp = w.n * ps / pw
    return {"batched_graph": {"value": bg, "ms_per_step": 1e3 * gw / steps, "agents": w.n,
                              "scenes": w.n_scenes, "steps": steps,
                              "autotune": None if tuned is None else list(tuned)},
            "batched_per_scene_plain": {"value": bp, "ms_per_step": 1e3 * pw / ps, "steps": ps},
            "batched_speedup": bg / bp}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="dense_uniform")
    ap.add_argument("--profile-steps", type=int, default=10)
    ap.add_argument("--cpu-sample", type=int, default=262144)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="plain,batched",
                    help="comma list: plain (always), batched (512 scenes, graph replay vs "
                         "per-scene plain steps)")
    ap.add_argument("--batched-steps", type=int, default=20)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one elementwise copy of 256 MiB (reads and writes known bytes) "
                         "to scale hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1908_10107_amd import orca

    w = make_workload(args.workload)
    kmax = max(p.max_neighbors for p in w.params)
    print("# workload %s: %d agents, %d scenes" % (args.workload, w.n, w.n_scenes),
          file=sys.stderr, flush=True)
    base = orca.to_device(w)
    ctx = orca.Context(max_agents=w.n, max_scenes=w.n_scenes, k_max=kmax)
    st = dict(pos=base["pos"].clone(), vel=base["vel"].clone(), pref=base["pref_vel"].clone())
    step = lambda k: ctx.step(w.offsets, w.params, st["pos"], st["vel"], st["pref"],
                              goals=base["goals"], n_steps=k)
    tuned = None
    if not args.no_autotune:
        ctx.build_grid(w.offsets, w.params, st["pos"])
        tuned = ctx.autotune(st["pos"], st["vel"], st["pref"], goals=base["goals"], reps=2)
    if args.warmup:
        step(args.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    step(args.steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    ms_per_step = 1e3 * wall / args.steps
    value = w.n * args.steps / wall
    print("# timed %d steps: %.3f s wall, %.3f s on the stream" % (args.steps, wall,
                                                                  gpu_ms / 1e3),
          file=sys.stderr, flush=True)

    # per-stage timing on a separate pass (each step waits for its stream)
    ctx.profile(True)
    step(args.profile_steps)
    ms, passes, fb = ctx.profile_read()
    ctx.profile(False)
    avg = [m / max(passes, 1) for m in ms]
    fb_avg = fb / max(passes, 1)
    dom = int(np.argmax(avg))
    cells = 4 * w.n  # upper bound of the cell budget; the 12 B/cell term is small
    alg = stage_bytes(dom, w.n, kmax, cells, fb_avg)
    achieved = alg / (avg[dom] * 1e-3) / 1e9
    stages = {orca.STAGE_NAMES[i]: round(avg[i], 4) for i in range(orca.PROF_STAGES)}
    roofline = dict(bound="hbm", achieved=round(achieved, 3), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 6), traffic=None,
                    kernel="k_fallback" if dom == 3 else ("k_lp" if dom == 2 else
                                                          ("k_knn" if dom == 1 else "binning")),
                    stage_ms=stages, fallback_agents_per_step=round(fb_avg, 1))

    # the same plain step replayed from a captured graph (launch cost only differs)
    gstep = lambda k: ctx.step_graph(w.offsets, w.params, st["pos"], st["vel"], st["pref"],
                                     goals=base["goals"], n_steps=k)
    gstep(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gstep(args.steps)
    torch.cuda.synchronize()
    gwall = time.perf_counter() - t0
    forms = {"plain_graph": {"value": w.n * args.steps / gwall,
                             "ms_per_step": 1e3 * gwall / args.steps}}
    ctx.close()
    del st, base
    if "batched" in args.forms.split(","):
        forms.update(batched_forms(args.batched_steps, args.no_autotune))

    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = src * 1.0
        torch.cuda.synchronize()
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, args.cpu_sample)

    line = {
        "metric": METRIC, "value": value, "unit": "agent-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "agents": w.n, "scenes": w.n_scenes,
                   "max_neighbors": kmax,
                   "neighbor_dist": w.params[0].neighbor_dist,
                   "state": "f32", "lp": "f64", "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "autotune": None if tuned is None else {"knn_block": tuned[0],
                                                "fallback_waves_per_cu": tuned[1]},
        "forms": forms,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
