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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="dense_uniform")
    ap.add_argument("--profile-steps", type=int, default=10)
    ap.add_argument("--cpu-sample", type=int, default=262144)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
