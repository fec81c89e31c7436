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
import dataclasses
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

# Algorithmic work of each stage.
#   binning (HBM): bbox 8 + key pass 28 + scatter 56 = 92 B per agent, + 12 B per cell.
#   neighbours (HBM figure): own row 24 + list 4K + count 4 = 28 + 4K B per agent.
#   half-planes + 2D LP (FP64 ALU): 29.2 K + 15.5 K operations per agent
#     (half-plane construction; projection and the choice of the fallback's
#     first plane; 715 at K = 16).
#   fallback (FP64 ALU): 28.7 K operations per fallback agent (460 at K = 16).
# The FP64 operation counts come from the kernels' own programs built for the
# host with their work-counting hooks (csrc/orca_work_count.cpp), run on 4,000
# agents of an evolved dense state; tests/test_work_counts.py recounts them
# and holds these constants to 3%.
HP_OPS_PER_K = 29.2
LP2_OPS_PER_K = 15.5
FB_OPS_PER_K = 28.7


def stage_roofline(stage: int, ms: float, n: int, k: int, cells: int, n_fallback: float):
    """(bound, achieved, peak, unit) of one stage at its average duration ms."""
    s = ms * 1e-3
    if stage == 0:
        return "hbm", (92.0 * n + 12.0 * cells) / s / 1e9, HBM_PEAK_GBS, "GB/s"
    if stage == 1:
        return "hbm", (28.0 + 4.0 * k) * n / s / 1e9, HBM_PEAK_GBS, "GB/s"
    if stage == 2:
        return "alu", (HP_OPS_PER_K + LP2_OPS_PER_K) * k * n / s / 1e12, FP64_PEAK_TFLOPS, "TFLOP/s"
    return "alu", FB_OPS_PER_K * k * n_fallback / s / 1e12, FP64_PEAK_TFLOPS, "TFLOP/s"


PROFILE_MD = os.path.join(ROOT, "profiles", "dense_uniform_1M_kernels.md")
KERNEL_SOURCES = ("paper_1908_10107_amd/csrc/orca_kernels.hip", "paper_1908_10107_amd/csrc/orca_lp.h",
                  "paper_1908_10107_amd/csrc/orca_internal.h")


def profiled_traffic(kernel: str):
    """HBM bytes per dispatch of ``kernel`` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a copy kernel), or None when
    the kernel sources have changed since the counters were taken."""
    import hashlib
    try:
        text = open(PROFILE_MD).read()
    except OSError:
        return None
    d = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            d.update(fh.read())
    if "kernel-source-sha256: %s " % d.hexdigest()[:16] not in text:
        return None
    tag = "traffic-bytes-per-dispatch %s: " % kernel
    for line in text.splitlines():
        if line.startswith(tag):
            return float(line[len(tag):])
    return None


def profiled_lane_use():
    """VALU lane utilisation per kernel from the committed counter summary,
    or None when the kernel sources have changed since it was taken."""
    import hashlib
    try:
        text = open(PROFILE_MD).read()
    except OSError:
        return None
    d = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            d.update(fh.read())
    if "kernel-source-sha256: %s " % d.hexdigest()[:16] not in text:
        return None
    out = {}
    for line in text.splitlines():
        if line.startswith("lane-use "):
            k, v = line[len("lane-use "):].split(": ")
            out[k] = float(v)
    return out or None


def grid_cells(w, margin=1.0 + 1.0 / 1024.0):
    """Grid cells of the current positions: per scene, cells of side
    neighbor_dist * margin / c over the bounding box, with the library's
    choice of c = 2, 3 or 4 cells per neighbor_dist (the 3 x 3 cells around an
    agent hold about 2.75 K agents at the scene's mean density)."""
    c = 0
    per_nd = {}
    for s, p in enumerate(w.params):
        lo, hi = int(w.offsets[s]), int(w.offsets[s + 1])
        if hi <= lo:
            c += 1
            continue
        x = w.pos[:, lo:hi].astype(np.float64)
        nd = float(np.float32(p.neighbor_dist))
        ext = x.max(axis=1) - x.min(axis=1)
        cpn = 2
        if p.max_neighbors > 0:
            rho = (hi - lo) / max(ext[0] * ext[1], nd * nd)
            cpn = int(min(max(np.rint(nd * np.sqrt(9.0 * rho / (2.75 * p.max_neighbors))), 2), 4))
        side = nd * margin / cpn
        c += int((np.floor(ext[0] / side) + 1) * (np.floor(ext[1] / side) + 1))
        per_nd[cpn] = per_nd.get(cpn, 0) + 1
    return c, per_nd


def apply_launch(ctx, launch):
    """Fixed launch shapes: (knn_block, fallback waves per CU[, agents per lane,
    velocity waves per CU[, fallback work units]]) as orca_autotune returns them."""
    if not launch:
        return
    ctx.set_launch(launch[0], launch[1])
    if len(launch) >= 4:
        ctx.set_kernels(launch[2], launch[3], launch[4] if len(launch) >= 5 else 0)


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


def host_cpu():
    """Logical CPUs of the host, those this process may use, and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return dict(nproc=os.cpu_count(), usable=usable, model=model)


def cpu_baseline(w, min_seconds: float, evolved=None):
    """The reference (float64 C, OpenMP over agents) on the host's cores.

    value: whole steps of the timed workload from its initial state (binning,
    velocities, Euler, steering), stepped one at a time until ``min_seconds``
    have passed, on every thread.  Also: three whole steps from the GPU's
    state at the end of the timed steps (``evolved``: pos, vel, pref_vel, the
    crowd the GPU figure was measured on); one thread on a 100,000-agent
    sample of the initial state; the 1,024-agent square's whole 100-step
    run; the 4,096-agent 200-step trajectory with its forward-mode
    derivative."""
    import oracle
    from paper_1908_10107_amd import scenes
    threads = oracle.threads()
    pos, vel, pref = w.pos, w.vel, w.pref_vel
    steps = 0
    t0 = time.perf_counter()
    while True:
        pos, vel, pref, _ = oracle.step(pos, vel, pref, w.offsets, w.params, goals=w.goals)
        steps += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds or steps >= 200:
            break
    out = dict(value=w.n * steps / dt, unit="agent-steps/s", cores=threads, kind="oracle",
               sample="%d whole steps of all %d agents from the initial state, %.1f s"
                      % (steps, w.n, dt), host=host_cpu())
    if evolved is not None:
        pos, vel, pref = evolved
        t0 = time.perf_counter()
        oracle.step(pos, vel, pref, w.offsets, w.params, goals=w.goals, n_steps=3)
        de = time.perf_counter() - t0
        out["evolved"] = dict(value=w.n * 3 / de, unit="agent-steps/s", cores=threads,
                              sample="3 whole steps of all %d agents from the GPU's state after "
                                     "the timed steps, %.1f s" % (w.n, de))
    # one thread, velocities of a sample of the same initial state
    rng = np.random.default_rng(1)
    m = min(w.n, 100000)
    agents = np.sort(rng.choice(w.n, m, replace=False))
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.velocities(w.pos, w.vel, w.pref_vel, w.offsets, w.params, goals=w.goals,
                          agents=agents)
        d1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(threads)
    out["one_thread"] = dict(value=m / d1, unit="agent-steps/s", cores=1,
                             sample="velocities of %d sampled agents of the initial state "
                                    "(binning included), %.1f s" % (m, d1))
    # the 1,024-agent square, all 100 steps
    u = scenes.uniform_rsa()
    t0 = time.perf_counter()
    oracle.step(u.pos, u.vel, u.pref_vel, u.offsets, u.params, goals=u.goals, n_steps=u.steps)
    du = time.perf_counter() - t0
    out["uniform_rsa_1024x100"] = dict(value=u.n * u.steps / du, unit="agent-steps/s",
                                       cores=threads, seconds=round(du, 3))
    # the differentiable workload: forward with one forward-mode tangent
    g = scenes.grad()
    p = g.params[0]
    r = np.random.default_rng(2)
    t0 = time.perf_counter()
    oracle.traj_jvp(g.pos.astype(np.float64), g.vel.astype(np.float64),
                    g.pref_vel.astype(np.float64), g.offsets, g.params,
                    np.array([p.max_speed], float), np.array([p.time_horizon], float), g.steps,
                    g.targets, r.normal(size=g.pref_vel.shape), np.ones(1), np.ones(1))
    dg = time.perf_counter() - t0
    out["grad_4096x200_forward_mode"] = dict(value=g.n * g.steps / dg, unit="agent-steps/s",
                                             cores=threads, seconds=round(dg, 3))
    return out


def full_length_forms(launch):
    """Each workload over its whole length from t = 0 in one call (one
    orca_step of all steps, or graph replays), the two smaller ones both
    ways: at their sizes a step's kernels are short enough for the host's
    launches to show."""
    import torch
    from paper_1908_10107_amd import orca, scenes
    out = {}
    for name, make, graph in (("uniform_rsa_1024x100", scenes.uniform_rsa, False),
                              ("uniform_rsa_1024x100_graph", scenes.uniform_rsa, True),
                              ("ring_65536x2000", scenes.ring, False),
                              ("ring_65536x2000_graph", scenes.ring, True),
                              ("dense_1M_x500", scenes.dense_uniform, False),
                              ("batched_512x300", scenes.batched, True)):
        w = make()
        kmax = max(p.max_neighbors for p in w.params)
        d = orca.to_device(w)
        ctx = orca.Context(max_agents=w.n, max_scenes=w.n_scenes, k_max=kmax)
        apply_launch(ctx, launch)
        fn = ctx.step_graph if graph else ctx.step
        kw = {} if graph else {"save_tape": False}
        if graph:
            # capture the graph (one step), then put the initial state back in
            # place: the timed replays start at t = 0 on the captured pointers
            init = {k: d[k].clone() for k in ("pos", "vel", "pref_vel")}
            ctx.step_graph(w.offsets, w.params, d["pos"], d["vel"], d["pref_vel"],
                           goals=d["goals"], n_steps=1)
            for k in init:
                d[k].copy_(init[k])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn(w.offsets, w.params, d["pos"], d["vel"], d["pref_vel"], goals=d["goals"],
           n_steps=w.steps, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.close()
        out[name] = {"value": w.n * w.steps / dt, "ms_per_step": 1e3 * dt / w.steps,
                     "agents": w.n, "scenes": w.n_scenes, "steps": "0-%d" % (w.steps - 1),
                     "launch": "graph replays" if graph else "one orca_step call"}
    return out


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
        tuned = ctx.autotune(d["pos"], d["vel"], d["pref_vel"], goals=d["goals"], reps=5)
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


def adjoint_forms():
    """Forward + adjoint: the 4,096-agent 200-step trajectory with checkpoints
    every 20 steps, and one 20-step segment at 1,048,576 agents.  A step of
    the forward counts once; the time includes the checkpointed forward, the
    recorded replay and the adjoint steps."""
    import torch
    from paper_1908_10107_amd import autograd, orca, scenes
    out = {}
    for name, w, steps in (("grad_4096x200", scenes.grad(), 200),
                           ("dense_1M_segment20", scenes.dense_uniform(), 20)):
        if name.startswith("dense"):
            w.goals = None  # fixed preferred velocities for the differentiable form
            rng = np.random.default_rng(4)
            a = rng.uniform(0, 2 * np.pi, w.n)
            w.pref_vel = np.ascontiguousarray((1.3 * np.stack([np.cos(a), np.sin(a)]))
                                              .astype(np.float32))
        d = orca.to_device(w)
        p = w.params[0]
        spec = autograd.TrajectorySpec(offsets=list(w.offsets), params=list(w.params),
                                       n_steps=steps, segment=20)

        def run():
            pref = d["pref_vel"].clone().requires_grad_(True)
            vmax = torch.tensor([p.max_speed], device="cuda", requires_grad=True)
            tau = torch.tensor([p.time_horizon], device="cuda", requires_grad=True)
            pos, vel = autograd.trajectory(d["pos"], d["vel"], pref, vmax, tau, spec)
            (pos.double() ** 2).sum().backward()
            return pref.grad

        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 3 if w.n < 100000 else 1
        for _ in range(reps):
            run()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out[name] = {"value": w.n * steps / dt, "unit": "agent-steps/s", "agents": w.n,
                     "steps": steps, "ms_per_step": 1e3 * dt / steps, "segment": 20}
        spec.ctx.close()
    return out


def hetero_forms(steps: int, launch):
    """The two-way crossing whose people differ in size and speed (section 4),
    262,144 agents: plain steps with per-agent radius, max speed and walking
    speed."""
    import torch
    from paper_1908_10107_amd import orca, scenes
    w = scenes.crossing_hetero(n=1 << 18)
    d = orca.to_device(w)
    ctx = orca.Context(max_agents=w.n, max_scenes=1, k_max=w.params[0].max_neighbors)
    ctx.set_agents(d["radius"], d["max_speed"], d["pref_speed"])
    apply_launch(ctx, launch)
    step = lambda k: ctx.step(w.offsets, w.params, d["pos"], d["vel"], d["pref_vel"],
                              goals=d["goals"], n_steps=k)
    step(5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    return {"hetero_crossing_262k": {"value": w.n * steps / dt, "ms_per_step": 1e3 * dt / steps,
                                     "agents": w.n, "steps": steps}}


def spawn_forms(steps: int, launch):
    """Spawning and removal (section 4) at the 1M-agent density: the dense
    uniform square with each agent entering at a uniform step in [0, 200),
    a goal 2-10 m away and removal on arrival; timed from step 100 (about half
    present, arrivals under way), graph replays."""
    import numpy as np
    import torch
    from paper_1908_10107_amd import orca, scenes
    w = scenes.dense_uniform()
    rng = np.random.default_rng(scenes.BASE_SEED + 9)
    ang = rng.uniform(0.0, 2.0 * np.pi, w.n)
    dist = rng.uniform(2.0, 10.0, w.n)
    w.goals = np.ascontiguousarray(
        (w.pos + dist * np.stack([np.cos(ang), np.sin(ang)])).astype(np.float32))
    w.spawn_step = rng.integers(0, 200, w.n).astype(np.int32)
    d = orca.to_device(w)
    state = torch.zeros(w.n, dtype=torch.uint8, device="cuda")
    ctx = orca.Context(max_agents=w.n, max_scenes=1, k_max=w.params[0].max_neighbors)
    apply_launch(ctx, launch)
    ctx.set_lifecycle(d["spawn_step"], state, 0)
    step = lambda k: ctx.step_graph(w.offsets, w.params, d["pos"], d["vel"], d["pref_vel"],
                                    goals=d["goals"], n_steps=k)
    step(100)
    _, present0, removed0 = ctx.population()
    t0 = time.perf_counter()
    step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    t_end, present1, removed1 = ctx.population()
    ctx.close()
    return {"spawn_removal_1M": {"value": w.n * steps / dt, "ms_per_step": 1e3 * dt / steps,
                                 "agents": w.n, "steps": steps, "first_step": 100,
                                 "present_at_start": present0, "present_at_end": present1,
                                 "removed_in_timed_steps": removed1 - removed0}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="dense_uniform")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="the CPU reference steps the workload until this much time has passed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="plain,batched,adjoint,hetero,spawn,full",
                    help="comma list: plain (always), batched (512 scenes, graph replay vs "
                         "per-scene plain steps), adjoint (forward + adjoint), hetero "
                         "(people of different sizes and speeds), spawn (spawning and "
                         "removal), full (each workload over its whole length from t = 0)")
    ap.add_argument("--batched-steps", type=int, default=20)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--launch", default=None,
                    help="KNN_BLOCK,FALLBACK_WAVES_PER_CU[,AGENTS_PER_LANE,VELOCITY_WAVES_PER_CU"
                         "[,FALLBACK_WORK_UNITS]]: fixed launch shapes instead of autotuning "
                         "(agents per lane 0: split neighbour and LP kernels)")
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
    if args.launch:
        tuned = tuple(int(x) for x in args.launch.split(","))
        apply_launch(ctx, tuned)
    elif not args.no_autotune:
        ctx.build_grid(w.offsets, w.params, st["pos"])
        tuned = ctx.autotune(st["pos"], st["vel"], st["pref"], goals=base["goals"], reps=5)
    if args.warmup:
        step(args.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # per-stage HIP events recorded on the library's stream inside the timed
    # steps themselves (no waiting; read after the timed region)
    ctx.profile(2)
    t0 = time.perf_counter()
    e0.record()
    step(args.steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    ms_per_step = 1e3 * wall / args.steps
    value = w.n * args.steps / wall
    ms, passes, fb = ctx.profile_read()
    ctx.profile(False)
    print("# timed %d steps: %.3f s wall, %.3f s on the stream" % (args.steps, wall,
                                                                  gpu_ms / 1e3),
          file=sys.stderr, flush=True)
    avg = [m / max(passes, 1) for m in ms]
    fb_avg = fb / max(passes, 1)
    dom = int(np.argmax(avg))
    # cells of the grid at the end of the timed steps (the 12 B/cell term is small)
    state_now = dataclasses.replace(w, pos=st["pos"].cpu().numpy())
    evolved = (st["pos"].cpu().numpy(), st["vel"].cpu().numpy(), st["pref"].cpu().numpy())
    cells, cells_per_nd = grid_cells(state_now)
    stages = {orca.STAGE_NAMES[i]: round(avg[i], 4) for i in range(orca.PROF_STAGES)}
    bound, achieved, peak, unit = stage_roofline(dom, avg[dom], w.n, kmax, cells, fb_avg)
    others = {}
    for i in range(orca.PROF_STAGES):
        b_, a_, p_, u_ = stage_roofline(i, avg[i], w.n, kmax, cells, fb_avg)
        others[orca.STAGE_NAMES[i]] = {"bound": b_, "achieved": round(a_, 4), "unit": u_,
                                       "frac": round(a_ / p_, 6)}
    kdisp = 10 if kmax <= 10 else (16 if kmax <= 16 else 32)
    apl = tuned[2] if tuned is not None and len(tuned) > 2 else 0
    wu = tuned[4] if tuned is not None and len(tuned) > 4 else 0
    kname = ("k_key", "k_knn<%d>" % kdisp,
             "k_velocity<%d,%d>" % (kdisp, apl) if apl else "k_lp<%d,0>" % kdisp,
             "k_fallback<%d,0,%s>" % (kdisp, "true" if wu else "false"))[dom]
    traffic = profiled_traffic(kname) if args.workload == "dense_uniform" else None
    # the whole step against HBM: 144 B per agent + 12 B per cell, each array
    # touched once (state, sort, neighbour state, outputs, goals)
    step_bytes = 144.0 * w.n + 12.0 * cells
    step_gbs = step_bytes / (ms_per_step * 1e-3) / 1e9
    roofline = dict(bound=bound, achieved=round(achieved, 4), peak=peak, unit=unit,
                    frac=round(achieved / peak, 6), traffic=traffic, traffic_unit="B/launch",
                    kernel=kname,
                    step_hbm={"bytes_per_step": step_bytes, "cells": cells,
                              "achieved": round(step_gbs, 2), "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": round(step_gbs / HBM_PEAK_GBS, 6)},
                    lane_use=profiled_lane_use(),
                    stage_ms=stages, stages=others,
                    fallback_agents_per_step=round(fb_avg, 1))

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
    if "adjoint" in args.forms.split(","):
        forms.update(adjoint_forms())
    if "hetero" in args.forms.split(","):
        forms.update(hetero_forms(50, tuned if args.launch else None))
    if "spawn" in args.forms.split(","):
        forms.update(spawn_forms(100, tuned if args.launch else None))
    if "full" in args.forms.split(","):
        forms.update(full_length_forms(tuned))

    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = src * 1.0
        torch.cuda.synchronize()
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, args.cpu_seconds, evolved)

    line = {
        "metric": METRIC, "value": value, "unit": "agent-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "agents": w.n, "scenes": w.n_scenes,
                   "max_neighbors": kmax,
                   "neighbor_dist": w.params[0].neighbor_dist,
                   "cell": "neighbor_dist * (1 + 2^-10) / c, c = 2, 3 or 4 per scene from its "
                           "density and K (same neighbours as cells of neighbor_dist); scenes "
                           "per c: " + ", ".join(f"c = {k}: {v}" for k, v in sorted(cells_per_nd.items())),
                   "state": "f32", "lp": "f64", "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "autotune": None if tuned is None else dict(zip(
            ("knn_block", "fallback_waves_per_cu", "agents_per_lane", "velocity_waves_per_cu",
             "fallback_work_units"),
            tuned)),
        "forms": forms,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
