"""Batched form on the GPU: many scenes in one launch sequence, replayed from a
captured HIP graph, against the plain per-scene forward on the same GPU.

  * graph replays equal eager steps bit for bit, replay after replay, with
    eager work and synchronisation between the replays;
  * one launch over many scenes equals stepping each scene alone (the scenes
    never see each other), bit for bit;
  * the autotuner's launch shapes leave every result unchanged.
"""
import sys

import numpy as np
import pytest

from paper_1908_10107_amd import scenes

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_graph_replay_equals_eager():
    torch = _torch()
    from paper_1908_10107_amd import orca
    say("case graph replay vs eager")
    w = scenes.batched(n_scenes=40, n_min=64, n_max=2000, seed=11)
    kmax = max(p.max_neighbors for p in w.params)
    a = orca.to_device(w)
    b = {k: (None if v is None else v.clone()) for k, v in a.items()}
    ca = orca.Context(max_agents=w.n, max_scenes=w.n_scenes, k_max=kmax)
    cb = orca.Context(max_agents=w.n, max_scenes=w.n_scenes, k_max=kmax)
    side = torch.zeros(1 << 20, device="cuda")
    for t in range(6):
        ca.step(w.offsets, w.params, a["pos"], a["vel"], a["pref_vel"], goals=a["goals"])
        cb.step_graph(w.offsets, w.params, b["pos"], b["vel"], b["pref_vel"], goals=b["goals"])
        side.add_(1.0)           # unrelated eager work between replays
        torch.cuda.synchronize()
        for k in ("pos", "vel", "pref_vel"):
            assert torch.equal(a[k], b[k]), (t, k)
    ca.close()
    cb.close()


def test_graph_blocks_equal_eager():
    """Graph replays of 10-step blocks (resident between their steps) plus
    single-step replays for the rest equal one eager multi-step call and
    one-step calls bit for bit, replay after replay, also when the captured
    graphs are reused by a later call and after the pointers change."""
    torch = _torch()
    from paper_1908_10107_amd import orca
    say("case graph blocks vs eager")
    w = scenes.batched(n_scenes=30, n_min=64, n_max=3000, seed=13)
    kmax = max(p.max_neighbors for p in w.params)
    a = orca.to_device(w)
    b = {k: (None if v is None else v.clone()) for k, v in a.items()}
    c = {k: (None if v is None else v.clone()) for k, v in a.items()}
    ca = orca.Context(max_agents=w.n, max_scenes=w.n_scenes, k_max=kmax)
    cb = orca.Context(max_agents=w.n, max_scenes=w.n_scenes, k_max=kmax)
    side = torch.zeros(1 << 20, device="cuda")
    done = 0
    for n in (23, 10, 7, 12):
        ca.step(w.offsets, w.params, a["pos"], a["vel"], a["pref_vel"], goals=a["goals"],
                n_steps=n)
        cb.step_graph(w.offsets, w.params, b["pos"], b["vel"], b["pref_vel"], goals=b["goals"],
                      n_steps=n)
        side.add_(1.0)           # unrelated eager work between replays
        torch.cuda.synchronize()
        done += n
        for k in ("pos", "vel", "pref_vel"):
            assert torch.equal(a[k], b[k]), (done, k)
    # new pointers: the graphs are captured again
    for k in ("pos", "vel", "pref_vel"):
        c[k].copy_(b[k])
    cb.step_graph(w.offsets, w.params, c["pos"], c["vel"], c["pref_vel"], goals=c["goals"],
                  n_steps=15)
    for _ in range(15):
        ca.step(w.offsets, w.params, a["pos"], a["vel"], a["pref_vel"], goals=a["goals"])
    torch.cuda.synchronize()
    for k in ("pos", "vel", "pref_vel"):
        assert torch.equal(a[k], c[k]), k
    ca.close()
    cb.close()


def test_batched_equals_per_scene():
    torch = _torch()
    from paper_1908_10107_amd import orca
    say("case batched vs per-scene")
    w = scenes.batched(n_scenes=48, n_min=64, n_max=3000, seed=12)
    kmax = max(p.max_neighbors for p in w.params)
    big = orca.to_device(w)
    cb = orca.Context(max_agents=w.n, max_scenes=w.n_scenes, k_max=kmax)
    cb.step_graph(w.offsets, w.params, big["pos"], big["vel"], big["pref_vel"],
                  goals=big["goals"], n_steps=3)
    torch.cuda.synchronize()
    nmax = int(np.diff(w.offsets).max())
    cs = orca.Context(max_agents=nmax, max_scenes=1, k_max=kmax)
    worst = 0.0
    for s in range(w.n_scenes):
        one = w.subset_scenes([s])
        d = orca.to_device(one)
        cs.step(one.offsets, one.params, d["pos"], d["vel"], d["pref_vel"], goals=d["goals"],
                n_steps=3)
        torch.cuda.synchronize()
        lo, hi = int(w.offsets[s]), int(w.offsets[s + 1])
        for k in ("pos", "vel"):
            diff = (d[k] - big[k][:, lo:hi]).abs().max().item() if hi > lo else 0.0
            worst = max(worst, diff)
            assert torch.equal(d[k], big[k][:, lo:hi]), (s, k, diff)
    say("batched vs per-scene: max difference %g" % worst)
    cb.close()
    cs.close()


def test_autotune_keeps_results():
    torch = _torch()
    from paper_1908_10107_amd import orca
    say("case autotune")
    w = scenes.dense_uniform(n=50000)
    d = orca.to_device(w)
    ctx = orca.Context(max_agents=w.n, max_scenes=1, k_max=16)
    ctx.build_grid(w.offsets, w.params, d["pos"])
    before = ctx.compute_velocities(d["pos"], d["vel"], goals=d["goals"]).clone()
    choice = ctx.autotune(d["pos"], d["vel"], goals=d["goals"], reps=2)
    say("autotune choice", choice)
    assert choice[0] in (64, 128, 256, 512) and choice[1] in (4, 8, 16, 32)
    after = ctx.compute_velocities(d["pos"], d["vel"], goals=d["goals"])
    torch.cuda.synchronize()
    assert torch.equal(before, after)
    for kb, fw in ((64, 1), (128, 8), (256, 64), (512, 32)):
        ctx.set_launch(kb, fw)
        again = ctx.compute_velocities(d["pos"], d["vel"], goals=d["goals"])
        torch.cuda.synchronize()
        assert torch.equal(before, again), (kb, fw)
    with pytest.raises(RuntimeError):
        ctx.set_launch(96, 8)
    with pytest.raises(RuntimeError):
        ctx.set_launch(256, 0)
    ctx.close()


def test_profile_modes_agree():
    """The two timing modes of orca_profile over the same steps: mode 2 (events
    recorded without waiting, fallback agents counted on the device) gives the
    fallback count that mode 1 (every pass waits, counts read on the host)
    gives, and stage times that are positive and sum to at most the wall time
    of the steps."""
    torch = _torch()
    import time
    from paper_1908_10107_amd import orca
    say("case profile modes")
    w = scenes.dense_uniform(n=60000, seed=scenes.BASE_SEED + 50)
    res = []
    for mode in (1, 2):
        d = orca.to_device(w)
        with orca.Context(max_agents=w.n, max_scenes=1, k_max=16) as ctx:
            ctx.step(w.offsets, w.params, d["pos"], d["vel"], d["pref_vel"], goals=d["goals"],
                     n_steps=3)
            torch.cuda.synchronize()
            ctx.profile(mode)
            t0 = time.perf_counter()
            ctx.step(w.offsets, w.params, d["pos"], d["vel"], d["pref_vel"], goals=d["goals"],
                     n_steps=12)
            ms, passes, fb = ctx.profile_read()
            torch.cuda.synchronize()
            wall = 1e3 * (time.perf_counter() - t0)
            ctx.profile(0)
        say("  mode %d: stages %s ms, %d passes, %d fallback agents, %.2f ms wall"
            % (mode, [round(x, 3) for x in ms], passes, fb, wall))
        assert passes == 12
        assert all(x > 0 for x in ms) and sum(ms) <= wall
        res.append(fb)
    assert res[0] == res[1] and res[0] > 0
