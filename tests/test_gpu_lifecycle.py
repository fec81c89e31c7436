"""Spawning and removal on the GPU against the CPU reference (section 4: the
2-way and 8-way crossings whose people enter over time and leave at their
goal).

From each checked state (the GPU's own, copied back before the step) one
reference step with the same spawn steps and removal state is compared with
the GPU's step: present agents' velocities within 1e-4 m/s and positions
within that times dt plus one float32 rounding; absent agents untouched, bit
for bit; the removal state equal, except for an agent whose distance to its
goal after the step is within 1e-5 m of its radius (there the velocity
tolerance can move it either way); and the device counters (step index,
agents present, agents removed) equal to what the reference's arrays give.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1908_10107_amd import scenes

from crowd_measures import lane_order, turning_speed

pytestmark = pytest.mark.gpu

TOL_V = 1e-4
TOL_ARRIVE = 1e-5


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def props(w):
    return dict(radius=w.radius, max_speed=w.max_speed, pref_speed=w.pref_speed)


def small_crossing(ways, hetero, n=None, seed=None):
    # a few hundred people spawning at about 3 a second per region, 18-24 m
    # from their goals: arrivals start within a few hundred steps
    n = n or (120 if ways == 2 else 480)
    kw = dict(ways=ways, n=n, spawn_steps=200, ring=9.0 if ways == 2 else 12.0, region=6.0,
              hetero=hetero)
    if seed is not None:
        kw["seed"] = seed
    return scenes.crossing_spawn(**kw)


def setup(w, torch, t0=0):
    from paper_1908_10107_amd import orca
    kmax = max(p.max_neighbors for p in w.params)
    ctx = orca.Context(max_agents=w.n, max_scenes=w.n_scenes, k_max=kmax)
    d = orca.to_device(w)
    ctx.set_agents(d["radius"], d["max_speed"], d["pref_speed"])
    d["state"] = torch.zeros(w.n, dtype=torch.uint8, device="cuda")
    ctx.set_lifecycle(d["spawn_step"], d["state"], t0)
    return ctx, d


def radii(w):
    return w.radius.astype(np.float64) if w.radius is not None else np.full(w.n, w.params[0].radius)


@pytest.mark.parametrize("ways,hetero", [(2, False), (8, False), (8, True)])
def test_life_steps_match_reference(ways, hetero):
    torch = _torch()
    say("case life steps ways=%d hetero=%s" % (ways, hetero))
    w = small_crossing(ways, hetero)
    ctx, d = setup(w, torch)
    dt = float(np.float32(w.params[0].dt))
    r = radii(w)
    removed = 0
    arrivals = 0
    for t in range(600):
        check = t % 3 == 0 or t >= 250
        if check:
            pos0 = d["pos"].cpu().numpy()
            vel0 = d["vel"].cpu().numpy()
            pref0 = d["pref_vel"].cpu().numpy()
            state0 = d["state"].cpu().numpy()
        ctx.step(w.offsets, w.params, d["pos"], d["vel"], d["pref_vel"], goals=d["goals"])
        if not check:
            continue
        torch.cuda.synchronize()
        p1, v1 = d["pos"].cpu().numpy(), d["vel"].cpu().numpy()
        s1 = d["state"].cpu().numpy()
        po, vo, _, so, st = oracle.life_step(pos0, vel0, pref0, w.offsets, w.params, w.goals,
                                             w.spawn_step, state0, t, n_steps=1, **props(w))
        present = (w.spawn_step <= t) & (state0 == 0)
        absent = ~present
        assert np.array_equal(p1[:, absent], pos0[:, absent]), t
        assert np.array_equal(v1[:, absent], vel0[:, absent]), t
        assert np.all(st[absent] == 2)
        err = np.abs(v1[:, present].astype(np.float64) - vo[:, present]).max() if present.any() \
            else 0.0
        assert err < TOL_V, (t, err)
        want_p = pos0[:, present].astype(np.float64) + dt * vo[:, present].astype(np.float64)
        perr = np.abs(p1[:, present] - want_p) - (dt * TOL_V + np.spacing(
            np.abs(want_p).astype(np.float32)))
        assert perr.size == 0 or perr.max() <= 0, t
        # removal state: equal except within TOL_ARRIVE of the radius
        dist = np.hypot(*(w.goals.astype(np.float64) - po.astype(np.float64)))
        near = np.abs(dist - r) < TOL_ARRIVE
        diff = (s1 != so) & ~near
        assert not diff.any(), (t, np.flatnonzero(diff)[:10])
        arrivals += int(((s1 == 1) & (state0 == 0)).sum())
        removed = int((s1 == 1).sum())
        step, n_present, n_removed = ctx.population()
        assert step == t + 1
        assert n_present == int(present.sum())
        assert n_removed == removed, (t, n_removed, removed)
        if t % 30 == 0:
            say("  t=%d present %d removed %d max |dv| %.3g" % (t, n_present, removed, err))
        # keep the GPU state in step with the reference where an arrival flipped
        if (s1 != so).any():
            d["state"].copy_(torch.from_numpy(so).cuda())
            ctx.set_lifecycle(d["spawn_step"], d["state"], t + 1)
    assert arrivals >= 10, arrivals
    ctx.close()


def test_life_velocity_call_reports_absent_agents():
    torch = _torch()
    say("case life velocity call")
    w = small_crossing(8, True, n=960)
    rng = np.random.default_rng(3)
    state = (rng.random(w.n) < 0.2).astype(np.uint8)
    t0 = 60
    ctx, d = setup(w, torch, t0=t0)
    d["state"].copy_(torch.from_numpy(state).cuda())
    kmax = max(p.max_neighbors for p in w.params)
    nbr = torch.full((w.n, kmax), -7, dtype=torch.int32, device="cuda")
    st = torch.full((w.n,), 9, dtype=torch.uint8, device="cuda")
    nv = torch.full_like(d["pos"], 5.0)
    ctx.build_grid(w.offsets, w.params, d["pos"])
    ctx.compute_velocities(d["pos"], d["vel"], pref_vel=d["pref_vel"], goals=d["goals"],
                           new_vel=nv, nbr_out=nbr, lp_status=st)
    torch.cuda.synchronize()
    present = (w.spawn_step <= t0) & (state == 0)
    o = oracle.velocities(w.pos, w.vel, w.pref_vel, w.offsets, w.params, goals=w.goals,
                          present=present.astype(np.uint8), **props(w))
    g_st = st.cpu().numpy()
    assert np.array_equal(g_st == 2, ~present)
    assert np.array_equal(nbr.cpu().numpy().astype(np.int64), o["nbr"][:, :kmax])
    g_nv = nv.cpu().numpy().T.astype(np.float64)
    assert np.all(g_nv[~present] == 0)
    assert np.abs(g_nv - o["new_vel"]).max() < TOL_V
    step, n_present, removed = ctx.population()
    assert (step, n_present, removed) == (t0, int(present.sum()), int(state.sum()))
    ctx.close()


def test_life_graph_replay_equals_eager_steps():
    torch = _torch()
    say("case life graph vs eager")
    w = small_crossing(2, False, n=200, seed=scenes.BASE_SEED + 11)
    a, da = setup(w, torch)
    b, db = setup(w, torch)
    for t in range(0, 500, 25):
        a.step(w.offsets, w.params, da["pos"], da["vel"], da["pref_vel"], goals=da["goals"],
               n_steps=25)
        b.step_graph(w.offsets, w.params, db["pos"], db["vel"], db["pref_vel"],
                     goals=db["goals"], n_steps=25)
        torch.cuda.synchronize()
        for k in ("pos", "vel", "pref_vel", "state"):
            assert torch.equal(da[k], db[k]), (t, k)
        assert a.population() == b.population()
    step, n_present, removed = b.population()
    assert step == 500 and removed == int(db["state"].sum().item()) and removed > 0
    a.close()
    b.close()


@pytest.mark.parametrize("ways", [2, 8])
def test_full_crossing_runs_until_everyone_arrives(ways):
    torch = _torch()
    say("case life full crossing ways=%d" % ways)
    w = scenes.crossing_spawn(ways=ways)
    ctx, d = setup(w, torch)
    r = radii(w)
    steps = 0
    while steps < 12000:
        ctx.step_graph(w.offsets, w.params, d["pos"], d["vel"], d["pref_vel"], goals=d["goals"],
                       n_steps=100)
        steps += 100
        step, n_present, removed = ctx.population()
        assert step == steps
        if removed == w.n:
            break
    say("  ways=%d: everyone removed after %d steps" % (ways, steps))
    state = d["state"].cpu().numpy()
    assert removed == w.n and np.all(state == 1)
    pos = d["pos"].cpu().numpy().astype(np.float64)
    dist = np.hypot(*(w.goals.astype(np.float64) - pos))
    assert np.all(dist <= r + 1e-12)
    # a last pass sees nobody
    st = torch.full((w.n,), 9, dtype=torch.uint8, device="cuda")
    ctx.build_grid(w.offsets, w.params, d["pos"])
    ctx.compute_velocities(d["pos"], d["vel"], goals=d["goals"], lp_status=st)
    assert int((st == 2).sum().item()) == w.n
    assert ctx.population()[1] == 0
    ctx.close()


def test_life_argument_errors():
    torch = _torch()
    from paper_1908_10107_amd import orca
    w = small_crossing(2, False, n=100)
    ctx, d = setup(w, torch)
    assert ctx.population()[1] == -1          # nothing binned yet
    with pytest.raises(orca.OrcaError):
        ctx.step(w.offsets, w.params, d["pos"], d["vel"], d["pref_vel"])   # no goals
    with pytest.raises(orca.OrcaError):
        ctx.step(w.offsets, w.params, d["pos"], d["vel"], d["pref_vel"], goals=d["goals"],
                 save_tape=True)
    rc = ctx.lib.orca_set_lifecycle(ctx.h, None, ctypes_ptr(d["state"]), 0)
    assert rc == orca.EINVAL
    # off again: the plain step, bit for bit
    ctx.set_lifecycle()
    e, de = setup(w, torch)
    e.set_lifecycle()
    ctx.step(w.offsets, w.params, d["pos"], d["vel"], d["pref_vel"], goals=d["goals"], n_steps=5)
    e.step(w.offsets, w.params, de["pos"], de["vel"], de["pref_vel"], goals=de["goals"],
           n_steps=5)
    torch.cuda.synchronize()
    assert torch.equal(d["pos"], de["pos"]) and torch.equal(d["vel"], de["vel"])
    assert ctx.population() == (0, w.n, 0)
    ctx.close()
    e.close()


def ctypes_ptr(t):
    import ctypes
    return ctypes.c_void_p(t.data_ptr())


def test_crossing_lanes_and_turning_on_the_gpu():
    """The crowd phenomena of section 4 in GPU runs: lanes in the 2-way
    crossing (band order above that of shuffled groups from step 1000 to
    3000) and one turning sense in the 8-way crossing while people cross in
    numbers."""
    torch = _torch()
    say("case life lanes and vortex")
    w = scenes.crossing_spawn(ways=2)
    ctx, d = setup(w, torch)
    group = (w.goals[0] < 0).astype(int)
    rng = np.random.default_rng(0)
    real, mixed = [], []
    for t in range(0, 3000, 100):
        ctx.step_graph(w.offsets, w.params, d["pos"], d["vel"], d["pref_vel"], goals=d["goals"],
                       n_steps=100)
        if t + 100 >= 1000:
            pos = d["pos"].cpu().numpy()
            present = (w.spawn_step <= t + 99) & (d["state"].cpu().numpy() == 0)
            real.append(lane_order(pos, present, group))
            mixed.append(np.mean([lane_order(pos, present, rng.permutation(group))
                                  for _ in range(4)]))
    say("  lanes: band order %.3f, shuffled %.3f" % (np.mean(real), np.mean(mixed)))
    assert np.mean(real) > np.mean(mixed) + 0.1
    ctx.close()
    w = scenes.crossing_spawn(ways=8)
    ctx, d = setup(w, torch)
    lz = []
    for t in range(0, 2000, 100):
        ctx.step_graph(w.offsets, w.params, d["pos"], d["vel"], d["pref_vel"], goals=d["goals"],
                       n_steps=100)
        present = (w.spawn_step <= t + 99) & (d["state"].cpu().numpy() == 0)
        if present.sum() >= w.n // 3:
            lz.append(turning_speed(d["pos"].cpu().numpy(), d["vel"].cpu().numpy(), present))
    say("  turning speed %.3f .. %.3f m/s over %d samples" % (min(lz), max(lz), len(lz)))
    assert len(lz) >= 8 and min(lz) > 0.25
    ctx.close()


def concat_scenes(ws):
    """Back-to-back scenes of several workloads (each one scene) as one workload."""
    pos = np.concatenate([w.pos for w in ws], axis=1)
    goals = np.concatenate([w.goals for w in ws], axis=1)
    n = pos.shape[1]
    offs = np.zeros(len(ws) + 1, np.int64)
    offs[1:] = np.cumsum([w.pos.shape[1] for w in ws])
    params = [w.params[0] for w in ws]
    out = scenes.Workload("multi", np.ascontiguousarray(pos), np.zeros((2, n), np.float32),
                          np.ascontiguousarray(goals), np.zeros((2, n), np.float32), offs,
                          params, 0)
    out.spawn_step = np.concatenate([w.spawn_step for w in ws]).astype(np.int32)
    return out


def test_life_steps_with_several_scenes():
    """Three scenes with their own parameters (one empty) share the cell of
    absent agents: every step from the GPU's state matches the reference."""
    torch = _torch()
    say("case life several scenes")
    a = small_crossing(2, False)
    b = scenes.crossing_spawn(ways=8, n=240, spawn_steps=150, ring=10.0, region=6.0,
                              neighbor_dist=4.0, max_neighbors=7, time_horizon=3.0)
    e = scenes.crossing_spawn(ways=2, n=2, spawn_steps=1)
    e.pos, e.goals, e.spawn_step = e.pos[:, :0], e.goals[:, :0], e.spawn_step[:0]
    w = concat_scenes([a, e, b])
    assert list(np.diff(w.offsets)) == [a.n, 0, b.n] and w.n == a.n + b.n
    ctx, d = setup(w, torch)
    dt = np.array([np.float32(p.dt) for p in w.params], np.float64)
    scene = np.repeat(np.arange(3), np.diff(w.offsets))
    arrivals = 0
    for t in range(400):
        check = t % 4 == 0 or t >= 250
        if check:
            pos0 = d["pos"].cpu().numpy()
            vel0 = d["vel"].cpu().numpy()
            pref0 = d["pref_vel"].cpu().numpy()
            state0 = d["state"].cpu().numpy()
        ctx.step(w.offsets, w.params, d["pos"], d["vel"], d["pref_vel"], goals=d["goals"])
        if not check:
            continue
        p1, v1 = d["pos"].cpu().numpy(), d["vel"].cpu().numpy()
        s1 = d["state"].cpu().numpy()
        po, vo, _, so, st = oracle.life_step(pos0, vel0, pref0, w.offsets, w.params, w.goals,
                                             w.spawn_step, state0, t, n_steps=1)
        present = (w.spawn_step <= t) & (state0 == 0)
        assert np.array_equal(p1[:, ~present], pos0[:, ~present]), t
        if present.any():
            err = np.abs(v1[:, present].astype(np.float64) - vo[:, present]).max()
            assert err < TOL_V, (t, err)
            want = pos0[:, present].astype(np.float64) + dt[scene[present]] * \
                vo[:, present].astype(np.float64)
            perr = np.abs(p1[:, present] - want) - (dt[scene[present]] * TOL_V + np.spacing(
                np.abs(want).astype(np.float32)))
            assert perr.max() <= 0, t
        dist = np.hypot(*(w.goals.astype(np.float64) - po.astype(np.float64)))
        near = np.abs(dist - w.params[0].radius) < TOL_ARRIVE
        assert not ((s1 != so) & ~near).any(), t
        if (s1 != so).any():
            d["state"].copy_(torch.from_numpy(so).cuda())
            ctx.set_lifecycle(d["spawn_step"], d["state"], t + 1)
        arrivals += int(((s1 == 1) & (state0 == 0)).sum())
        assert ctx.population()[1] == int(present.sum())
    say("  arrivals %d" % arrivals)
    assert arrivals >= 10
    ctx.close()
