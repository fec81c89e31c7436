"""Kernel variants against the default kernels and the oracle, through the C ABI.

- The fused persistent velocity kernel (neighbour search + half-planes + 2D LP
  in one kernel over per-XCD tile queues) runs the same arithmetic as the
  split kernels: new velocities, neighbour lists and fallback labels must be
  equal bit for bit for every agents-per-lane choice, and its steps must give
  the same trajectories.
- The fallback with work units folds a violated line's earlier rows in shares
  on several lanes and combines the partial intervals in row order.  With
  exact comparisons that is the one-lane result; the fractions are compared
  after rounding, so a near-tie between two bounds may resolve the other way:
  its velocities are held to the oracle (1e-4 m/s) and to the default
  fallback within two float32 ulps, with at most one agent in a thousand
  differing at all.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1908_10107_amd import scenes

from test_gpu_parity import compare, props

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def velocity_pass(w, apl, waves=12, use_goals=True, wu=0):
    torch = _torch()
    from paper_1908_10107_amd import orca
    kmax = max(1, max(p.max_neighbors for p in w.params))
    krow = max(1, max(p.max_neighbors for p in w.params))
    with orca.Context(max_agents=max(w.n, 1), max_scenes=w.n_scenes, k_max=kmax) as ctx:
        d = orca.to_device(w)
        ctx.set_agents(d["radius"], d["max_speed"], d["pref_speed"])
        ctx.set_kernels(apl, waves, wu)
        if wu:
            ctx.set_launch(256, 6)
        nbr = torch.full((max(w.n, 1), krow), -7, dtype=torch.int32, device="cuda")
        st = torch.full((max(w.n, 1),), 9, dtype=torch.uint8, device="cuda")
        ctx.build_grid(w.offsets, w.params, d["pos"])
        nv = ctx.compute_velocities(d["pos"], d["vel"], pref_vel=d["pref_vel"],
                                    goals=d["goals"] if use_goals else None, nbr_out=nbr,
                                    lp_status=st)
        torch.cuda.synchronize()
        return dict(new_vel=nv.cpu().numpy().T.copy(), nbr=nbr.cpu().numpy()[:, :krow].copy(),
                    status=st.cpu().numpy().copy())


def same(a, b, label):
    for key in ("new_vel", "nbr", "status"):
        diff = int(np.count_nonzero(a[key] != b[key]))
        assert diff == 0, "%s: %s differs in %d entries" % (label, key, diff)


CASES = [
    # name, workload, goals
    ("one agent", lambda: scenes.tiny_random(1, 1.0, seed=200), False),
    ("37 agents", lambda: scenes.tiny_random(37, 6.0, seed=201), False),
    ("3000 K=16", lambda: scenes.tiny_random(3000, 30.0, seed=202, max_neighbors=16), False),
    ("1500 K=0", lambda: scenes.tiny_random(1500, 25.0, seed=203, max_neighbors=0), False),
    ("1500 K=1", lambda: scenes.tiny_random(1500, 25.0, seed=204, max_neighbors=1), False),
    ("700 K=32", lambda: scenes.tiny_random(700, 12.0, seed=205, max_neighbors=32), False),
    ("dense 20000", lambda: scenes.dense_uniform(n=20000, seed=206), True),
    ("uniform_rsa", lambda: scenes.uniform_rsa(), True),
    ("40 scenes", lambda: scenes.batched().subset_scenes(list(range(40))), True),
    ("hetero crossing", lambda: scenes.crossing_hetero(n=2500), True),
]


@pytest.mark.parametrize("name,make,goals", CASES, ids=[c[0] for c in CASES])
def test_fused_equals_split(name, make, goals):
    say("case fused vs split: %s" % name)
    w = make()
    ref = velocity_pass(w, 0, use_goals=goals)
    for apl in (1, 2, 4):
        got = velocity_pass(w, apl, waves=8 if apl == 2 else 12, use_goals=goals)
        same(ref, got, "%s apl=%d" % (name, apl))
    say("%s: %d agents, fused (1, 2, 4 agents per lane) equal to split" % (name, w.n))


def test_fused_against_oracle():
    """The fused kernel's own output held to the oracle (lists bit for bit,
    velocities within 1e-4 m/s), on a dense state with K = 16 and on mixed
    scenes."""
    for label, w, goals in (("dense 12000", scenes.dense_uniform(n=12000, seed=207), True),
                            ("25 scenes", scenes.batched().subset_scenes(list(range(25, 50))),
                             True)):
        say("case fused vs oracle: %s" % label)
        g = velocity_pass(w, 1, use_goals=goals)
        g["new_vel"] = g["new_vel"].astype(np.float64)
        o = oracle.velocities(w.pos, w.vel, w.pref_vel, w.offsets, w.params,
                              goals=w.goals if goals else None, neighbor_mode=1, **props(w))
        compare(w, g, o, label="fused " + label)


def _steps(w, apl, n_steps, graph=False, waves=12):
    torch = _torch()
    from paper_1908_10107_amd import orca
    kmax = max(p.max_neighbors for p in w.params)
    d = orca.to_device(w)
    with orca.Context(max_agents=w.n, max_scenes=w.n_scenes, k_max=kmax) as ctx:
        ctx.set_kernels(apl, waves)
        fn = ctx.step_graph if graph else ctx.step
        fn(w.offsets, w.params, d["pos"], d["vel"], d["pref_vel"], goals=d["goals"],
           n_steps=n_steps)
        torch.cuda.synchronize()
    return {k: d[k].cpu().numpy() for k in ("pos", "vel", "pref_vel")}


@pytest.mark.parametrize("make,n_steps", [
    (lambda: scenes.dense_uniform(n=30000, seed=208), 12),
    (lambda: scenes.ring(n=4096, radius_m=75.0), 12),
], ids=["dense30000", "ring4096"])
def test_fused_steps_equal_split_steps(make, n_steps):
    w = make()
    say("case fused steps: %d agents, %d steps" % (w.n, n_steps))
    a = _steps(w, 0, n_steps)
    for apl in (1, 4):
        b = _steps(w, apl, n_steps)
        for k in a:
            assert np.array_equal(a[k], b[k]), (apl, k)


def test_fused_graph_replays_equal_eager():
    w = scenes.batched().subset_scenes(list(range(60)))
    say("case fused graph: %d agents, %d scenes" % (w.n, w.n_scenes))
    a = _steps(w, 2, 6)
    b = _steps(w, 2, 6, graph=True)
    c = _steps(w, 0, 6)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k], c[k]), k


@pytest.mark.parametrize("make", [scenes.dense_uniform, scenes.batched],
                         ids=["dense1M", "batched512"])
def test_fused_full_size_steps(make):
    """Full-size workloads: three fused steps (the autotuner's candidates at
    their extremes) equal three split steps bit for bit."""
    w = make()
    say("case fused full size: %d agents, %d scenes" % (w.n, w.n_scenes))
    a = _steps(w, 0, 3)
    for apl, waves in ((1, 12), (4, 8)):
        b = _steps(w, apl, 3, waves=waves)
        for k in a:
            assert np.array_equal(a[k], b[k]), (apl, k)


def test_autotune_choice_is_valid_and_changes_nothing():
    torch = _torch()
    from paper_1908_10107_amd import orca
    w = scenes.dense_uniform(n=60000, seed=209)
    d = orca.to_device(w)
    with orca.Context(max_agents=w.n, max_scenes=1, k_max=16) as ctx:
        ctx.build_grid(w.offsets, w.params, d["pos"])
        choice = ctx.autotune(d["pos"], d["vel"], d["pref_vel"], goals=d["goals"], reps=2)
        say("autotune choice: %s" % (choice,))
        assert choice[0] in (64, 128, 256, 512) and choice[1] in (4, 6, 8, 16, 32)
        assert choice[2] in (0, 1, 2, 4) and choice[3] in (8, 12) and choice[4] in (0, 1)
        ctx.step(w.offsets, w.params, d["pos"], d["vel"], d["pref_vel"], goals=d["goals"],
                 n_steps=4)
        torch.cuda.synchronize()
        got = {k: d[k].cpu().numpy() for k in ("pos", "vel", "pref_vel")}
    want = _steps(w, 0, 4)
    for k in want:
        assert np.array_equal(want[k], got[k]), k


def test_set_kernels_rejects_bad_values():
    _torch()
    from paper_1908_10107_amd import orca
    with orca.Context(max_agents=8, max_scenes=1, k_max=4) as ctx:
        for apl, waves, wu in ((3, 12, 0), (-1, 12, 0), (1, 0, 0), (1, 33, 0), (0, 12, 2)):
            with pytest.raises(orca.OrcaError) as e:
                ctx.set_kernels(apl, waves, wu)
            assert e.value.code == orca.EINVAL


WU_CASES = [
    ("dense 20000 K=16", lambda: scenes.dense_uniform(n=20000, seed=210), True),
    ("dense 3000 K=10", lambda: scenes.tiny_random(3000, 38.0, seed=211, max_neighbors=10),
     False),
    ("ring 4096", lambda: scenes.ring(n=4096, radius_m=75.0), True),
    ("hetero crossing", lambda: scenes.crossing_hetero(n=2500), True),
    ("40 scenes", lambda: scenes.batched().subset_scenes(list(range(40))), True),
    ("one agent", lambda: scenes.tiny_random(1, 1.0, seed=212), False),
]


@pytest.mark.parametrize("name,make,goals", WU_CASES, ids=[c[0] for c in WU_CASES])
def test_fallback_work_units(name, make, goals):
    say("case fallback work units: %s" % name)
    w = make()
    ref = velocity_pass(w, 0, use_goals=goals)
    got = velocity_pass(w, 0, use_goals=goals, wu=1)
    assert np.array_equal(ref["nbr"], got["nbr"]) and np.array_equal(ref["status"], got["status"])
    dv = np.abs(ref["new_vel"].astype(np.float64) - got["new_vel"].astype(np.float64)).max(axis=1)
    ndiff = int(np.count_nonzero(dv))
    say("%s: %d agents, %d fallback, %d differ from the default fallback (max %.3g m/s)"
        % (name, w.n, int((ref["status"] == 1).sum()), ndiff, dv.max() if w.n else 0.0))
    assert dv.max() <= 2.4e-7 and ndiff <= max(2, w.n // 1000)
    got["new_vel"] = got["new_vel"].astype(np.float64)
    o = oracle.velocities(w.pos, w.vel, w.pref_vel, w.offsets, w.params,
                          goals=w.goals if goals else None, neighbor_mode=1, **props(w))
    compare(w, got, o, label="work units " + name)


def test_fallback_work_units_full_size_step():
    """One step of the 1M-agent square (about 57% of the agents take the
    fallback) and of the 512 scenes with work units, against the default."""
    for make in (scenes.dense_uniform, scenes.batched):
        w = make()
        say("case work units full size: %d agents" % w.n)
        a = velocity_pass(w, 0)
        b = velocity_pass(w, 0, wu=1)
        assert np.array_equal(a["status"], b["status"])
        dv = np.abs(a["new_vel"].astype(np.float64) - b["new_vel"].astype(np.float64)).max(axis=1)
        ndiff = int(np.count_nonzero(dv))
        say("%d agents, %d fallback, %d differ (max %.3g m/s)"
            % (w.n, int((a["status"] == 1).sum()), ndiff, dv.max()))
        assert dv.max() <= 2.4e-7 and ndiff <= w.n // 1000


RESIDENT_CASES = [
    ("uniform_rsa goals", lambda: scenes.uniform_rsa(), True),
    ("3000 no goals K=16", lambda: scenes.tiny_random(3000, 30.0, seed=213, max_neighbors=16),
     False),
    ("dense 20000", lambda: scenes.dense_uniform(n=20000, seed=214), True),
    ("40 scenes", lambda: scenes.batched().subset_scenes(list(range(40))), True),
    ("hetero crossing", lambda: scenes.crossing_hetero(n=2500), True),
    ("ring 4096", lambda: scenes.ring(n=4096, radius_m=75.0), True),
]


@pytest.mark.parametrize("name,make,goals", RESIDENT_CASES, ids=[c[0] for c in RESIDENT_CASES])
def test_resident_steps_equal_single_steps(name, make, goals):
    """The inner steps of one multi-step call keep the state in cell order (only
    the first reads and the last writes the caller's arrays): seven steps in
    one call equal seven one-step calls bit for bit, with the split and the
    fused velocity kernels, with goals or fixed preferred velocities, with
    several scenes and with per-agent properties."""
    torch = _torch()
    from paper_1908_10107_amd import orca
    w = make()
    if not goals:
        w.goals = None
    say("case resident steps: %s, %d agents, %d scenes" % (name, w.n, w.n_scenes))
    kmax = max(1, max(p.max_neighbors for p in w.params))
    out = []
    for apl, calls in ((0, [7]), (0, [1] * 7), (2, [7]), (0, [3, 1, 3])):
        d = orca.to_device(w)
        with orca.Context(max_agents=w.n, max_scenes=w.n_scenes, k_max=kmax) as ctx:
            ctx.set_agents(d["radius"], d["max_speed"], d["pref_speed"])
            ctx.set_kernels(apl, 12)
            for c in calls:
                ctx.step(w.offsets, w.params, d["pos"], d["vel"], d["pref_vel"],
                         goals=d["goals"], n_steps=c)
            torch.cuda.synchronize()
        out.append({k: d[k].cpu().numpy() for k in ("pos", "vel", "pref_vel")})
    for r in out[1:]:
        for k in out[0]:
            assert np.array_equal(out[0][k], r[k]), k
