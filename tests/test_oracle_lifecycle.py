"""Pins of the reference's spawning and removal (section 4: the 2-way and
8-way crossings, where people enter over time and leave at their goal).

  * a lone walker arrives at the step a closed form gives: it walks s dt per
    step toward the goal and is removed at the first step that ends within its
    own radius of the goal, counted from its spawn step;
  * an agent not yet spawned, or already removed, is invisible: the others'
    velocities equal those of the scene with that agent deleted, bit for bit;
  * an agent does not move before its spawn step, and a removed agent stays
    removed and does not move again;
  * the scene generator never places a new person on top of someone spawned
    in the same region who cannot yet have walked clear;
  * a small 2-way and 8-way crossing run until everyone has arrived, with no
    two present agents that both solved the 2D LP ending a step overlapped;
  * the crowd phenomena the paper reports, as measures: lanes in the 2-way
    crossing (a band order parameter above that of shuffled groups) and one
    turning sense in the 8-way crossing (a vortex about the centre).
"""
import numpy as np
import pytest

from paper_1908_10107_amd import scenes

from crowd_measures import lane_order, turning_speed


def lone(goal, radius=0.5, speed=1.0, dt=0.25, spawn=0):
    p = scenes.SceneParams(radius=radius, max_speed=1.5, neighbor_dist=5.0, time_horizon=2.0,
                           dt=dt, pref_speed=speed, max_neighbors=10)
    pos = np.zeros((2, 1), np.float32)
    goals = np.array(goal, np.float32).reshape(2, 1)
    return pos, goals, [p], np.array([0, 1], np.int64), np.array([spawn], np.int32)


@pytest.mark.parametrize("goal,spawn", [((10.1, 0.0), 0), ((6.06, 8.08), 0), ((-3.3, 6.5), 7)])
def test_lone_walker_arrives_at_closed_form_step(oracle_lib, goal, spawn):
    # |g| - r = k s dt is crossed at k = ceil((|g| - r) / (s dt)); the inputs
    # keep that ratio at least 0.1 step away from an integer
    pos, goals, params, offs, sp = lone(goal, spawn=spawn)
    ratio = (np.hypot(*goal) - 0.5) / (1.0 * 0.25)
    assert abs(ratio - round(ratio)) > 0.1
    k = int(np.ceil(ratio))
    zero = np.zeros((2, 1), np.float32)
    st = np.zeros(1, np.uint8)
    p1, v1, _, s1, _ = oracle_lib.life_step(pos, zero, zero, offs, params, goals, sp, st, 0,
                                            n_steps=spawn + k - 1)
    assert s1[0] == 0
    assert np.hypot(*(goals[:, 0] - p1[:, 0])) > 0.5
    assert np.isclose(np.hypot(*p1[:, 0]), (k - 1) * 0.25, atol=1e-5)
    p2, v2, _, s2, _ = oracle_lib.life_step(p1, v1, zero, offs, params, goals, sp, s1,
                                            spawn + k - 1, n_steps=1)
    assert s2[0] == 1
    assert np.hypot(*(goals[:, 0] - p2[:, 0])) <= 0.5


def test_spawn_step_and_removal_freeze(oracle_lib):
    pos, goals, params, offs, sp = lone((2.0, 0.0), spawn=4)
    zero = np.zeros((2, 1), np.float32)
    st = np.zeros(1, np.uint8)
    p, v, _, s, _ = oracle_lib.life_step(pos, zero, zero, offs, params, goals, sp, st, 0,
                                         n_steps=4)
    assert np.array_equal(p, pos) and s[0] == 0 and np.all(v == 0)
    p, v, _, s, _ = oracle_lib.life_step(p, v, zero, offs, params, goals, sp, s, 4, n_steps=1)
    assert p[0, 0] == np.float32(0.25) and s[0] == 0
    # arrival after ceil(1.5 / 0.25) = 6 steps from the spawn step
    p, v, _, s, _ = oracle_lib.life_step(p, v, zero, offs, params, goals, sp, s, 5, n_steps=5)
    assert s[0] == 1
    frozen = p.copy()
    far = np.array([[50.0], [0.0]], np.float32)      # a new goal far away: still removed
    p, v2, _, s, st = oracle_lib.life_step(p, v, zero, offs, params, far, sp, s, 10, n_steps=3)
    assert s[0] == 1 and np.array_equal(p, frozen) and st[0] == 2


def crowd(seed, n=300):
    w = scenes.tiny_random(n, 25.0, seed=seed, max_neighbors=10)
    rng = np.random.default_rng(seed)
    goals = ((rng.random((2, n)) - 0.5) * 25.0).astype(np.float32)
    return w, goals


@pytest.mark.parametrize("seed", range(3))
def test_absent_agents_are_invisible(oracle_lib, seed):
    w, goals = crowd(90 + seed)
    rng = np.random.default_rng(seed)
    absent = rng.random(w.n) < 0.3
    out = oracle_lib.velocities(w.pos, w.vel, w.pref_vel, w.offsets, w.params, goals=goals,
                                present=(~absent).astype(np.uint8))
    keep = np.flatnonzero(~absent)
    sub = oracle_lib.velocities(w.pos[:, keep], w.vel[:, keep], w.pref_vel[:, keep],
                                np.array([0, keep.size], np.int64), w.params,
                                goals=goals[:, keep])
    assert np.all(out["status"][absent] == 2)
    assert np.all(out["new_vel"][absent] == 0) and np.all(out["n_nbr"][absent] == 0)
    assert np.array_equal(out["new_vel"][keep], sub["new_vel"])
    assert np.array_equal(out["status"][keep], sub["status"])
    # neighbour ids map back through the kept index list
    nb = out["nbr"][keep]
    mapped = np.where(sub["nbr"] >= 0, keep[np.maximum(sub["nbr"], 0)], -1)
    assert np.array_equal(nb, mapped)


def test_future_and_removed_agents_do_not_steer_others(oracle_lib):
    w, goals = crowd(97)
    n = w.n
    spawn = np.zeros(n, np.int32)
    spawn[::5] = 1000                                  # not yet in
    state = np.zeros(n, np.uint8)
    state[1::7] = 1                                    # already out
    state[::5] = 0
    present = (spawn <= 0) & (state == 0)
    zero = np.zeros((2, n), np.float32)
    p, v, pr, s, st = oracle_lib.life_step(w.pos, zero, zero, w.offsets, w.params, goals, spawn,
                                           state, 0, n_steps=1)
    keep = np.flatnonzero(present)
    q, u, qr, _ = oracle_lib.step(w.pos[:, keep], zero[:, keep], zero[:, keep],
                                  np.array([0, keep.size], np.int64), w.params,
                                  goals=goals[:, keep])
    assert np.array_equal(p[:, keep], q) and np.array_equal(v[:, keep], u)
    assert np.array_equal(pr[:, keep], qr)
    gone = ~present
    assert np.array_equal(p[:, gone], w.pos[:, gone]) and np.all(v[:, gone] == 0)
    assert np.all(st[gone] == 2)


@pytest.mark.parametrize("ways,hetero", [(2, False), (2, True), (8, False), (8, True)])
def test_spawn_points_clear_of_recent_spawns(ways, hetero):
    w = scenes.crossing_spawn(ways=ways, hetero=hetero)
    p = w.params[0]
    r = w.radius if hetero else np.full(w.n, p.radius)
    v = w.pref_speed if hetero else np.full(w.n, p.pref_speed)
    per = w.n // ways
    checked = 0
    for g in range(ways):
        idx = np.arange(g * per, (g + 1) * per)
        for a in idx:
            for b in idx[idx < a]:
                if (w.spawn_step[a] - w.spawn_step[b]) * v[b] * p.dt < r[a] + r[b]:
                    d = np.hypot(*(w.pos[:, a].astype(np.float64) - w.pos[:, b]))
                    assert d >= r[a] + r[b], (g, a, b)
                    checked += 1
    assert checked > w.n
    assert w.spawn_step.min() == 0 and np.all(np.diff(w.spawn_step[:per]) >= 0)


@pytest.mark.parametrize("ways", [2, 8])
def test_small_crossing_runs_until_everyone_arrives(oracle_lib, ways):
    w = scenes.crossing_spawn(ways=ways, n=96 if ways == 8 else 80, spawn_steps=60, ring=12.0,
                              region=6.0)
    p = w.params[0]
    n = w.n
    pos, vel, pref = w.pos, w.vel, w.pref_vel
    state = np.zeros(n, np.uint8)
    entered = np.zeros(n, bool)
    for t in range(0, 1500, 10):
        pos, vel, pref, state, st = oracle_lib.life_step(pos, vel, pref, w.offsets, w.params,
                                                         w.goals, w.spawn_step, state, t,
                                                         n_steps=10)
        entered |= w.spawn_step <= t + 9
        ok = np.flatnonzero(st == 0)
        if ok.size > 1:
            x, y = pos[0, ok].astype(np.float64), pos[1, ok].astype(np.float64)
            d = np.hypot(x[:, None] - x[None, :], y[:, None] - y[None, :])
            np.fill_diagonal(d, np.inf)
            # both solved the 2D LP: apart up to float32 rounding of the positions
            assert d.min() > 2 * p.radius - 1e-5, t
        if state.all():
            break
    assert entered.all() and state.all(), (t, int(state.sum()))
    assert np.all(np.hypot(*(w.goals - pos)) <= p.radius)


def test_two_way_crossing_forms_lanes(oracle_lib):
    # section 4: the two crowds pass amongst each other in lanes.  From step
    # 1000 to 3000, the band order of the real groups beats that of the same
    # people with their groups shuffled.
    w = scenes.crossing_spawn(ways=2)
    group = (w.goals[0] < 0).astype(int)
    rng = np.random.default_rng(0)
    pos, vel, pref = w.pos, w.vel, w.pref_vel
    state = np.zeros(w.n, np.uint8)
    real, mixed = [], []
    for t in range(0, 3000, 100):
        pos, vel, pref, state, _ = oracle_lib.life_step(pos, vel, pref, w.offsets, w.params,
                                                        w.goals, w.spawn_step, state, t,
                                                        n_steps=100)
        if t + 100 >= 1000:
            present = (w.spawn_step <= t + 99) & (state == 0)
            real.append(lane_order(pos, present, group))
            mixed.append(np.mean([lane_order(pos, present, rng.permutation(group))
                                  for _ in range(4)]))
    assert np.mean(real) > np.mean(mixed) + 0.1, (np.mean(real), np.mean(mixed))


def test_eight_way_crossing_turns_one_way(oracle_lib):
    # section 4: every crowd crosses 135 degrees on, so the crowd as a whole
    # turns about the centre in one sense (a vortex): its angular momentum
    # about the centre keeps one sign while people are crossing.
    w = scenes.crossing_spawn(ways=8)
    pos, vel, pref = w.pos, w.vel, w.pref_vel
    state = np.zeros(w.n, np.uint8)
    lz = []
    for t in range(0, 2000, 100):
        pos, vel, pref, state, _ = oracle_lib.life_step(pos, vel, pref, w.offsets, w.params,
                                                        w.goals, w.spawn_step, state, t,
                                                        n_steps=100)
        present = (w.spawn_step <= t + 99) & (state == 0)
        if present.sum() >= w.n // 3:   # people crossing in numbers
            lz.append(turning_speed(pos, vel, present))
    assert len(lz) >= 8 and min(lz) > 0.25, lz
