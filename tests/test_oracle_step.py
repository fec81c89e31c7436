"""Whole-step pins of the reference (sections 3 and 4).

  * collision-free guarantee: if two agents that see each other both find a
    permitted velocity, their new relative motion keeps them at least R apart
    for the whole look-ahead (or separates an overlapping pair within dt);
  * every chosen speed is within the max-speed disc;
  * the step is deterministic and synchronous (x += dt v' with the v' that
    the velocity call returns);
  * goal steering: walking speed toward the goal, and the exact remaining
    offset / dt on the final step;
  * the paper's two-way crossing with its printed agent parameters keeps the
    guarantee over many steps.
"""
import json
import os

import numpy as np
import pytest

from paper_1908_10107_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def pair_checks(w, out, tol=1e-9):
    pos = w.pos.astype(np.float64)
    nv = out["new_vel"]
    nbr = out["nbr"]
    st = out["status"]
    p = w.params[0]
    R = 2 * p.radius
    sets = [set(r[r >= 0].tolist()) for r in nbr]
    pairs = 0
    for i in range(w.n):
        if st[i] != 0:
            continue
        for j in sets[i]:
            if j <= i or st[j] != 0 or i not in sets[j]:
                continue
            P = pos[:, j] - pos[:, i]
            W = nv[i] - nv[j]
            if P @ P > R * R:
                ww = W @ W
                t = 0.0 if ww == 0 else np.clip((P @ W) / ww, 0.0, p.time_horizon)
                assert np.linalg.norm(P - t * W) >= R - tol, (i, j)
            else:
                assert np.linalg.norm(P - p.dt * W) >= R - tol, (i, j)
            pairs += 1
    return pairs


@pytest.mark.parametrize("seed", range(4))
def test_collision_free_when_feasible(oracle_lib, seed):
    w = scenes.tiny_random(400, 30.0, seed=seed)
    out = oracle_lib.velocities(w.pos, w.vel, w.pref_vel, w.offsets, w.params)
    assert (out["status"] == 0).sum() > 100
    assert pair_checks(w, out) > 100


def test_collision_free_dense_with_overlaps(oracle_lib):
    w = scenes.dense_uniform(n=3000)
    out = oracle_lib.velocities(w.pos, w.vel, w.pref_vel, w.offsets, w.params, goals=w.goals)
    assert 0 < (out["status"] == 1).sum() < w.n     # both branches occur
    assert pair_checks(w, out) > 100
    sp = np.linalg.norm(out["new_vel"], axis=1)
    assert sp.max() <= w.params[0].max_speed + 1e-9


def test_step_is_euler_of_velocity_call(oracle_lib):
    w = scenes.uniform_rsa(n=1024)
    out = oracle_lib.velocities(w.pos, w.vel, w.pref_vel, w.offsets, w.params, goals=w.goals)
    pos1, vel1, pref1, st = oracle_lib.step(w.pos, w.vel, w.pref_vel, w.offsets, w.params,
                                            goals=w.goals)
    dt = float(np.float32(w.params[0].dt))   # the parameter is float32
    want = (w.pos.astype(np.float64) + dt * out["new_vel"].T).astype(np.float32)
    assert np.array_equal(pos1, want)
    assert np.array_equal(vel1, out["new_vel"].T.astype(np.float32))
    assert np.array_equal(pref1, out["vhat"].T.astype(np.float32))
    assert np.array_equal(st, out["status"])
    pos2, *_ = oracle_lib.step(w.pos, w.vel, w.pref_vel, w.offsets, w.params, goals=w.goals)
    assert np.array_equal(pos1, pos2)


def test_binned_and_definition_give_same_velocities(oracle_lib):
    w = scenes.dense_uniform(n=2000)
    a = oracle_lib.velocities(w.pos, w.vel, w.pref_vel, w.offsets, w.params, goals=w.goals,
                              neighbor_mode=0)
    b = oracle_lib.velocities(w.pos, w.vel, w.pref_vel, w.offsets, w.params, goals=w.goals,
                              neighbor_mode=1)
    assert np.array_equal(a["new_vel"], b["new_vel"])


def test_steering_closed_form(oracle_lib):
    v = oracle_lib.steer((1.0, 2.0), (4.0, 6.0), 1.3, 0.1)
    np.testing.assert_allclose(v, [0.78, 1.04], atol=1e-15)
    v = oracle_lib.steer((1.0, 2.0), (1.06, 2.08), 1.3, 0.1)    # 0.1 m left < 0.13 m
    np.testing.assert_allclose(v, [0.6, 0.8], atol=1e-12)
    v = oracle_lib.steer((1.0, 2.0), (1.0, 2.0), 1.3, 0.1)
    assert np.array_equal(v, [0.0, 0.0])


def test_no_neighbours_is_clipped_preference(oracle_lib):
    w = scenes.tiny_random(3, 1000.0, seed=5)
    w.pref_vel[:] = np.array([[3.0, 0.1, -1.0], [4.0, 0.2, 0.0]], np.float32)
    out = oracle_lib.velocities(w.pos, w.vel, w.pref_vel, w.offsets, w.params)
    assert (out["n_nbr"] == 0).all()
    np.testing.assert_allclose(out["new_vel"][0], [0.9, 1.2], atol=1e-15)
    np.testing.assert_allclose(out["new_vel"][1], [0.1, 0.2], atol=1e-8)


def test_two_way_crossing_with_paper_parameters(oracle_lib):
    """Two crowds swap sides with the agent parameters printed for that scenario."""
    with open(os.path.join(GOLDEN, "paper_agent_parameters.json")) as f:
        g = json.load(f)["two_way_crossing"]
    rng = np.random.default_rng(11)
    n_side = 60
    a = np.stack([rng.uniform(-30, -20, n_side), rng.uniform(-8, 8, n_side)])
    b = np.stack([rng.uniform(20, 30, n_side), rng.uniform(-8, 8, n_side)])
    pos = np.concatenate([a, b], 1)
    # spread starts so nobody overlaps (the paper spawns without overlap)
    from scipy.spatial import cKDTree
    while True:
        d, _ = cKDTree(pos.T).query(pos.T, k=2)
        bad = d[:, 1] < 2 * g["radius_m"] + 0.05
        if not bad.any():
            break
        pos[:, bad] += rng.normal(size=(2, bad.sum())) * 0.5
    goals = np.concatenate([b, a], 1)
    p = scenes.SceneParams(radius=g["radius_m"], max_speed=g["max_speed_mps"],
                           pref_speed=g["desired_speed_mps"], neighbor_dist=5.0,
                           time_horizon=5.0, dt=0.1, max_neighbors=10)
    w = scenes.Workload("cross", pos.astype(np.float32), np.zeros_like(pos, np.float32),
                        goals.astype(np.float32), np.zeros_like(pos, np.float32),
                        np.array([0, pos.shape[1]]), [p], 1)
    for _ in range(60):
        out = oracle_lib.velocities(w.pos, w.vel, w.pref_vel, w.offsets, w.params,
                                    goals=w.goals)
        pair_checks(w, out)
        assert np.linalg.norm(out["new_vel"], axis=1).max() <= p.max_speed + 1e-9
        w.pos, w.vel, w.pref_vel, _ = oracle_lib.step(w.pos, w.vel, w.pref_vel, w.offsets,
                                                      w.params, goals=w.goals)
    # the crowds made progress toward their goals
    assert np.linalg.norm(w.goals - w.pos, axis=0).mean() < np.linalg.norm(goals - pos, axis=0).mean() - 3.0


def test_scene_offsets_are_checked_against_the_agents(oracle_lib):
    # the C reference trusts the offsets for every array bound, so the binding
    # refuses offsets that do not split the agents into the scenes
    w = scenes.tiny_random(50, 10.0, seed=3)
    for bad in ([0, 52], [0, 30, 25, 50], [1, 50], [0, 50, 50]):
        with pytest.raises(ValueError):
            oracle_lib.velocities(w.pos, w.vel, w.pref_vel, np.array(bad), w.params)
    with pytest.raises(ValueError):
        oracle_lib.step(w.pos, w.vel, w.pref_vel, [0, 49], w.params)
    oracle_lib.velocities(w.pos, w.vel, w.pref_vel, [0, 50], w.params)


def test_lone_walkers_closed_form(oracle_lib):
    """The Euler update and goal steering against their closed form: agents
    far beyond each other's observation radius walk straight at their walking
    speed s (or at v_max when v_max < s), covering min(s, v_max) * dt per step,
    reach the goal on the step that leaves at most that far to go, and then
    stand still.  Positions follow x_n = x_0 + n * v * dt up to one float32
    rounding per step."""
    dt = 0.1
    cases = [  # start, goal, s, v_max
        ((0.0, 0.0), (10.05, 0.0), 1.3, 1.5),
        ((1000.0, 0.0), (1000.0, -7.03), 1.3, 1.0),       # clipped to v_max
        ((-1000.0, 500.0), (-1000.0, 505.25), 2.0, 2.5),
        ((500.0, -800.0), (496.13, -800.0), 0.7, 1.5),
    ]  # distances off multiples of v * dt, so float32 drift cannot move the arrival step
    n = len(cases)
    pos = np.array([c[0] for c in cases], np.float32).T.copy()
    goals = np.array([c[1] for c in cases], np.float32).T.copy()
    # one scene per walker, so each has its own walking and max speed
    params = [scenes.SceneParams(pref_speed=c[2], max_speed=c[3], dt=dt) for c in cases]
    w = scenes.Workload("walkers", pos, np.zeros((2, n), np.float32), goals,
                        np.zeros((2, n), np.float32), np.arange(n + 1), params, 1)
    x, v, pref = w.pos, w.vel, w.pref_vel
    dt32 = float(np.float32(dt))
    speed = np.array([min(np.float32(c[2]), np.float32(c[3])) for c in cases], np.float64)
    start = pos.astype(np.float64)
    dist = np.linalg.norm(goals.astype(np.float64) - start, axis=0)
    unit = (goals.astype(np.float64) - start) / dist
    arrive = np.ceil(dist / (speed * dt32) - 1e-9).astype(int)
    for step in range(1, int(arrive.max()) + 4):
        x, v, pref, st = oracle_lib.step(x, v, pref, w.offsets, w.params, goals=w.goals)
        assert np.all(st == 0)
        for i in range(n):
            walked = min(step * speed[i] * dt32, dist[i])
            want = start[:, i] + walked * unit[:, i]
            tol = (step + 1) * np.spacing(np.float32(np.abs(want).max() + 1.0))
            assert np.abs(x[:, i] - want).max() <= tol, (i, step, x[:, i], want)
            if step < arrive[i]:
                # full speed along the goal direction
                np.testing.assert_allclose(v[:, i], speed[i] * unit[:, i], atol=1e-6)
            else:
                # on the goal from the arrival step on, then standing (rounding only)
                assert np.abs(x[:, i] - goals[:, i]).max() <= 2 * np.spacing(
                    np.float32(np.abs(goals[:, i]).max())), (i, step)
                if step > arrive[i]:
                    assert np.abs(v[:, i]).max() <= 1e-3
