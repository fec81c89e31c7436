"""Pins of the reference with per-agent properties (section 4: the crossing
whose people differ in size and speed).

  * the collision-free guarantee with a pair's combined radius r_i + r_j;
  * each agent's speed stays within its own max speed, and an agent with no
    neighbours takes its preferred velocity clipped to its own max speed;
  * goal steering walks at the agent's own desired speed;
  * per-agent arrays that hold the scene's values give the scene's results
    bit for bit (the per-agent path adds nothing else);
  * the paper's heterogeneous crossing, with its printed radius and speed
    choices (tests/golden/paper_agent_parameters.json), keeps the guarantee.
"""
import json
import os

import numpy as np
import pytest

from paper_1908_10107_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def hetero_pair_checks(w, out, radius, tol=1e-9):
    """No overlap within tau (or separation within dt for pairs already in
    contact) for mutual neighbours that both found a permitted velocity."""
    pos = w.pos.astype(np.float64)
    nv = out["new_vel"]
    st = out["status"]
    p = w.params[0]
    sets = [set(r[r >= 0].tolist()) for r in out["nbr"]]
    pairs = 0
    for i in range(w.n):
        if st[i] != 0:
            continue
        for j in sets[i]:
            if j <= i or st[j] != 0 or i not in sets[j]:
                continue
            R = float(radius[i]) + float(radius[j])
            P = pos[:, j] - pos[:, i]
            W = nv[i] - nv[j]
            if P @ P > R * R:
                ww = W @ W
                t = 0.0 if ww == 0 else np.clip((P @ W) / ww, 0.0, p.time_horizon)
                assert np.linalg.norm(P - t * W) >= R - tol, (i, j)
            else:
                assert np.linalg.norm(P - float(np.float32(p.dt)) * W) >= R - tol, (i, j)
            pairs += 1
    return pairs


@pytest.mark.parametrize("seed", range(3))
def test_collision_free_with_combined_radii(oracle_lib, seed):
    w = scenes.tiny_random(500, 45.0, seed=70 + seed, max_neighbors=16)
    rng = np.random.default_rng(seed)
    radius = rng.choice(np.array([0.1, 0.25, 0.5, 0.75], np.float32), w.n)
    out = oracle_lib.velocities(w.pos, w.vel, w.pref_vel, w.offsets, w.params, radius=radius)
    assert (out["status"] == 0).sum() > 100
    assert hetero_pair_checks(w, out, radius) > 100


def test_own_max_speed_caps_each_agent(oracle_lib):
    w = scenes.tiny_random(1500, 40.0, seed=75, max_neighbors=16)
    rng = np.random.default_rng(5)
    vmax = rng.uniform(0.3, 2.5, w.n).astype(np.float32)
    out = oracle_lib.velocities(w.pos, w.vel, w.pref_vel, w.offsets, w.params, max_speed=vmax)
    sp = np.linalg.norm(out["new_vel"], axis=1)
    assert np.all(sp <= vmax.astype(np.float64) + 1e-9)
    assert np.sum(sp > w.params[0].max_speed + 1e-6) > 10   # the scene cap is not what binds


def test_lone_agents_take_their_own_clip(oracle_lib):
    w = scenes.tiny_random(3, 1000.0, seed=5)
    w.pref_vel[:] = np.array([[3.0, 0.1, -1.0], [4.0, 0.2, 0.0]], np.float32)
    vmax = np.array([2.5, 0.1, 5.0], np.float32)
    out = oracle_lib.velocities(w.pos, w.vel, w.pref_vel, w.offsets, w.params, max_speed=vmax)
    assert (out["n_nbr"] == 0).all()
    np.testing.assert_allclose(out["new_vel"][0], [1.5, 2.0], atol=1e-7)   # |(3,4)| = 5 -> 2.5
    s = float(np.float32(0.1)) / np.hypot(0.1, 0.2)
    np.testing.assert_allclose(out["new_vel"][1], [0.1 * s, 0.2 * s], rtol=1e-6)
    np.testing.assert_allclose(out["new_vel"][2], [-1.0, 0.0], atol=1e-15)


def test_steering_at_each_agents_speed(oracle_lib):
    w = scenes.tiny_random(4, 1000.0, seed=6)
    w.goals = np.ascontiguousarray(w.pos + np.array([[300.0], [400.0]], np.float32))
    speed = np.array([1.0, 1.33, 2.0, 0.5], np.float32)
    out = oracle_lib.velocities(w.pos, w.vel, w.pref_vel, w.offsets, w.params, goals=w.goals,
                                pref_speed=speed, max_speed=np.full(4, 5.0, np.float32))
    np.testing.assert_allclose(np.linalg.norm(out["vhat"], axis=1), speed, rtol=1e-6)
    np.testing.assert_allclose(out["new_vel"], out["vhat"], atol=1e-12)   # alone: v' = vhat


def test_scene_values_as_arrays_change_nothing(oracle_lib):
    w = scenes.dense_uniform(n=3000)
    p = w.params[0]
    a = oracle_lib.velocities(w.pos, w.vel, w.pref_vel, w.offsets, w.params, goals=w.goals)
    b = oracle_lib.velocities(w.pos, w.vel, w.pref_vel, w.offsets, w.params, goals=w.goals,
                              radius=np.full(w.n, p.radius, np.float32),
                              max_speed=np.full(w.n, p.max_speed, np.float32),
                              pref_speed=np.full(w.n, p.pref_speed, np.float32))
    assert np.array_equal(a["new_vel"], b["new_vel"])
    assert np.array_equal(a["nbr"], b["nbr"])


def test_paper_heterogeneous_crossing_keeps_the_guarantee(oracle_lib):
    with open(os.path.join(GOLDEN, "paper_agent_parameters.json")) as f:
        g = json.load(f)["two_way_crossing_heterogeneous"]
    w = scenes.crossing_hetero(n=600, density=0.2, height=30.0, gap=5.0)
    assert set(np.unique(w.radius).astype(np.float64).round(3)) == set(np.round(g["radius_m"], 3))
    assert (set(np.unique(w.pref_speed).astype(np.float64).round(3)) ==
            set(np.round(g["desired_speed_mps"], 3)))
    np.testing.assert_allclose(w.max_speed, g["max_speed_over_desired"] * w.pref_speed, rtol=1e-6)
    pos, vel, pref = w.pos, w.vel, w.pref_vel
    checked = 0
    for t in range(40):
        st = scenes.Workload("s", pos, vel, w.goals, pref, w.offsets, w.params, 1)
        out = oracle_lib.velocities(pos, vel, pref, w.offsets, w.params, goals=w.goals,
                                    radius=w.radius, max_speed=w.max_speed,
                                    pref_speed=w.pref_speed)
        sp = np.linalg.norm(out["new_vel"], axis=1)
        assert np.all(sp <= w.max_speed.astype(np.float64) + 1e-9)
        if t % 10 == 0:
            checked += hetero_pair_checks(st, out, w.radius)
        pos, vel, pref, _ = oracle_lib.step(pos, vel, pref, w.offsets, w.params, goals=w.goals,
                                            radius=w.radius, max_speed=w.max_speed,
                                            pref_speed=w.pref_speed)
    assert checked > 50
