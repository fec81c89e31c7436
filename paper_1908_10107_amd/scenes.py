"""Seeded synthetic workloads for the ORCA step.

This module only draws inputs: start positions, goals, preferred velocities for
the fixed-leaf workload, and the per-scene parameters.  It contains none of the
collision-avoidance arithmetic, so both the GPU library and the CPU reference can
consume its output without sharing any of the method's code.

The paper (section 4) evaluates on synthetic crossing scenarios whose people
spawn at random non-overlapping points; it names no public dataset.  The five
workloads below follow that recipe at the sizes the measurements use:

* ``uniform_rsa``   1,024 agents at 0.5 agents/m^2, random sequential addition
  with minimum separation 2r, goals uniform in the same square.
* ``ring``          65,536 agents evenly spaced on a 1,200 m circle, goal = the
  antipodal point.
* ``dense_uniform`` 1,048,576 agents uniform at 2 agents/m^2 (no rejection, so
  many pairs start overlapping and many LPs are infeasible), K=16, 3 m radius.
* ``batched``       512 independent scenes with log-uniform sizes in [64, 16384],
  per-scene density, max speed and time horizon.
* ``grad``          4,096 agents uniform at 1 agent/m^2 with a fixed preferred
  velocity per agent and a target point per agent.
* ``crossing_hetero`` the two-way crossing whose people differ in size and
  speed (section 4): two groups swap places; per-agent radius 0.5, 0.75 or
  1 m and desired speed 1, 1.33 or 2 m/s, each equally likely, max speed 125%
  of the desired speed.
* ``crossing_spawn`` the 2-way and 8-way crossings with people entering over
  time and leaving at their goal (section 4): start regions spawn at a steady
  rate, each new person clear of everyone spawned in the same region within a
  time window set by size and speed; goals are uniform in the paired end region
  (the other group's start region; for 8 ways, the region 135 degrees on).

Every generator is deterministic in its seed (``numpy.random.default_rng``).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

BASE_SEED = 190810107

# Agent parameters shared by the single-scene workloads.
DEFAULT_PARAMS = dict(radius=0.25, max_speed=1.5, neighbor_dist=5.0,
                      time_horizon=5.0, dt=0.1, pref_speed=1.3, max_neighbors=10)


@dataclasses.dataclass
class SceneParams:
    radius: float = 0.25
    max_speed: float = 1.5
    neighbor_dist: float = 5.0
    time_horizon: float = 5.0
    dt: float = 0.1
    pref_speed: float = 1.3
    max_neighbors: int = 10


@dataclasses.dataclass
class Workload:
    """A batch of independent scenes laid out back to back.

    Arrays are float32 ``[2, N]`` (row 0 = x, row 1 = y) over all agents of all
    scenes; scene ``s`` owns agents ``offsets[s]:offsets[s+1]``.
    """
    name: str
    pos: np.ndarray
    vel: np.ndarray
    goals: Optional[np.ndarray]
    pref_vel: np.ndarray
    offsets: np.ndarray
    params: List[SceneParams]
    steps: int
    targets: Optional[np.ndarray] = None
    # optional per-agent properties [N] float32 (None: the scene's value)
    radius: Optional[np.ndarray] = None
    max_speed: Optional[np.ndarray] = None
    pref_speed: Optional[np.ndarray] = None
    # optional step at which each agent enters [N] int32 (None: all from the start)
    spawn_step: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return int(self.offsets[-1])

    @property
    def n_scenes(self) -> int:
        return len(self.params)

    def subset_scenes(self, idx) -> "Workload":
        """Return a workload made of the listed scenes only (copied)."""
        idx = list(idx)
        parts = [(int(self.offsets[s]), int(self.offsets[s + 1])) for s in idx]
        cat = lambda a: None if a is None else np.ascontiguousarray(
            np.concatenate([a[:, lo:hi] for lo, hi in parts], axis=1))
        sizes = [hi - lo for lo, hi in parts]
        offs = np.zeros(len(idx) + 1, np.int64)
        offs[1:] = np.cumsum(sizes)
        cat1 = lambda a: None if a is None else np.ascontiguousarray(
            np.concatenate([a[lo:hi] for lo, hi in parts]))
        return Workload(self.name + "_subset", cat(self.pos), cat(self.vel), cat(self.goals),
                        cat(self.pref_vel), offs, [self.params[s] for s in idx], self.steps,
                        cat(self.targets), cat1(self.radius), cat1(self.max_speed),
                        cat1(self.pref_speed))


def _rsa_square(rng: np.random.Generator, n: int, side: float, dmin: float,
                margin: float = 1e-4) -> np.ndarray:
    """Random sequential addition of ``n`` points in ``[-side/2, side/2]^2``.

    Proposals are drawn in batches; a proposal is kept if it is at least
    ``dmin + margin`` from every kept point and from every earlier proposal
    of its batch.  The margin keeps the separation >= ``dmin`` after the
    coordinates are rounded to float32.
    """
    from scipy.spatial import cKDTree

    need = dmin + margin
    kept = np.empty((0, 2))
    tries = 0
    while kept.shape[0] < n:
        tries += 1
        if tries > 10000:
            raise RuntimeError("random sequential addition did not converge")
        b = max(2 * (n - kept.shape[0]), 256)
        cand = (rng.random((b, 2)) - 0.5) * side
        if kept.shape[0]:
            d, _ = cKDTree(kept).query(cand, k=1)
            cand = cand[d >= need]
        if cand.shape[0] > 1:
            pairs = cKDTree(cand).query_pairs(need, output_type="ndarray")
            if pairs.size:
                drop = np.zeros(cand.shape[0], bool)
                drop[pairs.max(axis=1)] = True
                cand = cand[~drop]
        kept = np.concatenate([kept, cand[: n - kept.shape[0]]], axis=0)
    return kept


def _rsa_box_radii(rng: np.random.Generator, radii: np.ndarray, box, margin: float = 1e-4):
    """Random sequential addition of discs in the box (x0, x1, y0, y1): a
    proposal of radius r is kept if it is at least r + r_j + margin from every
    kept disc j and from every earlier proposal of its batch.  Each proposal
    takes a radius from those not yet placed; returns (centres [n, 2], radii in
    the order placed), a permutation of ``radii``."""
    from scipy.spatial import cKDTree

    x0, x1, y0, y1 = box
    rmax = float(radii.max()) if len(radii) else 0.0
    reach = 2 * rmax + margin
    kept = np.empty((0, 2))
    kept_r = np.empty(0)
    todo = np.array(radii, dtype=np.float64)
    tries = 0
    while todo.size:
        tries += 1
        if tries > 10000:
            raise RuntimeError("random sequential addition did not converge")
        b = max(256, 2 * todo.size)
        cand = np.stack([rng.uniform(x0, x1, b), rng.uniform(y0, y1, b)], axis=1)
        cr = todo[rng.integers(0, todo.size, b)]
        ok = np.ones(b, bool)
        if kept.shape[0]:
            k = min(32, kept.shape[0])
            d, j = cKDTree(kept).query(cand, k=k, distance_upper_bound=reach)
            d = d.reshape(b, k)
            j = j.reshape(b, k)
            rj = np.where(j < kept.shape[0], kept_r[np.minimum(j, kept.shape[0] - 1)], 0.0)
            ok = np.all(d >= cr[:, None] + rj + margin, axis=1)
        pairs = cKDTree(cand).query_pairs(reach, output_type="ndarray")
        if pairs.size:
            dd = np.hypot(*(cand[pairs[:, 0]] - cand[pairs[:, 1]]).T)
            bad = pairs[dd < cr[pairs[:, 0]] + cr[pairs[:, 1]] + margin]
            ok[bad.max(axis=1)] = False
        cand, cr = cand[ok], cr[ok]
        # take only radii still to place (a radius value is used as often as it occurs)
        vals, counts = np.unique(todo, return_counts=True)
        take = np.zeros(cand.shape[0], bool)
        for v, c in zip(vals, counts):
            idx = np.flatnonzero(cr == v)[:c]
            take[idx] = True
        cand, cr = cand[take], cr[take]
        kept = np.concatenate([kept, cand], axis=0)
        kept_r = np.concatenate([kept_r, cr])
        for v in np.unique(cr):
            c = int(np.sum(cr == v))
            idx = np.flatnonzero(todo == v)[:c]
            todo = np.delete(todo, idx)
    return kept, kept_r


def _check_separation(p32: np.ndarray, dmin: float) -> None:
    from scipy.spatial import cKDTree
    pts = p32.T.astype(np.float64)
    if pts.shape[0] > 1:
        d, _ = cKDTree(pts).query(pts, k=2)
        assert d[:, 1].min() >= dmin, "separation lost in float32 rounding"


def _pack(name, pos_list, goal_list, params, steps, pref_list=None, targets=None):
    pos = np.ascontiguousarray(np.concatenate(pos_list, axis=1).astype(np.float32))
    goals = None if goal_list is None else np.ascontiguousarray(
        np.concatenate(goal_list, axis=1).astype(np.float32))
    n = pos.shape[1]
    pref = (np.zeros((2, n), np.float32) if pref_list is None else
            np.ascontiguousarray(np.concatenate(pref_list, axis=1).astype(np.float32)))
    offs = np.zeros(len(pos_list) + 1, np.int64)
    offs[1:] = np.cumsum([p.shape[1] for p in pos_list])
    return Workload(name, pos, np.zeros((2, n), np.float32), goals, pref, offs, params, steps,
                    targets)


def uniform_rsa(n: int = 1024, density: float = 0.5, seed: int = BASE_SEED + 0,
                steps: int = 100, **over) -> Workload:
    """Uniform square, rejection-sampled to separation 2r; goals uniform."""
    rng = np.random.default_rng(seed)
    p = SceneParams(**{**DEFAULT_PARAMS, **over})
    side = math.sqrt(n / density)
    pos = _rsa_square(rng, n, side, 2 * p.radius).T.astype(np.float32)
    _check_separation(pos, 2 * p.radius)
    goals = ((rng.random((n, 2)) - 0.5) * side).T
    return _pack("uniform_rsa", [pos], [goals], [p], steps)


def ring(n: int = 65536, radius_m: float = 1200.0, steps: int = 2000, **over) -> Workload:
    """Agents evenly spaced on a circle; each heads for the antipodal point."""
    p = SceneParams(**{**DEFAULT_PARAMS, **over})
    th = 2.0 * np.pi * np.arange(n, dtype=np.float64) / n
    pos = np.stack([radius_m * np.cos(th), radius_m * np.sin(th)])
    return _pack("ring", [pos], [-pos], [p], steps)


def dense_uniform(n: int = 1 << 20, density: float = 2.0, seed: int = BASE_SEED + 2,
                  steps: int = 500, **over) -> Workload:
    """Plain uniform square (no rejection): overlapping starts, many infeasible LPs."""
    rng = np.random.default_rng(seed)
    kw = {**DEFAULT_PARAMS, "max_neighbors": 16, "neighbor_dist": 3.0}
    kw.update(over)
    p = SceneParams(**kw)
    side = math.sqrt(n / density)
    pos = ((rng.random((n, 2)) - 0.5) * side).T
    goals = ((rng.random((n, 2)) - 0.5) * side).T
    return _pack("dense_uniform", [pos], [goals], [p], steps)


def batched(n_scenes: int = 512, seed: int = BASE_SEED + 3, steps: int = 300,
            n_min: int = 64, n_max: int = 16384, density=(0.3, 2.0)) -> Workload:
    """Independent scenes of log-uniform size with per-scene density (uniform in
    ``density``), v_max and tau."""
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), n_scenes))).astype(int)
    dens = rng.uniform(density[0], density[1], n_scenes)
    vmax = rng.uniform(1.0, 2.0, n_scenes)
    tau = rng.uniform(2.0, 8.0, n_scenes)
    pos_l, goal_l, params = [], [], []
    for s in range(n_scenes):
        p = SceneParams(**{**DEFAULT_PARAMS, "max_speed": float(vmax[s]),
                           "time_horizon": float(tau[s])})
        side = math.sqrt(sizes[s] / dens[s])
        pos = _rsa_square(rng, int(sizes[s]), side, 2 * p.radius).T.astype(np.float32)
        _check_separation(pos, 2 * p.radius)
        pos_l.append(pos)
        goal_l.append(((rng.random((int(sizes[s]), 2)) - 0.5) * side).T)
        params.append(p)
    return _pack("batched", pos_l, goal_l, params, steps)


def grad(n: int = 4096, density: float = 1.0, seed: int = BASE_SEED + 4, steps: int = 200,
         **over) -> Workload:
    """Uniform square with a fixed preferred velocity per agent and a target per agent.

    The preferred velocity has speed ``pref_speed`` and a uniform random heading;
    targets come from a separate random stream.
    """
    rng = np.random.default_rng(seed)
    p = SceneParams(**{**DEFAULT_PARAMS, **over})
    side = math.sqrt(n / density)
    pos = ((rng.random((n, 2)) - 0.5) * side).T
    ang = rng.uniform(0.0, 2.0 * np.pi, n)
    pref = p.pref_speed * np.stack([np.cos(ang), np.sin(ang)])
    trng = np.random.default_rng(seed + 1000)
    targets = ((trng.random((n, 2)) - 0.5) * side).T.astype(np.float32)
    return _pack("grad", [pos], None, [p], steps, pref_list=[pref], targets=targets)


def crossing_hetero(n: int = 2500, density: float = 0.2, gap: float = 10.0, height: float = 100.0,
                    seed: int = BASE_SEED + 5, steps: int = 600, **over) -> Workload:
    """Two-way crossing of people of different sizes and speeds (section 4).

    Two groups of n/2 swap places: each starts in a rectangle of height
    ``height`` at density ``density`` on one side of a ``2 gap`` wide corridor
    and heads for its mirror image in the other group's start region.  Radius
    and desired speed are drawn independently with equal probability from the
    values the paper gives; max speed is 125% of the desired speed.
    Positions are random sequential additions with separation r_i + r_j.
    """
    rng = np.random.default_rng(seed)
    kw = {**DEFAULT_PARAMS, "radius": 0.75, "max_speed": 1.25 * 1.33, "pref_speed": 1.33}
    kw.update(over)
    p = SceneParams(**kw)
    half = n // 2
    width = (half / density) / height
    radius = rng.choice(np.array([0.5, 0.75, 1.0]), n)
    speed = rng.choice(np.array([1.0, 1.33, 2.0]), n)
    left, rl = _rsa_box_radii(rng, radius[:half], (-gap - width, -gap, -height / 2, height / 2))
    right, rr = _rsa_box_radii(rng, radius[half:], (gap, gap + width, -height / 2, height / 2))
    radius = np.concatenate([rl, rr])
    pos = np.concatenate([left, right], axis=0).T
    goals = pos.copy()
    goals[0] = -goals[0]
    w = _pack("crossing_hetero", [pos], [goals], [p], steps)
    w.radius = radius.astype(np.float32)
    w.pref_speed = speed.astype(np.float32)
    w.max_speed = (1.25 * speed).astype(np.float32)
    return w


def crossing_spawn(ways: int = 2, n: int = 2500, spawn_steps: Optional[int] = None,
                   ring: Optional[float] = None, region: Optional[float] = None,
                   hetero: bool = False, seed: int = BASE_SEED + 6, steps: int = 6000,
                   **over) -> Workload:
    """2-way or 8-way crossing with spawning (section 4).

    ``ways`` square start regions of side ``region`` sit on a circle of radius
    ``ring`` (2 ways: facing each other across it).  Each spawns n / ways
    people at a steady rate over ``spawn_steps`` steps.  Defaults: a 40 m
    region, a 50 m ring and 3000 steps for 2 ways, a 20 m region, a 50 m ring
    and 1000 steps for 8 (about 4 and 3 people a second per region: crowds
    dense enough to form lanes, sparse enough to clear in a few thousand
    steps).  A spawn point is drawn
    uniformly in the region and redrawn while it is within r_i + r_j of anyone
    spawned in that region too recently to have walked r_i + r_j at their
    desired speed.  Goals are uniform in the paired end region:
    the opposite one for 2 ways, the one 135 degrees on for 8 ways.  With
    ``hetero`` the people draw radius and desired speed as in the second
    variation of the 2-way crossing; otherwise they share the first variation's
    radius 0.5 m, desired speed 1.0 m/s and max speed 1.33 m/s.
    """
    if ways not in (2, 8):
        raise ValueError("ways must be 2 or 8")
    spawn_steps = spawn_steps or (3000 if ways == 2 else 1000)
    ring = ring or 50.0
    region = region or (40.0 if ways == 2 else 20.0)
    rng = np.random.default_rng(seed)
    kw = {**DEFAULT_PARAMS, "radius": 0.5, "max_speed": 1.33, "pref_speed": 1.0}
    kw.update(over)
    p = SceneParams(**kw)
    per = n // ways
    n = per * ways
    if hetero:
        radius = rng.choice(np.array([0.5, 0.75, 1.0]), n)
        speed = rng.choice(np.array([1.0, 1.33, 2.0]), n)
        vmax = 1.25 * speed
    else:
        radius = np.full(n, p.radius)
        speed = np.full(n, p.pref_speed)
        vmax = np.full(n, p.max_speed)
    ang = 2.0 * np.pi * np.arange(ways) / ways
    centres = ring * np.stack([np.cos(ang), np.sin(ang)], axis=1)
    end = (np.arange(ways) + (1 if ways == 2 else 3)) % ways   # 2: opposite; 8: 135 degrees
    pos = np.zeros((n, 2))
    goals = np.zeros((n, 2))
    spawn = np.zeros(n, np.int32)
    for g in range(ways):
        idx = np.arange(g * per, (g + 1) * per)
        spawn[idx] = (np.arange(per) * spawn_steps) // per
        first = idx[0]
        for i in idx:
            # j still covers its spawn point while it has walked less than r_i + r_j
            j = np.arange(first, i)
            recent = j[(spawn[i] - spawn[j]) * speed[j] * p.dt < radius[i] + radius[j]]
            for _ in range(10000):
                q = centres[g] + (rng.random(2) - 0.5) * region
                d = np.hypot(pos[recent, 0] - q[0], pos[recent, 1] - q[1])
                if np.all(d >= radius[recent] + radius[i] + 1e-3):
                    break
            else:
                raise RuntimeError("no free spawn point; enlarge the region or the spawn time")
            pos[i] = q
            goals[i] = centres[end[g]] + (rng.random(2) - 0.5) * region
    w = _pack("crossing_spawn%d" % ways, [pos.T], [goals.T], [p], steps)
    w.spawn_step = spawn
    if hetero:
        w.radius = radius.astype(np.float32)
        w.pref_speed = speed.astype(np.float32)
        w.max_speed = vmax.astype(np.float32)
    return w


def tiny_random(n: int, side: float, seed: int, vel_scale: float = 1.0, **over) -> Workload:
    """Small uniform scene with random current and preferred velocities (parity cases)."""
    rng = np.random.default_rng(seed)
    p = SceneParams(**{**DEFAULT_PARAMS, **over})
    pos = ((rng.random((n, 2)) - 0.5) * side).T
    w = _pack("tiny_random", [pos], [((rng.random((n, 2)) - 0.5) * side).T], [p], 1,
              pref_list=[(rng.random((n, 2)) - 0.5).T * 2.0 * p.pref_speed])
    w.vel = np.ascontiguousarray(((rng.random((n, 2)) - 0.5).T * 2.0 * vel_scale)
                                 .astype(np.float32))
    return w


WORKLOADS = {
    "uniform_rsa": uniform_rsa,
    "ring": ring,
    "dense_uniform": dense_uniform,
    "batched": batched,
    "grad": grad,
    "crossing_hetero": crossing_hetero,
    "crossing_spawn": crossing_spawn,
}
