"""ctypes front end of the CPU reference (``orca_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The GPU library never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orca_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GCC_FLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
             "-fno-fast-math"]

ARC, LEFT, RIGHT, OVERLAP = 0, 1, 2, 3
DELTA = 1e-5


def build(force: bool = True) -> str:
    """Compile the reference with gcc (always when ``force``)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OracleParams(ctypes.Structure):
    _fields_ = [("radius", ctypes.c_float), ("max_speed", ctypes.c_float),
                ("neighbor_dist", ctypes.c_float), ("time_horizon", ctypes.c_float),
                ("dt", ctypes.c_float), ("pref_speed", ctypes.c_float),
                ("max_neighbors", ctypes.c_int32), ("pad", ctypes.c_int32)]


class HalfPlane(ctypes.Structure):
    _fields_ = [("qx", ctypes.c_double), ("qy", ctypes.c_double),
                ("nx", ctypes.c_double), ("ny", ctypes.c_double)]


class OracleAgents(ctypes.Structure):
    """Per-agent radius, max speed and walking speed ([N] float32 or NULL each) and
    presence ([N] uint8, 0 = not in the simulation, or NULL)."""
    _fields_ = [("radius", ctypes.c_void_p), ("max_speed", ctypes.c_void_p),
                ("pref_speed", ctypes.c_void_p), ("present", ctypes.c_void_p)]


_lib = None
P = ctypes.c_void_p
I64, I32, F32, F64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_float, ctypes.c_double


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        L.oracle_threads.argtypes = []
        L.oracle_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = None
        L.oracle_dist2_f32.argtypes = [F32, F32, F32, F32]
        L.oracle_dist2_f32.restype = F32
        L.oracle_knn_brute.argtypes = [I64, P, I64, I64, I64, F32, I32, P, P]
        L.oracle_knn_brute.restype = I32
        L.oracle_knn_binned_scene.argtypes = [I64, P, I64, I64, F32, I32, P]
        L.oracle_knn_binned_scene.restype = None
        L.oracle_halfplane.argtypes = [F64, F64, F64, F64, F64, F64, F64, ctypes.c_int] + [P] * 4
        L.oracle_halfplane.restype = ctypes.c_int
        L.oracle_project.argtypes = [ctypes.c_int, P, F64, F64, F64, F64, P, P]
        L.oracle_project.restype = ctypes.c_int
        L.oracle_min_max.argtypes = [ctypes.c_int, P, F64, P, P]
        L.oracle_min_max.restype = F64
        L.oracle_steer.argtypes = [F64] * 6 + [P, P]
        L.oracle_steer.restype = None
        L.oracle_velocities.argtypes = [I64, P, P, P, P, P, I32, P, P, P, I64, I32, I32,
                                        P, P, P, P, P, P]
        L.oracle_velocities.restype = None
        L.oracle_step.argtypes = [I64, P, P, P, P, P, I32, P, P, I32, P]
        L.oracle_step.restype = None
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float32)


def _agents(radius=None, max_speed=None, pref_speed=None, present=None):
    """(OracleAgents or None, arrays to keep alive) for optional per-agent properties."""
    arrs = [_f32(a) for a in (radius, max_speed, pref_speed)]
    arrs.append(None if present is None else np.ascontiguousarray(present, np.uint8))
    if all(a is None for a in arrs):
        return None, arrs
    return ctypes.byref(OracleAgents(*[_ptr(a) for a in arrs])), arrs


def _offsets(offsets, n, n_scenes):
    """Scene offsets as int64, checked against the agent count: the C code
    trusts them for every array bound."""
    off = np.ascontiguousarray(offsets, np.int64)
    if off.ndim != 1 or off.size != n_scenes + 1 or off[0] != 0 or off[-1] != n or \
            np.any(np.diff(off) < 0):
        raise ValueError("scene offsets %s do not split %d agents into %d scenes"
                         % (off.tolist()[:8], n, n_scenes))
    return off


def params_array(params):
    arr = (OracleParams * len(params))()
    for s, p in enumerate(params):
        arr[s] = OracleParams(p.radius, p.max_speed, p.neighbor_dist, p.time_horizon, p.dt,
                              p.pref_speed, p.max_neighbors, 0)
    return arr


# ---------------------------------------------------------------- primitives

def threads() -> int:
    return lib().oracle_threads()


def set_threads(n: int) -> None:
    """Threads of later calls (n <= 0: one per processor)."""
    lib().oracle_set_threads(int(n))


def dist2_f32(xi, yi, xj, yj) -> float:
    return lib().oracle_dist2_f32(xi, yi, xj, yj)


def halfplane(P_, V, R, tau, dt, i_before_j=True):
    """Return (branch, u, n) for relative position P = x_j - x_i and velocity V = v_i - v_j."""
    out = [ctypes.c_double() for _ in range(4)]
    code = lib().oracle_halfplane(float(P_[0]), float(P_[1]), float(V[0]), float(V[1]),
                                  float(R), float(tau), float(dt), int(bool(i_before_j)),
                                  *[ctypes.byref(o) for o in out])
    return code, np.array([out[0].value, out[1].value]), np.array([out[2].value, out[3].value])


def _hp(q, n):
    q = np.asarray(q, np.float64).reshape(-1, 2)
    n = np.asarray(n, np.float64).reshape(-1, 2)
    m = q.shape[0]
    arr = (HalfPlane * max(m, 1))()
    for k in range(m):
        arr[k] = HalfPlane(q[k, 0], q[k, 1], n[k, 0], n[k, 1])
    return m, arr


def project(q, n, vmax, vhat, shift=0.0):
    """argmin |v - vhat| over |v| <= vmax and n_k.(v - q_k) >= -shift; None if empty."""
    m, arr = _hp(q, n)
    ox, oy = ctypes.c_double(), ctypes.c_double()
    ok = lib().oracle_project(m, arr, float(shift), float(vmax), float(vhat[0]), float(vhat[1]),
                              ctypes.byref(ox), ctypes.byref(oy))
    return np.array([ox.value, oy.value]) if ok else None


def min_max(q, n, vmax):
    """(d*, v*) with d* = min over |v| <= vmax of max_k n_k.(q_k - v)."""
    m, arr = _hp(q, n)
    ox, oy = ctypes.c_double(), ctypes.c_double()
    d = lib().oracle_min_max(m, arr, float(vmax), ctypes.byref(ox), ctypes.byref(oy))
    return d, np.array([ox.value, oy.value])


def solve(q, n, vmax, vhat):
    """The method's velocity choice for given half-planes: (v', status, d*)."""
    v = project(q, n, vmax, vhat)
    if v is not None:
        return v, 0, float("nan")
    d, vmm = min_max(q, n, vmax)
    v2 = project(q, n, vmax, vhat, shift=d + DELTA)
    return (vmm if v2 is None else v2), 1, d


def steer(p, g, s, dt):
    ox, oy = ctypes.c_double(), ctypes.c_double()
    lib().oracle_steer(float(p[0]), float(p[1]), float(g[0]), float(g[1]), float(s), float(dt),
                       ctypes.byref(ox), ctypes.byref(oy))
    return np.array([ox.value, oy.value])


def knn_brute(pos, i, nd, k, lo=0, hi=None):
    pos = _f32(pos)
    n = pos.shape[1]
    hi = n if hi is None else hi
    ids = np.full(max(k, 1), -1, np.int64)
    d2 = np.zeros(max(k, 1), np.float32)
    m = lib().oracle_knn_brute(n, _ptr(pos), lo, hi, i, nd, k, _ptr(ids), _ptr(d2))
    return ids[:m], d2[:m]


def knn_binned(pos, nd, k, lo=0, hi=None):
    pos = _f32(pos)
    n = pos.shape[1]
    hi = n if hi is None else hi
    ids = np.full((hi - lo, k), -1, np.int64)
    lib().oracle_knn_binned_scene(n, _ptr(pos), lo, hi, nd, k, _ptr(ids))
    return ids


# ---------------------------------------------------------------- whole state

def velocities(pos, vel, pref, offsets, params, goals=None, agents=None, neighbor_mode=1,
               radius=None, max_speed=None, pref_speed=None, present=None):
    """New velocities (float64) of ``agents`` (default: all) from one state.

    radius, max_speed, pref_speed: optional per-agent values [N] in place of
    the scene's; present: optional [N] mask of agents in the simulation.
    Returns a dict with new_vel [M,2], vhat [M,2], nbr [M,kcap] (-1 padded),
    n_nbr [M], status [M] (0 = 2D LP, 1 = fallback, 2 = absent) and dstar [M].
    """
    pos, vel, pref, goals = map(_f32, (pos, vel, pref, goals))
    props, keep = _agents(radius, max_speed, pref_speed, present)
    n = pos.shape[1]
    offsets = _offsets(offsets, n, len(params))
    pa = params_array(params)
    if agents is None:
        m = n
        ag = None
    else:
        ag = np.ascontiguousarray(agents, np.int64)
        m = ag.shape[0]
    kcap = max(1, max(p.max_neighbors for p in params))
    out = dict(new_vel=np.zeros((m, 2)), vhat=np.zeros((m, 2)),
               nbr=np.full((m, kcap), -1, np.int64), n_nbr=np.zeros(m, np.int32),
               status=np.zeros(m, np.uint8), dstar=np.zeros(m))
    lib().oracle_velocities(n, _ptr(pos), _ptr(vel), _ptr(pref), _ptr(goals), props,
                            len(params), _ptr(offsets), pa, _ptr(ag), m, neighbor_mode, kcap,
                            _ptr(out["new_vel"]), _ptr(out["vhat"]), _ptr(out["nbr"]),
                            _ptr(out["n_nbr"]), _ptr(out["status"]), _ptr(out["dstar"]))
    return out


def step(pos, vel, pref, offsets, params, goals=None, n_steps=1, radius=None, max_speed=None,
         pref_speed=None):
    """Advance copies of the float32 state by ``n_steps``; returns (pos, vel, pref, status)."""
    pos = np.array(pos, np.float32, copy=True, order="C")
    vel = np.array(vel, np.float32, copy=True, order="C")
    pref = np.array(pref, np.float32, copy=True, order="C")
    goals = _f32(goals)
    ag, keep = _agents(radius, max_speed, pref_speed)
    n = pos.shape[1]
    st = np.zeros(n, np.uint8)
    lib().oracle_step(n, _ptr(pos), _ptr(vel), _ptr(pref), _ptr(goals), ag,
                      len(params), _ptr(_offsets(offsets, n, len(params))),
                      params_array(params), int(n_steps), _ptr(st))
    return pos, vel, pref, st


def life_step(pos, vel, pref, offsets, params, goals, spawn_step, state, t0, n_steps=1,
              radius=None, max_speed=None, pref_speed=None):
    """Steps t0 .. t0+n_steps-1 with spawning and removal on copies of the state.

    spawn_step [N] int32: the step at which each agent enters; state [N] uint8:
    1 = removed.  Returns (pos, vel, pref, state, status of the last step)."""
    pos = np.array(pos, np.float32, copy=True, order="C")
    vel = np.array(vel, np.float32, copy=True, order="C")
    pref = np.array(pref, np.float32, copy=True, order="C")
    state = np.array(state, np.uint8, copy=True, order="C")
    spawn = np.ascontiguousarray(spawn_step, np.int32)
    goals = _f32(goals)
    ag, keep = _agents(radius, max_speed, pref_speed)
    n = pos.shape[1]
    st = np.zeros(n, np.uint8)
    L = lib()
    if not hasattr(L, "_life_ready"):
        L.oracle_life_step.argtypes = [I64, P, P, P, P, P, I32, P, P, I32, P, P, I32, P]
        L.oracle_life_step.restype = None
        L._life_ready = True
    L.oracle_life_step(n, _ptr(pos), _ptr(vel), _ptr(pref), _ptr(goals), ag, len(params),
                       _ptr(_offsets(offsets, n, len(params))), params_array(params),
                       int(n_steps), _ptr(spawn), _ptr(state), int(t0), _ptr(st))
    return pos, vel, pref, state, st


# ---------------------------------------------------------------- gradients

def _grad_lib():
    L = lib()
    if not hasattr(L, "_grad_ready"):
        L.oracle_traj_loss.argtypes = [I64, P, P, P, I32, P, P, P, P, I32, P, P]
        L.oracle_traj_loss.restype = F64
        L.oracle_traj_jvp.argtypes = [I64, P, P, P, I32, P, P, P, P, I32, P, P, P, P, I32, P, P,
                                      P]
        L.oracle_traj_jvp.restype = None
        L.oracle_step_jvp.argtypes = [I64, P, P, P, I32, P, P, P, P, P, P, P, P, P, P]
        L.oracle_step_jvp.restype = None
        L.oracle_choice_jvp.argtypes = [ctypes.c_int] + [P] * 6 + [F64] * 13 + [P]
        L.oracle_choice_jvp.restype = ctypes.c_int
        L.oracle_traj_curve.argtypes = [I64, P, P, P, I32, P, P, P, P, I32, P, P, P, P, I32, P,
                                        P, P, P]
        L.oracle_traj_curve.restype = None
        L._grad_ready = True
    return L


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def traj_loss(pos0, vel0, pref, offsets, params, vmax, tau, n_steps, targets, radius=None,
              max_speed=None):
    """L = sum |x(T) - y|^2 after n_steps float64 steps (fixed preferred velocities).

    radius / max_speed: optional per-agent constants (a per-agent max speed
    replaces the scene's leaf vmax for that agent)."""
    pos0, vel0, pref, targets, vmax, tau = map(_f64, (pos0, vel0, pref, targets, vmax, tau))
    ag, keep = _agents(radius, max_speed, None)
    n = pos0.shape[1]
    return _grad_lib().oracle_traj_loss(n, _ptr(pos0), _ptr(vel0), _ptr(pref), len(params),
                                        _ptr(_offsets(offsets, n, len(params))),
                                        params_array(params), _ptr(vmax), _ptr(tau), int(n_steps),
                                        _ptr(targets), ag)


def traj_jvp(pos0, vel0, pref, offsets, params, vmax, tau, n_steps, targets, dpref, dvmax, dtau,
             f32_state=False, radius=None, max_speed=None):
    """(L, dL) with dL the directional derivative along (dpref, dvmax, dtau), complex step.

    f32_state rounds the primal state to float32 after every step.
    """
    pos0, vel0, pref, targets, vmax, tau, dpref, dvmax, dtau = map(
        _f64, (pos0, vel0, pref, targets, vmax, tau, dpref, dvmax, dtau))
    ag, keep = _agents(radius, max_speed, None)
    n = pos0.shape[1]
    L, dL = ctypes.c_double(), ctypes.c_double()
    _grad_lib().oracle_traj_jvp(n, _ptr(pos0), _ptr(vel0), _ptr(pref), len(params),
                                _ptr(_offsets(offsets, n, len(params))),
                                params_array(params), _ptr(vmax), _ptr(tau), int(n_steps),
                                _ptr(targets), _ptr(dpref), _ptr(dvmax), _ptr(dtau),
                                int(bool(f32_state)), ag, ctypes.byref(L), ctypes.byref(dL))
    return L.value, dL.value


def step_jvp(pos, vel, pref, offsets, params, dpos, dvel, dpref, dvmax, dtau, radius=None,
             max_speed=None):
    """Tangent (dpos', dvel') of one float64 step from the float32 state (complex step)."""
    pos, vel, pref = map(_f32, (pos, vel, pref))
    ag, keep = _agents(radius, max_speed, None)
    dpos, dvel, dpref, dvmax, dtau = map(_f64, (dpos, dvel, dpref, dvmax, dtau))
    n = pos.shape[1]
    op = np.zeros((2, n))
    ov = np.zeros((2, n))
    _grad_lib().oracle_step_jvp(n, _ptr(pos), _ptr(vel), _ptr(pref), len(params),
                                _ptr(_offsets(offsets, n, len(params))),
                                params_array(params), _ptr(dpos), _ptr(dvel), _ptr(dpref),
                                _ptr(dvmax), _ptr(dtau), ag, _ptr(op), _ptr(ov))
    return op, ov


def traj_curve(pos0, vel0, pref, offsets, params, vmax, tau, n_steps, targets, dpref=None,
               dvmax=None, dtau=None, radius=None, max_speed=None, f32_state=False):
    """A float64 trajectory step by step: (loss after each step [n_steps],
    directional derivative of that loss along (dpref, dvmax, dtau) [n_steps]
    (zeros without a tangent), hash of each step's discrete decisions
    [n_steps] uint64).  With a tangent the run is a complex step; the
    decisions are the primal's either way.  f32_state rounds the primal state
    to float32 after every step."""
    pos0, vel0, pref, targets, vmax, tau, dpref, dvmax, dtau = map(
        _f64, (pos0, vel0, pref, targets, vmax, tau, dpref, dvmax, dtau))
    ag, keep = _agents(radius, max_speed, None)
    n = pos0.shape[1]
    loss = np.zeros(n_steps)
    dloss = np.zeros(n_steps)
    tape = np.zeros(n_steps, np.uint64)
    _grad_lib().oracle_traj_curve(n, _ptr(pos0), _ptr(vel0), _ptr(pref), len(params),
                                  _ptr(_offsets(offsets, n, len(params))), params_array(params),
                                  _ptr(vmax), _ptr(tau), int(n_steps), _ptr(targets),
                                  _ptr(dpref), _ptr(dvmax), _ptr(dtau), int(bool(f32_state)),
                                  ag, _ptr(loss), _ptr(dloss), _ptr(tape))
    return loss, dloss, tape
