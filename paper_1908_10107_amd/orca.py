"""Python binding of liborca (include/orca.h): argument marshalling only.

Every array is a float32 CUDA (HIP) tensor of shape [2, N] (row 0 = x, row 1 =
y).  Work is enqueued on torch's current stream of the tensors' device.  There
is no CPU path: calls raise if the library is missing or a tensor is not on
the GPU.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Iterable, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liborca.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "orca.h")

OK, EINVAL, ENOMEM, ECAPACITY, ESTATE, EHIP = 0, -1, -2, -3, -4, -5
K_LIMIT = 32
PROF_STAGES = 4
STAGE_NAMES = ("binning", "neighbours", "halfplanes_lp2d", "fallback_lp3d")
_NAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", ECAPACITY: "ECAPACITY", ESTATE: "ESTATE",
          EHIP: "EHIP"}


class OrcaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_NAMES.get(code, "?"), code, msg))
        self.code = code


class OrcaParams(ctypes.Structure):
    _fields_ = [("radius", ctypes.c_float), ("max_speed", ctypes.c_float),
                ("neighbor_dist", ctypes.c_float), ("time_horizon", ctypes.c_float),
                ("dt", ctypes.c_float), ("pref_speed", ctypes.c_float),
                ("max_neighbors", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None
_P = ctypes.c_void_p


def header_symbols() -> list:
    """Names of the functions include/orca.h declares."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(orca_[a-z_]+)\s*\(", text)))


def load(path: str = LIB_PATH):
    """Load liborca.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("liborca.so is not built (%s); run __graft_entry__.build()" % path)
    L = ctypes.CDLL(path)
    L.orca_create.argtypes = [ctypes.POINTER(_P), ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                              ctypes.c_int32, _P]
    L.orca_create.restype = ctypes.c_int
    L.orca_destroy.argtypes = [_P]
    L.orca_destroy.restype = None
    L.orca_last_error.argtypes = [_P]
    L.orca_last_error.restype = ctypes.c_char_p
    L.orca_set_stream.argtypes = [_P, _P]
    L.orca_set_stream.restype = ctypes.c_int
    L.orca_build_grid.argtypes = [_P, ctypes.c_int32, _P, _P, _P]
    L.orca_build_grid.restype = ctypes.c_int
    L.orca_compute_velocities.argtypes = [_P] + [_P] * 7
    L.orca_compute_velocities.restype = ctypes.c_int
    L.orca_step.argtypes = [_P, ctypes.c_int32, _P, _P, _P, _P, _P, _P, ctypes.c_int32,
                            ctypes.c_int32]
    L.orca_step.restype = ctypes.c_int
    L.orca_backward.argtypes = [_P, ctypes.c_int32] + [_P] * 7
    L.orca_backward.restype = ctypes.c_int
    L.orca_backward_steps.argtypes = [_P, ctypes.c_int32, ctypes.c_int32] + [_P] * 7
    L.orca_backward_steps.restype = ctypes.c_int
    L.orca_step_graph.argtypes = [_P, ctypes.c_int32, _P, _P, _P, _P, _P, _P, ctypes.c_int32]
    L.orca_step_graph.restype = ctypes.c_int
    L.orca_autotune.argtypes = [_P, _P, _P, _P, _P, _P, ctypes.c_int32, _P]
    L.orca_autotune.restype = ctypes.c_int
    L.orca_set_launch.argtypes = [_P, ctypes.c_int32, ctypes.c_int32]
    L.orca_set_launch.restype = ctypes.c_int
    L.orca_set_kernels.argtypes = [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.orca_set_kernels.restype = ctypes.c_int
    L.orca_set_agents.argtypes = [_P, _P, _P, _P]
    L.orca_set_agents.restype = ctypes.c_int
    L.orca_set_lifecycle.argtypes = [_P, _P, _P, ctypes.c_int32]
    L.orca_set_lifecycle.restype = ctypes.c_int
    L.orca_population.argtypes = [_P, _P, _P, _P]
    L.orca_population.restype = ctypes.c_int
    L.orca_profile.argtypes = [_P, ctypes.c_int32]
    L.orca_profile.restype = ctypes.c_int
    L.orca_profile_read.argtypes = [_P, _P, _P, _P]
    L.orca_profile_read.restype = ctypes.c_int
    L.orca_step_noalloc.argtypes = [ctypes.c_int64, _P, _P, _P, _P, _P, ctypes.c_int32, _P, _P,
                                    ctypes.c_int32]
    L.orca_step_noalloc.restype = ctypes.c_int
    _lib = L
    return L


def params_array(params: Sequence) -> ctypes.Array:
    arr = (OrcaParams * len(params))()
    for s, p in enumerate(params):
        arr[s] = OrcaParams(p.radius, p.max_speed, p.neighbor_dist, p.time_horizon, p.dt,
                            p.pref_speed, int(p.max_neighbors), 0)
    return arr


def _dev_ptr(t, what, n=None, shape2=True):
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % what)
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError("%s must be contiguous float32" % what)
    if shape2 and (t.dim() != 2 or t.shape[0] != 2 or (n is not None and t.shape[1] != n)):
        raise ValueError("%s must have shape [2, %s], got %s" % (what, n, tuple(t.shape)))
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """An orca_ctx: all scratch for up to ``max_agents`` agents in ``max_scenes`` scenes."""

    def __init__(self, max_agents: int, max_scenes: int = 1, k_max: int = 16,
                 tape_steps: int = 0, device=None):
        import torch
        self._torch = torch
        self.lib = load()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            h = ctypes.c_void_p()
            rc = self.lib.orca_create(ctypes.byref(h), int(max_agents), int(max_scenes),
                                      int(k_max), int(tape_steps), ctypes.c_void_p(stream))
        if rc != OK:
            raise OrcaError(rc, "orca_create(max_agents=%d, max_scenes=%d, k_max=%d)"
                            % (max_agents, max_scenes, k_max))
        self.h = h
        self.max_agents = max_agents
        self._scenes = None
        # counts orca_step calls: a recording is still the last thing the
        # context did while this has not moved on
        self.step_epoch = 0

    # ----------------------------------------------------------- plumbing
    def _check(self, rc):
        if rc != OK:
            raise OrcaError(rc, self.lib.orca_last_error(self.h).decode())

    def _sync_stream(self):
        s = self._torch.cuda.current_stream(self.device).cuda_stream
        self._check(self.lib.orca_set_stream(self.h, ctypes.c_void_p(s)))

    def _scene_args(self, offsets, params):
        offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        key = (offs.tobytes(), tuple((p.radius, p.max_speed, p.neighbor_dist, p.time_horizon,
                                      p.dt, p.pref_speed, p.max_neighbors) for p in params))
        if self._scenes is None or self._scenes[0] != key:
            self._scenes = (key, offs, params_array(params))
        _, offs, pa = self._scenes
        return len(params), offs, pa, int(offs[-1])

    # ----------------------------------------------------------- entry points
    def build_grid(self, offsets, params, pos):
        ns, offs, pa, n = self._scene_args(offsets, params)
        self._sync_stream()
        self._check(self.lib.orca_build_grid(self.h, ns, offs.ctypes.data_as(_P), pa,
                                             _dev_ptr(pos, "pos", n)))

    def compute_velocities(self, pos, vel, pref_vel=None, goals=None, new_vel=None,
                           nbr_out=None, lp_status=None):
        n = pos.shape[1]
        torch = self._torch
        if new_vel is None:
            new_vel = torch.empty_like(pos)
        if nbr_out is not None and (not nbr_out.is_cuda or nbr_out.dtype != torch.int32
                                    or not nbr_out.is_contiguous()):
            raise TypeError("nbr_out must be contiguous int32 on the GPU")
        if lp_status is not None and (not lp_status.is_cuda or lp_status.dtype != torch.uint8):
            raise TypeError("lp_status must be uint8 on the GPU")
        self._sync_stream()
        self._check(self.lib.orca_compute_velocities(
            self.h, _dev_ptr(pos, "pos", n), _dev_ptr(vel, "vel", n),
            _dev_ptr(pref_vel, "pref_vel", n), _dev_ptr(goals, "goals", n),
            _dev_ptr(new_vel, "new_vel", n),
            None if nbr_out is None else ctypes.c_void_p(nbr_out.data_ptr()),
            None if lp_status is None else ctypes.c_void_p(lp_status.data_ptr())))
        return new_vel

    def step(self, offsets, params, pos, vel, pref_vel, goals=None, n_steps=1, save_tape=False):
        ns, offs, pa, n = self._scene_args(offsets, params)
        self._sync_stream()
        self.step_epoch += 1
        self._check(self.lib.orca_step(self.h, ns, offs.ctypes.data_as(_P), pa,
                                       _dev_ptr(pos, "pos", n), _dev_ptr(vel, "vel", n),
                                       _dev_ptr(pref_vel, "pref_vel", n),
                                       _dev_ptr(goals, "goals", n), int(n_steps),
                                       int(bool(save_tape))))

    def step_graph(self, offsets, params, pos, vel, pref_vel, goals=None, n_steps=1):
        """orca_step replayed from a captured HIP graph (see orca_step_graph)."""
        ns, offs, pa, n = self._scene_args(offsets, params)
        self._sync_stream()
        self._check(self.lib.orca_step_graph(self.h, ns, offs.ctypes.data_as(_P), pa,
                                             _dev_ptr(pos, "pos", n), _dev_ptr(vel, "vel", n),
                                             _dev_ptr(pref_vel, "pref_vel", n),
                                             _dev_ptr(goals, "goals", n), int(n_steps)))

    def autotune(self, pos, vel, pref_vel=None, goals=None, reps=3):
        """Pick launch shapes on the current grid; returns (knn_block,
        fallback_waves_per_cu, agents_per_lane (0: split velocity kernels),
        velocity_waves_per_cu, fallback_work_units)."""
        n = pos.shape[1]
        scratch = self._torch.empty_like(pos)
        choice = (ctypes.c_int32 * 5)()
        self._sync_stream()
        self._check(self.lib.orca_autotune(self.h, _dev_ptr(pos, "pos", n), _dev_ptr(vel, "vel", n),
                                           _dev_ptr(pref_vel, "pref_vel", n),
                                           _dev_ptr(goals, "goals", n), _dev_ptr(scratch, "new_vel", n),
                                           int(reps), choice))
        return tuple(choice)

    def set_agents(self, radius=None, max_speed=None, pref_speed=None):
        """Per-agent radius / max speed / walking speed ([N] float32 CUDA tensors, each
        optional) for the following calls (see orca_set_agents).  The tensors are
        kept referenced here; pass nothing to return to the scene values."""
        ptrs = []
        for t, nm in ((radius, "radius"), (max_speed, "max_speed"), (pref_speed, "pref_speed")):
            if t is None:
                ptrs.append(None)
                continue
            if not (t.is_cuda and t.dtype == self._torch.float32 and t.dim() == 1 and
                    t.is_contiguous()):
                raise TypeError("%s must be a contiguous 1-D float32 CUDA tensor" % nm)
            ptrs.append(ctypes.c_void_p(t.data_ptr()))
        self._sync_stream()
        self._check(self.lib.orca_set_agents(self.h, *ptrs))
        self._agents = (radius, max_speed, pref_speed)

    def set_lifecycle(self, spawn_step=None, state=None, t0=0):
        """Spawning and removal (see orca_set_lifecycle): spawn_step [N] int32 and
        state [N] uint8 CUDA tensors (state is updated in place), step index t0.
        Pass nothing to turn it off.  The tensors are kept referenced here."""
        ptrs = []
        for t, nm, dt in ((spawn_step, "spawn_step", self._torch.int32),
                          (state, "state", self._torch.uint8)):
            if t is None:
                ptrs.append(None)
                continue
            if not (t.is_cuda and t.dtype == dt and t.dim() == 1 and t.is_contiguous()):
                raise TypeError("%s must be a contiguous 1-D %s CUDA tensor" % (nm, dt))
            ptrs.append(ctypes.c_void_p(t.data_ptr()))
        self._sync_stream()
        self._check(self.lib.orca_set_lifecycle(self.h, ptrs[0], ptrs[1], int(t0)))
        self._life = (spawn_step, state)

    def population(self):
        """(step, present, removed) from the device counters (see orca_population)."""
        st = ctypes.c_int32()
        pr, rm = ctypes.c_int64(), ctypes.c_int64()
        self._sync_stream()
        self._check(self.lib.orca_population(self.h, ctypes.byref(st), ctypes.byref(pr),
                                             ctypes.byref(rm)))
        return st.value, pr.value, rm.value

    def set_launch(self, knn_block, fallback_waves_per_cu):
        """Fix the launch shapes that autotune would pick (see orca_set_launch)."""
        self._check(self.lib.orca_set_launch(self.h, int(knn_block), int(fallback_waves_per_cu)))

    def set_kernels(self, agents_per_lane=0, velocity_waves_per_cu=12, fallback_work_units=0):
        """Kernel variants (see orca_set_kernels): agents_per_lane 0 = split
        neighbour and LP kernels, 1/2/4 = the fused persistent velocity kernel;
        fallback_work_units 1 = the fallback with work units."""
        self._check(self.lib.orca_set_kernels(self.h, int(agents_per_lane),
                                              int(velocity_waves_per_cu),
                                              int(fallback_work_units)))

    def backward(self, tape_step, g_pos_next, g_vel_next, g_pos, g_vel, g_pref_vel,
                 g_max_speed=None, g_time_horizon=None):
        """Adjoint of recorded step tape_step (see orca_backward): writes g_pos, g_vel,
        adds to g_pref_vel, g_max_speed [n_scenes], g_time_horizon [n_scenes]."""
        n = g_pos.shape[1]
        for t, nm in ((g_pos_next, "g_pos_next"), (g_vel_next, "g_vel_next"), (g_pos, "g_pos"),
                      (g_vel, "g_vel"), (g_pref_vel, "g_pref_vel")):
            _dev_ptr(t, nm, n)
        for t, nm in ((g_max_speed, "g_max_speed"), (g_time_horizon, "g_time_horizon")):
            if t is not None:
                _dev_ptr(t, nm, shape2=False)
        self._sync_stream()
        ptr = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
        self._check(self.lib.orca_backward(self.h, int(tape_step), ptr(g_pos_next),
                                           ptr(g_vel_next), ptr(g_pos), ptr(g_vel),
                                           ptr(g_pref_vel), ptr(g_max_speed),
                                           ptr(g_time_horizon)))

    def backward_steps(self, first, last, g_pos_next, g_vel_next, g_pos, g_vel, g_pref_vel,
                       g_max_speed=None, g_time_horizon=None):
        """Adjoint of recorded steps last .. first (see orca_backward_steps)."""
        n = g_pos.shape[1]
        for t, nm in ((g_pos_next, "g_pos_next"), (g_vel_next, "g_vel_next"), (g_pos, "g_pos"),
                      (g_vel, "g_vel"), (g_pref_vel, "g_pref_vel")):
            _dev_ptr(t, nm, n)
        for t, nm in ((g_max_speed, "g_max_speed"), (g_time_horizon, "g_time_horizon")):
            if t is not None:
                _dev_ptr(t, nm, shape2=False)
        self._sync_stream()
        ptr = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
        self._check(self.lib.orca_backward_steps(self.h, int(first), int(last), ptr(g_pos_next),
                                                 ptr(g_vel_next), ptr(g_pos), ptr(g_vel),
                                                 ptr(g_pref_vel), ptr(g_max_speed),
                                                 ptr(g_time_horizon)))

    def profile(self, enable):
        """Per-stage HIP-event timing (see orca_profile): 0/False stops, 1/True
        starts with every pass waiting for its stream, 2 starts without waiting
        (profile_read then waits); starting clears the sums."""
        mode = int(enable) if not isinstance(enable, bool) else int(enable)
        self._check(self.lib.orca_profile(self.h, mode))

    def profile_read(self):
        """(stage_ms[4] summed, passes, fallback agents summed); see orca_profile_read."""
        ms = (ctypes.c_double * PROF_STAGES)()
        passes, fb = ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.orca_profile_read(self.h, ms, ctypes.byref(passes),
                                               ctypes.byref(fb)))
        return list(ms), passes.value, fb.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.orca_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


NOALLOC_MAX_AGENTS = 16384
NOALLOC_MAX_NEIGHBORS = 16


def step_noalloc(params, pos, vel, pref_vel, goals=None, n_steps=1):
    """orca_step_noalloc: n_steps of one scene (params: one scenes.SceneParams)
    on torch's current stream, with the library's static scratch array instead
    of a context (see include/orca.h for its limits)."""
    import torch
    lib = load()
    n = pos.shape[1]
    pa = params_array([params])
    err = ctypes.create_string_buffer(512)
    stream = torch.cuda.current_stream(pos.device).cuda_stream
    with torch.cuda.device(pos.device):
        rc = lib.orca_step_noalloc(int(n), pa, _dev_ptr(pos, "pos", n), _dev_ptr(vel, "vel", n),
                                   _dev_ptr(pref_vel, "pref_vel", n), _dev_ptr(goals, "goals", n),
                                   int(n_steps), ctypes.c_void_p(stream), err, len(err))
    if rc != OK:
        raise OrcaError(rc, err.value.decode())


def to_device(w, device="cuda"):
    """Copy a scenes.Workload's arrays into float32 GPU tensors (dict)."""
    import torch
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(device)
    return dict(pos=t(w.pos), vel=t(w.vel), pref_vel=t(w.pref_vel), goals=t(w.goals),
                radius=t(getattr(w, "radius", None)), max_speed=t(getattr(w, "max_speed", None)),
                pref_speed=t(getattr(w, "pref_speed", None)),
                spawn_step=t(getattr(w, "spawn_step", None)))
