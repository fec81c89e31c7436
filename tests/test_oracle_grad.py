"""Pins of the reference's forward-mode derivatives (complex step).

Complex step carries i*h*tangent through the float64 reference with every
decision on real parts, so its imaginary part is the exact directional
derivative of the piecewise-smooth map with the primal's discrete choices.
It is pinned against central finite differences of the plain float64
reference: a direction is counted only where two FD step sizes agree (no
neighbour set, half-plane branch or active constraint switches inside the
FD interval).
"""
import numpy as np
import pytest

from paper_1908_10107_amd import scenes


def small_grad_scene(seed, n=96, side=10.0):
    w = scenes.grad(n=n, density=n / side ** 2, seed=seed)
    return w


@pytest.mark.parametrize("seed", range(3))
def test_trajectory_jvp_matches_central_differences(oracle_lib, seed):
    w = small_grad_scene(300 + seed)
    rng = np.random.default_rng(seed)
    steps = 12
    vmax = np.array([w.params[0].max_speed], float)
    tau = np.array([w.params[0].time_horizon], float)
    pos0 = w.pos.astype(np.float64)
    vel0 = w.vel.astype(np.float64)
    pref = w.pref_vel.astype(np.float64)
    counted = 0
    for d in range(10):
        dp = rng.normal(size=pref.shape)
        dv = rng.normal(size=1) * (d % 2)
        dt_ = rng.normal(size=1) * ((d + 1) % 2)
        L, dL = oracle_lib.traj_jvp(pos0, vel0, pref, w.offsets, w.params, vmax, tau, steps,
                                    w.targets, dp, dv, dt_)
        f = lambda eps: oracle_lib.traj_loss(pos0, vel0, pref + eps * dp, w.offsets, w.params,
                                             vmax + eps * dv, tau + eps * dt_, steps, w.targets)
        assert abs(f(0.0) - L) <= 1e-12 * max(1.0, abs(L))
        fd1 = (f(1e-6) - f(-1e-6)) / 2e-6
        fd2 = (f(5e-7) - f(-5e-7)) / 1e-6
        if abs(fd1 - fd2) > 1e-4 * max(1.0, abs(fd1)):
            continue  # a discrete switch inside the interval
        counted += 1
        assert abs(dL - fd1) <= 1e-3 * max(1.0, abs(fd1)), (d, dL, fd1, fd2)
    assert counted >= 3


def test_single_agent_jvp_matches_central_differences(oracle_lib):
    import ctypes
    L = oracle_lib._grad_lib()
    rng = np.random.default_rng(5)
    p = lambda a: a.ctypes.data
    checked = 0
    for trial in range(300):
        m = int(rng.integers(1, 12))
        P = rng.normal(size=(m, 2)) * 2.5
        V = rng.normal(size=(m, 2))
        first = np.ascontiguousarray((rng.random(m) < 0.5).astype(np.int32))
        Rs = np.full(m, 0.5)
        vi, vh = rng.normal(size=2) * 0.8, rng.normal(size=2) * 1.3
        tau, vmax = 5.0, 1.5
        dP, dV = rng.normal(size=(m, 2)), rng.normal(size=(m, 2))
        dvi, dvh = rng.normal(size=2), rng.normal(size=2)
        dvm, dta = rng.normal(), rng.normal()

        def run(eps, tang=True):
            out = np.zeros(6)
            Pc = np.ascontiguousarray(P + eps * dP)
            Vc = np.ascontiguousarray(V + eps * dV)
            z = np.zeros((m, 2))
            L.oracle_choice_jvp(m, p(Pc), p(dP if tang else z), p(Vc), p(dV if tang else z),
                                p(Rs), p(first), vi[0] + eps * dvi[0], vi[1] + eps * dvi[1],
                                dvi[0], dvi[1], tau + eps * dta, dta, 0.1, vmax + eps * dvm, dvm,
                                vh[0] + eps * dvh[0], vh[1] + eps * dvh[1], dvh[0], dvh[1], p(out))
            return out
        base = run(0.0)
        fd1 = (run(1e-6)[:2] - run(-1e-6)[:2]) / 2e-6
        fd2 = (run(5e-7)[:2] - run(-5e-7)[:2]) / 1e-6
        if np.abs(fd1 - fd2).max() > 1e-5 * max(1.0, np.abs(fd1).max()):
            continue
        checked += 1
        np.testing.assert_allclose(base[2:4], fd1, rtol=1e-4, atol=1e-6)
    assert checked > 200


@pytest.mark.parametrize("seed", range(2))
def test_f32_state_jvp(oracle_lib, seed):
    """The float32-state branch of the trajectory derivative (the trajectory a
    float32 state takes, the rounding differentiated as the identity).

    - Its primal loss equals the loss of the float32 stepper that the step
      parity uses (a separate driver: x <- f32(x + dt v'), v <- f32(v') with
      fixed preferred velocities), to float64 rounding.
    - On a short horizon, where the float32 and float64 trajectories stay
      within rounding of each other and no discrete choice switches, its
      derivative equals the float64-state derivative to 1e-5 of the size the
      derivative can reach, 2 sqrt(L) |x'| with |x'| <= steps * dt * |delta|
      (dL sums 2N terms of both signs, so the gap is set by their size, not by
      their sum; the float32 state is rounded by about 1e-6 m a step and the
      tangent moves with the state it is taken at), and central differences
      of the float64 loss to 1e-3.
    """
    w = small_grad_scene(310 + seed)
    rng = np.random.default_rng(40 + seed)
    steps = 6
    p = w.params[0]
    vmax = np.array([np.float32(p.max_speed)], float)
    tau = np.array([np.float32(p.time_horizon)], float)
    pos0 = w.pos.astype(np.float64)
    vel0 = w.vel.astype(np.float64)
    pref = w.pref_vel.astype(np.float64)
    x, v, _, _ = oracle_lib.step(w.pos, w.vel, w.pref_vel, w.offsets, w.params, n_steps=steps)
    want = float(((x.astype(np.float64) - w.targets) ** 2).sum())
    counted = 0
    for d in range(8):
        dp = rng.normal(size=pref.shape)
        dv = rng.normal(size=1) * (d % 2)
        dt_ = rng.normal(size=1) * ((d + 1) % 2)
        L32, dL32 = oracle_lib.traj_jvp(pos0, vel0, pref, w.offsets, w.params, vmax, tau, steps,
                                        w.targets, dp, dv, dt_, f32_state=True)
        L64, dL64 = oracle_lib.traj_jvp(pos0, vel0, pref, w.offsets, w.params, vmax, tau, steps,
                                        w.targets, dp, dv, dt_, f32_state=False)
        assert abs(L32 - want) <= 1e-12 * abs(want), (L32, want)
        assert abs(L32 - L64) <= 1e-5 * abs(L64)   # the two trajectories stay close
        f = lambda eps: oracle_lib.traj_loss(pos0, vel0, pref + eps * dp, w.offsets, w.params,
                                             vmax + eps * dv, tau + eps * dt_, steps, w.targets)
        fd1 = (f(1e-6) - f(-1e-6)) / 2e-6
        fd2 = (f(5e-7) - f(-5e-7)) / 1e-6
        if abs(fd1 - fd2) > 1e-4 * max(1.0, abs(fd1)):
            continue  # a discrete switch inside the interval
        counted += 1
        size = 2.0 * np.sqrt(L64) * steps * p.dt * np.sqrt((dp ** 2).sum() + dv @ dv + dt_ @ dt_)
        assert abs(dL32 - dL64) <= 1e-5 * size, (d, dL32, dL64, size)
        assert abs(dL32 - fd1) <= 1e-3 * max(1.0, abs(fd1)), (d, dL32, fd1)
    assert counted >= 3


def test_f32_state_curve(oracle_lib):
    """The float32-state branch of the per-step trajectory curve: after each
    step its loss equals that of the float32 stepper the step parity uses
    (a separate driver, one step at a time), its tangent equals the
    float32-state trajectory derivative, and its decision hashes equal the
    float64 curve's while the two paths take the same decisions (the first
    step always does: both start from the same state)."""
    w = small_grad_scene(330)
    rng = np.random.default_rng(50)
    steps = 5
    p = w.params[0]
    vmax = np.array([np.float32(p.max_speed)], float)
    tau = np.array([np.float32(p.time_horizon)], float)
    pos0, vel0 = w.pos.astype(np.float64), w.vel.astype(np.float64)
    pref = w.pref_vel.astype(np.float64)
    dp = rng.normal(size=pref.shape)
    L, dL, tape32 = oracle_lib.traj_curve(pos0, vel0, pref, w.offsets, w.params, vmax, tau, steps,
                                          w.targets, dpref=dp, dvmax=np.zeros(1),
                                          dtau=np.zeros(1), f32_state=True)
    Lp, _, tape32p = oracle_lib.traj_curve(pos0, vel0, pref, w.offsets, w.params, vmax, tau,
                                           steps, w.targets, f32_state=True)
    _, _, tape64 = oracle_lib.traj_curve(pos0, vel0, pref, w.offsets, w.params, vmax, tau, steps,
                                         w.targets)
    assert np.array_equal(tape32, tape32p)      # the tangent run takes the primal's decisions
    assert np.allclose(L, Lp, rtol=1e-12, atol=0)
    assert tape32[0] == tape64[0]
    x, v = w.pos, w.vel
    for t in range(steps):
        x, v, _, _ = oracle_lib.step(x, v, w.pref_vel, w.offsets, w.params)
        want = float(((x.astype(np.float64) - w.targets) ** 2).sum())
        assert abs(L[t] - want) <= 1e-12 * abs(want), (t, L[t], want)
    _, dL_jvp = oracle_lib.traj_jvp(pos0, vel0, pref, w.offsets, w.params, vmax, tau, steps,
                                    w.targets, dp, np.zeros(1), np.zeros(1), f32_state=True)
    assert abs(dL[-1] - dL_jvp) <= 1e-9 * max(1.0, abs(dL_jvp))
