"""Finite-difference check of the trajectory derivative at full size: 4,096
agents at 1 /m^2 (fixed preferred velocities, loss = sum |x(T) - y|^2), 200
steps, float64 state.

Central differences with h = 1e-4 along 16 random unit directions in
theta = (preferred velocities, v_max, tau) and along v_max and tau alone.  The
step is piecewise smooth (neighbour sets, half-plane branches, the winning
candidate of each program); the reference records every decision of every
step, and a direction counts at horizon T only while the decisions at
theta + h delta and theta - h delta equal those at theta for all steps
before T.  Counted directions must agree with the forward-mode derivative
(complex step along the primal's branch) to 1e-3: the plain difference at
h = 1e-4 where its truncation error allows, and the Richardson combination of
h and h / 2 (truncation O(h^4); the h / 2 decisions must match too) at every
counted horizon.  The test prints the table of counts, errors and derivative
sizes by horizon.
"""
import numpy as np
import pytest

from paper_1908_10107_amd import scenes

H = 1e-4
HORIZONS = [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 20, 50, 100, 200]
SHORT = 12  # steps run at h / 2 (no direction has counted beyond 8)


def directions(n_pref, seed):
    rng = np.random.default_rng(seed)
    out = []
    for d in range(16):
        v = rng.normal(size=n_pref + 2)
        v /= np.linalg.norm(v)
        out.append(("rand%d" % d, v[:-2], v[-2:-1], v[-1:]))
    out.append(("vmax", np.zeros(n_pref), np.ones(1), np.zeros(1)))
    out.append(("tau", np.zeros(n_pref), np.zeros(1), np.ones(1)))
    return out


@pytest.mark.slow
def test_config4_central_differences_with_switch_detection(oracle_lib):
    w = scenes.grad()
    p = w.params[0]
    steps = w.steps
    assert (w.n, steps) == (4096, 200)
    vmax = np.array([np.float32(p.max_speed)], float)
    tau = np.array([np.float32(p.time_horizon)], float)
    pos0, vel0 = w.pos.astype(np.float64), w.vel.astype(np.float64)
    pref = w.pref_vel.astype(np.float64)
    curve = lambda pr, vm, ta, n, **t: oracle_lib.traj_curve(
        pos0, vel0, pr, w.offsets, w.params, vm, ta, n, w.targets, **t)
    L0, _, tape0 = curve(pref, vmax, tau, steps)
    rows = []
    for name, dp, dv, dt_ in directions(pref.size, scenes.BASE_SEED + 4):
        dp = dp.reshape(pref.shape)
        _, fm, tape_fm = curve(pref, vmax, tau, steps, dpref=dp, dvmax=dv, dtau=dt_)
        assert np.array_equal(tape_fm, tape0)   # the tangent run takes the primal's decisions
        Lp, _, tp = curve(pref + H * dp, vmax + H * dv, tau + H * dt_, steps)
        Lm, _, tm = curve(pref - H * dp, vmax - H * dv, tau - H * dt_, steps)
        Lp2, _, tp2 = curve(pref + H / 2 * dp, vmax + H / 2 * dv, tau + H / 2 * dt_, SHORT)
        Lm2, _, tm2 = curve(pref - H / 2 * dp, vmax - H / 2 * dv, tau - H / 2 * dt_, SHORT)
        same = (tp == tape0) & (tm == tape0)
        same2 = (tp2 == tape0[:SHORT]) & (tm2 == tape0[:SHORT])
        clean = int(np.argmin(same)) if not same.all() else steps       # steps before a switch
        clean2 = int(np.argmin(same2)) if not same2.all() else SHORT
        fd = (Lp - Lm) / (2 * H)
        fd2 = (Lp2 - Lm2) / H
        rows.append(dict(name=name, clean=clean, clean2=clean2, fm=fm, fd=fd, fd2=fd2))
    rel = lambda a, b: abs(a - b) / max(abs(b), 1e-300)
    print("\nhorizon | counted /18 | max rel err FD(h=1e-4) | max rel err Richardson | "
          "median |dL/d delta| (forward mode)")
    table = {}
    for T in HORIZONS:
        t = T - 1
        counted = [r for r in rows if r["clean"] >= T]
        e_fd = max([rel(r["fd"][t], r["fm"][t]) for r in counted], default=float("nan"))
        rich = [r for r in counted if T <= SHORT and r["clean2"] >= T]
        e_r = max([rel((4 * r["fd2"][t] - r["fd"][t]) / 3, r["fm"][t]) for r in rich],
                  default=float("nan"))
        mag = float(np.median([abs(r["fm"][t]) for r in rows]))
        table[T] = (len(counted), e_fd, e_r, mag)
        print("%7d | %11d | %22.2e | %22.2e | %.3g" % (T, len(counted), e_fd, e_r, mag))
        # every counted direction agrees with the forward mode to 1e-3
        for r in rich:
            assert rel((4 * r["fd2"][t] - r["fd"][t]) / 3, r["fm"][t]) <= 1e-3, (r["name"], T)
        if T <= 2:
            for r in counted:
                assert rel(r["fd"][t], r["fm"][t]) <= 1e-3, (r["name"], T)
        assert len(rich) == len(counted) or T > SHORT
    half = max([T for T in HORIZONS if table[T][0] >= 9], default=0)
    print("longest horizon with at least half of the directions counted: %d steps" % half)
    assert table[1][0] == 18      # one step: no decision switches at h = 1e-4
    assert half >= 5
