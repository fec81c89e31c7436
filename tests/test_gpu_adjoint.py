"""Adjoint of the GPU step against the reference's forward mode.

  * per step: <gbar, J delta> from the reference's complex-step tangent of one
    step equals <J^T gbar, delta> from orca_backward, from the same float32
    state (dot-product test), for position, velocity, preferred velocity,
    max speed and time horizon;
  * recording a step does not change it;
  * a whole trajectory (4,096 agents, 200 steps, checkpoints every 20
    steps): the gradient of L = sum |x(T) - y|^2 through OrcaTrajectory
    against the reference's forward-mode derivative of the same float32-state
    trajectory along random directions and along max speed and time horizon,
    within 1e-3 relative.  (The forward mode itself is pinned against
    central finite differences of the float64 reference in
    test_oracle_grad.py.)
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1908_10107_amd import scenes

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def moving_scene(n, density, seed, **over):
    """Uniform square with random current velocities and fixed preferred ones."""
    w = scenes.grad(n=n, density=density, seed=seed, **over)
    rng = np.random.default_rng(seed + 7)
    w.vel = np.ascontiguousarray((rng.normal(size=(2, n)) * 0.7).astype(np.float32))
    return w


@pytest.mark.parametrize("case", ["moderate", "dense", "hetero"])
def test_step_vjp_dot_product(case):
    torch = _torch()
    from paper_1908_10107_amd import orca
    say("case step vjp", case)
    w = moving_scene(3000, 2.5, 42) if case == "dense" else moving_scene(3000, 1.0, 41)
    if case == "hetero":
        # per-agent radii and max speeds (section 4), constants of the step
        rng = np.random.default_rng(43)
        w.radius = rng.choice(np.array([0.1, 0.25, 0.5], np.float32), w.n)
        w.max_speed = rng.uniform(0.8, 2.0, w.n).astype(np.float32)
    d = orca.to_device(w)
    k = w.params[0].max_neighbors
    ctx = orca.Context(max_agents=w.n, max_scenes=1, k_max=k, tape_steps=1)
    ctx.set_agents(d["radius"], d["max_speed"])
    p1, v1 = d["pos"].clone(), d["vel"].clone()
    ctx.step(w.offsets, w.params, p1, v1, d["pref_vel"], n_steps=1, save_tape=True)
    p2, v2 = d["pos"].clone(), d["vel"].clone()
    ctx.step(w.offsets, w.params, p2, v2, d["pref_vel"], n_steps=1)
    torch.cuda.synchronize()
    assert torch.equal(p1, p2) and torch.equal(v1, v2)
    rng = np.random.default_rng(3)
    for trial in range(3):
        gxn = rng.normal(size=(2, w.n)).astype(np.float32)
        gvn = rng.normal(size=(2, w.n)).astype(np.float32)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        gx, gv = torch.zeros_like(d["pos"]), torch.zeros_like(d["pos"])
        gp = torch.zeros_like(d["pos"])
        gvm = torch.zeros(1, device="cuda")
        gta = torch.zeros(1, device="cuda")
        ctx.backward(0, t(gxn), t(gvn), gx, gv, gp, gvm, gta)
        torch.cuda.synchronize()
        dpos, dvel, dpref = (rng.normal(size=(2, w.n)) for _ in range(3))
        dvm, dta = rng.normal(size=1), rng.normal(size=1)
        if trial == 1:
            dpos[:] = 0.0
            dvel[:] = 0.0   # parameters only
        jp, jv = oracle.step_jvp(w.pos, w.vel, w.pref_vel, w.offsets, w.params, dpos, dvel,
                                 dpref, dvm, dta, radius=w.radius, max_speed=w.max_speed)
        lhs = float((gxn.astype(np.float64) * jp).sum() + (gvn.astype(np.float64) * jv).sum())
        G = lambda a: a.cpu().numpy().astype(np.float64)
        rhs = float((G(gx) * dpos).sum() + (G(gv) * dvel).sum() + (G(gp) * dpref).sum()
                    + G(gvm)[0] * dvm[0] + G(gta)[0] * dta[0])
        say("  dot test %s trial %d: <g, J d> = %.9g, <J^T g, d> = %.9g" % (case, trial, lhs, rhs))
        assert abs(lhs - rhs) <= 1e-5 * (abs(lhs) + abs(rhs)) + 1e-6, (lhs, rhs)
    ctx.close()


def test_trajectory_gradient_200_steps():
    torch = _torch()
    from paper_1908_10107_amd import autograd, orca
    say("case trajectory gradient 4096 x 200")
    w = scenes.grad()
    d = orca.to_device(w)
    p = w.params[0]
    pref = d["pref_vel"].clone().requires_grad_(True)
    vmax = torch.tensor([p.max_speed], device="cuda", requires_grad=True)
    tau = torch.tensor([p.time_horizon], device="cuda", requires_grad=True)
    spec = autograd.TrajectorySpec(offsets=list(w.offsets), params=list(w.params),
                                   n_steps=w.steps, segment=20)
    pos, vel = autograd.trajectory(d["pos"], d["vel"], pref, vmax, tau, spec)
    y = torch.from_numpy(w.targets).cuda()
    loss = ((pos.double() - y.double()) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    g_pref = pref.grad.cpu().numpy().astype(np.float64)
    g_vmax = float(vmax.grad.cpu()[0])
    g_tau = float(tau.grad.cpu()[0])
    say("  loss %.6f  |dL/dvhat| %.4g  dL/dvmax %.6g  dL/dtau %.6g"
        % (float(loss), np.linalg.norm(g_pref), g_vmax, g_tau))
    rng = np.random.default_rng(9)
    pos0 = w.pos.astype(np.float64)
    vel0 = w.vel.astype(np.float64)
    pr = w.pref_vel.astype(np.float64)
    vm, ta = np.array([np.float32(p.max_speed)], float), np.array([np.float32(p.time_horizon)], float)
    dirs = [("vmax", np.zeros_like(pr), np.ones(1), np.zeros(1)),
            ("tau", np.zeros_like(pr), np.zeros(1), np.ones(1))]
    for k in range(3):
        dirs.append(("rand%d" % k, rng.normal(size=pr.shape), np.zeros(1), np.zeros(1)))
    for name, dp, dv, dt_ in dirs:
        L, dL = oracle.traj_jvp(pos0, vel0, pr, w.offsets, w.params, vm, ta, w.steps, w.targets,
                                dp, dv, dt_, f32_state=True)
        mine = float((g_pref * dp).sum() + g_vmax * dv[0] + g_tau * dt_[0])
        say("  direction %-6s: adjoint %.8g  forward mode %.8g  (loss %.6f)" % (name, mine, dL, L))
        assert abs(mine - dL) <= 1e-3 * max(abs(dL), 1e-6 * abs(L)), (name, mine, dL)
    spec.ctx.close()


def test_trajectory_gradient_with_and_without_the_kept_recording():
    """The forward records its last segment; the backward uses that recording
    only if the context has not stepped since.  With another step in between
    it replays the segment, and the gradients agree (up to the order of the
    float64 atomic sums of the adjoint's scatter)."""
    torch = _torch()
    from paper_1908_10107_amd import autograd, orca
    say("case trajectory gradient: kept recording vs replay")
    w = scenes.grad(n=1024)
    d = orca.to_device(w)
    p = w.params[0]
    y = torch.from_numpy(w.targets).cuda()
    grads = []
    for disturb in (False, True):
        pref = d["pref_vel"].clone().requires_grad_(True)
        vmax = torch.tensor([p.max_speed], device="cuda", requires_grad=True)
        tau = torch.tensor([p.time_horizon], device="cuda", requires_grad=True)
        spec = autograd.TrajectorySpec(offsets=list(w.offsets), params=list(w.params),
                                       n_steps=50, segment=20)
        pos, vel = autograd.trajectory(d["pos"], d["vel"], pref, vmax, tau, spec)
        if disturb:
            # an unrelated recorded step on the same context overwrites the tape
            q, v = d["pos"].clone(), d["vel"].clone()
            spec.ctx.step(w.offsets, w.params, q, v, d["pref_vel"], n_steps=3, save_tape=True)
        ((pos.double() - y.double()) ** 2).sum().backward()
        torch.cuda.synchronize()
        grads.append((pref.grad.cpu().numpy(), vmax.grad.cpu().numpy(), tau.grad.cpu().numpy()))
        spec.ctx.close()
    for a, b in zip(*grads):
        assert np.allclose(a, b, rtol=1e-5, atol=1e-6 * np.abs(a).max())
    assert np.abs(grads[0][0]).max() > 0


@pytest.mark.parametrize("horizon", [2, 8])
def test_adjoint_against_central_differences(horizon):
    """The GPU adjoint of the 4,096-agent trajectory against float64 central
    differences of the reference's loss (h = 1e-4 and h / 2, Richardson
    combined), along 16 random unit directions in (preferred velocities, v_max,
    tau) and along v_max and tau, counting only directions whose every
    decision at theta +- h delta matches theta's over the horizon.

    The GPU keeps its state in float32 and differentiates the branch that
    float32 path takes (rounding counts as the identity).  Central differences
    of the float64 loss measure the float64 path's branch, so they are the
    reference only while the float32 path takes the float64 path's decisions:
    the reference's decision hashes of both paths decide.  Where the paths
    part (on this workload from step 3 on), the adjoint is held to the
    reference's forward mode along the float32 path, its own branch, and the
    central differences pin that forward mode on the float64 path (CPU test
    of the same workload)."""
    torch = _torch()
    from paper_1908_10107_amd import autograd, orca
    say("case adjoint vs central differences, 4096 agents x %d steps" % horizon)
    w = scenes.grad()
    d = orca.to_device(w)
    p = w.params[0]
    pref = d["pref_vel"].clone().requires_grad_(True)
    vmax = torch.tensor([p.max_speed], device="cuda", requires_grad=True)
    tau = torch.tensor([p.time_horizon], device="cuda", requires_grad=True)
    spec = autograd.TrajectorySpec(offsets=list(w.offsets), params=list(w.params),
                                   n_steps=horizon, segment=horizon)
    pos, vel = autograd.trajectory(d["pos"], d["vel"], pref, vmax, tau, spec)
    y = torch.from_numpy(w.targets).cuda()
    ((pos.double() - y.double()) ** 2).sum().backward()
    torch.cuda.synchronize()
    g_pref = pref.grad.cpu().numpy().astype(np.float64)
    g_vmax = float(vmax.grad.cpu()[0])
    g_tau = float(tau.grad.cpu()[0])
    spec.ctx.close()
    h = 1e-4
    pos0, vel0 = w.pos.astype(np.float64), w.vel.astype(np.float64)
    pr = w.pref_vel.astype(np.float64)
    vm = np.array([np.float32(p.max_speed)], float)
    ta = np.array([np.float32(p.time_horizon)], float)
    curve = lambda a, b, c, **kw: oracle.traj_curve(pos0, vel0, a, w.offsets, w.params, b, c,
                                                    horizon, w.targets, **kw)
    _, _, tape0 = curve(pr, vm, ta)
    _, _, tape32 = curve(pr, vm, ta, f32_state=True)
    same = tape32 == tape0
    shared = int(np.argmin(same)) if not same.all() else horizon
    say("  the float32 path keeps the float64 path's decisions for %d of %d steps"
        % (shared, horizon))
    assert shared >= 2
    rng = np.random.default_rng(scenes.BASE_SEED + 4)
    dirs = []
    for k in range(16):
        v = rng.normal(size=pr.size + 2)
        v /= np.linalg.norm(v)
        dirs.append(("rand%d" % k, v[:-2].reshape(pr.shape), v[-2], v[-1]))
    dirs += [("vmax", np.zeros_like(pr), 1.0, 0.0), ("tau", np.zeros_like(pr), 0.0, 1.0)]
    counted = 0
    worst = 0.0
    for name, dp, dv, dt_ in dirs:
        mine = float((g_pref * dp).sum() + g_vmax * dv + g_tau * dt_)
        runs = []
        for e in (h, -h, h / 2, -h / 2):
            L, _, tp = curve(pr + e * dp, vm + e * dv, ta + e * dt_)
            runs.append((L[-1], np.array_equal(tp, tape0)))
        fd_counts = all(r[1] for r in runs)  # no decision switches inside the interval
        fd = (runs[0][0] - runs[1][0]) / (2 * h)
        fd2 = (runs[2][0] - runs[3][0]) / h
        rich = (4 * fd2 - fd) / 3
        counted += int(fd_counts)
        if shared >= horizon:
            if not fd_counts:
                continue
            err = abs(mine - rich) / abs(rich)
            say("  %-6s adjoint %.9g  central differences %.9g  rel %.2e"
                % (name, mine, rich, err))
        else:
            _, jvp32 = oracle.traj_jvp(pos0, vel0, pr, w.offsets, w.params, vm, ta, horizon,
                                       w.targets, dp, np.array([dv]), np.array([dt_]),
                                       f32_state=True)
            err = abs(mine - jvp32) / abs(jvp32)
            say("  %-6s adjoint %.9g  forward mode (float32 path) %.9g  rel %.2e  "
                "central differences (float64 path%s) %.9g"
                % (name, mine, jvp32, err, "" if fd_counts else ", a switch inside", rich))
        worst = max(worst, err)
        assert err <= 1e-3, (name, mine)
    say("  %d of %d directions keep every float64 decision at +-h, worst relative difference "
        "%.2e" % (counted, len(dirs), worst))
    assert counted >= (18 if horizon == 2 else 9)


@pytest.mark.parametrize("case", ["plain", "hetero"])
def test_backward_steps_equals_per_step_backward(case):
    """orca_backward_steps over a recorded segment (gradients kept per agent id
    inside the context between the steps) equals orca_backward step by step
    (gradients through the caller's arrays), to float32 rounding of the
    accumulation order, with the output arrays aliasing the inputs; a
    single-step range equals orca_backward."""
    torch = _torch()
    from paper_1908_10107_amd import orca
    say("case backward_steps", case)
    w = moving_scene(5000, 2.0, 44)
    if case == "hetero":
        rng = np.random.default_rng(45)
        w.radius = rng.choice(np.array([0.15, 0.25, 0.4], np.float32), w.n)
        w.max_speed = rng.uniform(0.9, 2.0, w.n).astype(np.float32)
    d = orca.to_device(w)
    k = w.params[0].max_neighbors
    steps = 7
    ctx = orca.Context(max_agents=w.n, max_scenes=1, k_max=k, tape_steps=steps)
    ctx.set_agents(d["radius"], d["max_speed"])
    ctx.step(w.offsets, w.params, d["pos"], d["vel"], d["pref_vel"], n_steps=steps, save_tape=True)
    rng = np.random.default_rng(46)
    gp0 = torch.from_numpy(rng.normal(size=(2, w.n)).astype(np.float32)).cuda()
    gv0 = torch.from_numpy(rng.normal(size=(2, w.n)).astype(np.float32)).cuda()
    outs = []
    for mode in ("steps", "each"):
        gp, gv = gp0.clone(), gv0.clone()
        gpref = torch.zeros_like(gp)
        gvm = torch.zeros(1, device="cuda")
        gta = torch.zeros(1, device="cuda")
        if mode == "steps":
            ctx.backward_steps(0, steps - 1, gp, gv, gp, gv, gpref, gvm, gta)
        else:
            for t in reversed(range(steps)):
                ctx.backward(t, gp, gv, gp, gv, gpref, gvm, gta)
        torch.cuda.synchronize()
        outs.append([x.cpu().numpy().astype(np.float64) for x in (gp, gv, gpref, gvm, gta)])
    for name, a, b in zip(("g_pos", "g_vel", "g_pref", "g_vmax", "g_tau"), *outs):
        scale = max(np.abs(b).max(), 1e-30)
        err = np.abs(a - b).max() / scale
        say("  %s: max |steps - each| / max |each| = %.2e" % (name, err))
        assert err <= 1e-5, (name, err)
    # a range of one step is orca_backward
    gp1, gv1 = gp0.clone(), gv0.clone()
    gp2, gv2 = gp0.clone(), gv0.clone()
    z = [torch.zeros_like(gp0) for _ in range(2)]
    ctx.backward_steps(steps - 1, steps - 1, gp1, gv1, gp1, gv1, z[0])
    ctx.backward(steps - 1, gp2, gv2, gp2, gv2, z[1])
    torch.cuda.synchronize()
    for a, b in ((gp1, gp2), (gv1, gv2), (z[0], z[1])):
        a, b = a.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)
        assert np.abs(a - b).max() <= 1e-5 * max(np.abs(b).max(), 1e-30)
    with pytest.raises(orca.OrcaError):
        ctx.backward_steps(3, 2, gp1, gv1, gp1, gv1, z[0])
    with pytest.raises(orca.OrcaError):
        ctx.backward_steps(0, steps, gp1, gv1, gp1, gv1, z[0])
    ctx.close()
