"""orca_step_noalloc (the step on the library's static scratch array, for
callers that cannot allocate) against orca_step on a context, through the C ABI.

Both run the same kernels with the same launch shapes, so positions,
velocities and steered preferred velocities must be equal bit for bit; the
first call is also held to the oracle's velocities (1e-4 m/s).  Two calls in a
row, the second with a smaller scene and a smaller neighbour cap, check that
nothing the first call left in the shared scratch leaks into the second.
"""
import ctypes
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


def run_both(w, n_steps):
    """(context result, no-alloc result): pos, vel, pref_vel after n_steps."""
    torch = _torch()
    from paper_1908_10107_amd import orca
    assert w.n_scenes == 1
    p = w.params[0]
    a = orca.to_device(w)
    b = orca.to_device(w)
    with orca.Context(max_agents=max(w.n, 1), max_scenes=1, k_max=max(1, p.max_neighbors)) as ctx:
        ctx.step(w.offsets, w.params, a["pos"], a["vel"], a["pref_vel"], goals=a["goals"],
                 n_steps=n_steps)
        torch.cuda.synchronize()
    orca.step_noalloc(p, b["pos"], b["vel"], b["pref_vel"], goals=b["goals"], n_steps=n_steps)
    torch.cuda.synchronize()
    get = lambda d: {k: d[k].cpu().numpy().copy() for k in ("pos", "vel", "pref_vel")}
    return get(a), get(b)


def test_noalloc_equals_context_step_twice():
    torch = _torch()
    # first call: a dense scene at the scratch array's capacity, K = 16
    big = scenes.dense_uniform(n=16384, seed=scenes.BASE_SEED + 40)
    say("no-alloc call 1: %d agents, K = %d, 3 steps" % (big.n, big.params[0].max_neighbors))
    ref, got = run_both(big, 3)
    for k in ref:
        diff = int(np.count_nonzero(ref[k] != got[k]))
        assert diff == 0, "call 1: %s differs in %d entries" % (k, diff)
    # one step from the initial state against the oracle (the parity bar)
    from paper_1908_10107_amd import orca
    d = orca.to_device(big)
    orca.step_noalloc(big.params[0], d["pos"], d["vel"], d["pref_vel"], goals=d["goals"])
    torch.cuda.synchronize()
    o = oracle.velocities(big.pos, big.vel, big.pref_vel, big.offsets, big.params,
                          goals=big.goals)
    v = d["vel"].cpu().numpy().T.astype(np.float64)
    err = float(np.abs(v - o["new_vel"]).max())
    say("call 1 against the oracle: max |dv| = %.3g m/s" % err)
    assert err < 1e-4
    # second call: a smaller scene with a smaller neighbour cap
    small = scenes.uniform_rsa()
    say("no-alloc call 2: %d agents, K = %d, 5 steps" % (small.n, small.params[0].max_neighbors))
    ref, got = run_both(small, 5)
    for k in ref:
        diff = int(np.count_nonzero(ref[k] != got[k]))
        assert diff == 0, "call 2: %s differs in %d entries" % (k, diff)


def test_noalloc_without_goals_and_empty():
    torch = _torch()
    from paper_1908_10107_amd import orca
    w = scenes.tiny_random(3000, 30.0, seed=207, max_neighbors=16)
    say("no-alloc without goals: %d agents, 4 steps" % w.n)
    ref, got = run_both(w, 4)
    for k in ref:
        assert np.array_equal(ref[k], got[k]), k
    # an empty scene enqueues nothing that touches agents
    e = torch.zeros((2, 0), dtype=torch.float32, device="cuda")
    orca.step_noalloc(w.params[0], e, e.clone(), e.clone())
    torch.cuda.synchronize()


def test_noalloc_rejects_sizes_beyond_its_scratch():
    _torch()
    from paper_1908_10107_amd import orca
    lib = orca.load()
    p = scenes.uniform_rsa().params[0]
    err = ctypes.create_string_buffer(256)
    # rejected on the host before anything is enqueued (no device pointer is read)
    rc = lib.orca_step_noalloc(orca.NOALLOC_MAX_AGENTS + 1, orca.params_array([p]), None, None,
                               None, None, 1, None, err, len(err))
    assert rc == orca.ECAPACITY and b"capacity" in err.value
    q = orca.params_array([p])
    q[0].max_neighbors = orca.NOALLOC_MAX_NEIGHBORS + 1
    rc = lib.orca_step_noalloc(10, q, None, None, None, None, 1, None, err, len(err))
    assert rc == orca.ECAPACITY
    rc = lib.orca_step_noalloc(10, orca.params_array([p]), None, None, None, None, 0, None, err,
                               len(err))
    assert rc == orca.EINVAL


def test_noalloc_under_graph_capture():
    """The entry point enqueues kernels only, so it can be captured into a HIP
    graph: replays of a captured 4-step call, with eager work and waits
    between them, equal the same steps run eagerly, replay after replay."""
    torch = _torch()
    from paper_1908_10107_amd import orca
    w = scenes.uniform_rsa()
    p = w.params[0]
    say("no-alloc under graph capture: %d agents" % w.n)
    a = orca.to_device(w)
    b = orca.to_device(w)
    orca.step_noalloc(p, a["pos"], a["vel"], a["pref_vel"], goals=a["goals"])  # warm-up
    orca.step_noalloc(p, b["pos"], b["vel"], b["pref_vel"], goals=b["goals"])
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            orca.step_noalloc(p, b["pos"], b["vel"], b["pref_vel"], goals=b["goals"], n_steps=4)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    # capture does not run the steps: b is still one step in
    side = torch.zeros(1 << 20, device="cuda")
    for r in range(3):
        orca.step_noalloc(p, a["pos"], a["vel"], a["pref_vel"], goals=a["goals"], n_steps=4)
        g.replay()
        side.add_(1.0)
        torch.cuda.synchronize()
        for k in ("pos", "vel", "pref_vel"):
            assert torch.equal(a[k], b[k]), (r, k)
