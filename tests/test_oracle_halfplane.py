"""Pins of the reference half-plane construction (section 3, Fig. 1).

Nothing here re-types the construction.  Each test checks a property that the
velocity obstacle's definition fixes on its own:
  * the obstacle is the set of relative velocities V' with |t V' - P| < R for
    some t in (0, tau]; u must be the shortest vector from V to its boundary,
    found here by brute-force ray marching with that membership test;
  * after both agents move half of u the pair grazes at distance exactly R;
  * swapping the agents negates u and n (each takes half, section 2);
  * u is continuous when V crosses from the arc region to a leg.
"""
import numpy as np
import pytest

R_PAIR = 0.5  # two agents of radius 0.25
TAU = 5.0
DT = 0.1


def cross(a, b):
    return a[0] * b[1] - a[1] * b[0]


def in_vo(Vp, P, R, tau):
    """Membership of relative velocities Vp [...,2] in the obstacle, by its definition."""
    Vp = np.asarray(Vp, np.float64)
    vv = (Vp * Vp).sum(-1)
    pv = (Vp * P).sum(-1)
    with np.errstate(invalid="ignore", divide="ignore"):
        t = np.where(vv > 0, pv / vv, 0.0)
    t = np.clip(t, 1e-300, tau)
    d = np.linalg.norm(t[..., None] * Vp - P, axis=-1)
    return d < R


def _first_crossing(V, dirs, P, R, tau, inside, far=40.0, n_samp=800):
    """Distance along each direction to the first change of membership (inf if none)."""
    samples = np.linspace(0.0, far, n_samp + 1)[1:]
    pts = V + samples[None, :, None] * dirs[:, None, :]
    flip = in_vo(pts, P, R, tau) != inside
    anyflip = flip.any(axis=1)
    first = np.where(anyflip, flip.argmax(axis=1), 0)
    hi = np.where(anyflip, samples[first], np.inf)
    lo = np.where(first > 0, samples[np.maximum(first - 1, 0)], 0.0)
    ok = np.isfinite(hi)
    lo, hi2 = lo[ok], hi[ok]
    for _ in range(55):
        mid = 0.5 * (lo + hi2)
        f = in_vo(V + mid[:, None] * dirs[ok], P, R, tau) != inside
        hi2 = np.where(f, mid, hi2)
        lo = np.where(f, lo, mid)
    hi[ok] = hi2
    return hi


def boundary_distance(V, P, R, tau, n_dir=1440):
    """Distance from V to the obstacle boundary: coarse ray sweep, then a fine sweep."""
    inside = bool(in_vo(V, P, R, tau))
    th = np.linspace(0.0, 2 * np.pi, n_dir, endpoint=False)
    dist = _first_crossing(V, np.stack([np.cos(th), np.sin(th)], -1), P, R, tau, inside)
    c = th[np.argmin(dist)]
    step = 2 * np.pi / n_dir
    th2 = c + np.linspace(-3 * step, 3 * step, 241)
    dirs2 = np.stack([np.cos(th2), np.sin(th2)], -1)
    dist2 = _first_crossing(V, dirs2, P, R, tau, inside)
    j = np.argmin(dist2)
    return dist2[j], V + dist2[j] * dirs2[j]


def closest_approach(P, W, horizon):
    """min over t in [0, horizon] of |P - t W| (relative motion with velocity W)."""
    ww = W @ W
    t = 0.0 if ww == 0 else np.clip((P @ W) / ww, 0.0, horizon)
    return np.linalg.norm(P - t * W), t


def two_agent(oracle, xa, xb, va, vb, vmax=1.5, dt=DT):
    """Both agents take the velocity the method picks with vhat = current velocity."""
    xa, xb, va, vb = map(lambda a: np.asarray(a, np.float64), (xa, xb, va, vb))
    out = []
    for xi, xj, vi, vj, first in ((xa, xb, va, vb, True), (xb, xa, vb, va, False)):
        code, u, n = oracle.halfplane(xj - xi, vi - vj, R_PAIR, TAU, dt, first)
        v, st, _ = oracle.solve([vi + 0.5 * u], [n], vmax, vi)
        out.append((code, u, n, v, st))
    return out


def test_leg_case_grazes(oracle_lib):
    (ca, ua, na, va2, sa), (cb, ub, nb, vb2, sb) = two_agent(
        oracle_lib, (-2, -0.05), (2, 0.05), (1, 0), (-1, 0))
    assert sa == sb == 0
    assert ca in (1, 2) and cb in (1, 2)
    P = np.array([4.0, 0.1])
    d, t = closest_approach(P, va2 - vb2, TAU)
    assert abs(d - R_PAIR) < 1e-12 and 0 < t < TAU
    np.testing.assert_allclose(va2, -vb2, atol=1e-15)


def test_cutoff_case_grazes_at_tau(oracle_lib):
    (ca, ua, _, va2, _), (_, _, _, vb2, _) = two_agent(
        oracle_lib, (0, 0), (3, 0), (0.55, 0), (0, 0))
    assert ca == 0
    d, t = closest_approach(np.array([3.0, 0.0]), va2 - vb2, TAU)
    assert abs(d - R_PAIR) < 1e-12 and abs(t - TAU) < 1e-12
    # each side moves by half of the same correction
    np.testing.assert_allclose(va2 - np.array([0.55, 0]), -(vb2 - 0), atol=1e-15)


def test_overlap_case_separates_in_one_step(oracle_lib):
    (ca, _, _, va2, _), (_, _, _, vb2, _) = two_agent(
        oracle_lib, (0, 0), (0.4, 0), (0, 0), (0, 0))
    assert ca == 3
    P = np.array([0.4, 0.0])
    sep = np.linalg.norm(P - DT * (va2 - vb2))
    assert abs(sep - R_PAIR) < 1e-12


def test_head_on_both_dodge_right(oracle_lib):
    (ca, ua, _, va2, _), (cb, ub, _, vb2, _) = two_agent(
        oracle_lib, (-2, 0), (2, 0), (1, 0), (-1, 0))
    # |u| = |V| R / |P| for an exactly head-on pair (tangent of the cone)
    assert abs(np.linalg.norm(ua) - 2.0 * R_PAIR / 4.0) < 1e-14
    for v, v2 in (((1, 0), va2), ((-1, 0), vb2)):
        d = v2 - np.asarray(v, float)
        assert cross(np.asarray(v, float), d) < 0  # clockwise = to the mover's right
    d, _ = closest_approach(np.array([4.0, 0.0]), va2 - vb2, TAU)
    assert abs(d - R_PAIR) < 1e-12


@pytest.mark.parametrize("seed", range(40))
def test_u_is_shortest_vector_to_boundary(oracle_lib, seed):
    rng = np.random.default_rng(1000 + seed)
    R = rng.uniform(0.3, 1.5)
    P = rng.normal(size=2)
    P *= rng.uniform(R * 1.05, 6.0) / np.linalg.norm(P)
    V = rng.normal(size=2) * rng.uniform(0.05, 2.0)
    tau = rng.uniform(1.0, 8.0)
    code, u, n = oracle_lib.halfplane(P, V, R, tau, DT, True)
    dist, pt = boundary_distance(V, P, R, tau)
    assert abs(np.linalg.norm(u) - dist) < 2e-5 * max(1.0, dist)
    assert np.linalg.norm(V + u - pt) < 5e-3 * max(1.0, dist) + 1e-4
    # n is the unit outward normal: stepping along n leaves the obstacle
    assert abs(np.linalg.norm(n) - 1) < 1e-14
    eps = 1e-6
    assert not in_vo(V + u + eps * n, P, R, tau)
    assert in_vo(V + u - eps * n, P, R, tau)


@pytest.mark.parametrize("seed", range(20))
def test_overlap_branch_lands_on_one_step_circle(oracle_lib, seed):
    rng = np.random.default_rng(2000 + seed)
    R = rng.uniform(0.3, 1.5)
    P = rng.normal(size=2)
    P *= rng.uniform(0.0, R) / np.linalg.norm(P)
    V = rng.normal(size=2)
    code, u, n = oracle_lib.halfplane(P, V, R, TAU, DT, True)
    assert code == 3
    # after the correction the pair is exactly R apart after dt
    assert abs(np.linalg.norm(DT * (V + u) - P) - R) < 1e-12
    # and u is radial from the centre P/dt (shortest way onto that circle)
    w = V - P / DT
    assert abs(cross(w, u)) < 1e-12 * (1 + np.linalg.norm(w) * np.linalg.norm(u))


@pytest.mark.parametrize("seed", range(200))
def test_reciprocal(oracle_lib, seed):
    rng = np.random.default_rng(3000 + seed)
    P = rng.normal(size=2) * rng.uniform(0.0, 3.0)
    V = rng.normal(size=2)
    if seed % 10 == 0:
        V = P * rng.uniform(-2, 2)        # exactly head-on: det(P, w) = 0
    if seed % 25 == 1:
        P = np.zeros(2)
        V = np.zeros(2)                   # coincident, equal velocities
    _, u1, n1 = oracle_lib.halfplane(P, V, 0.5, TAU, DT, True)
    _, u2, n2 = oracle_lib.halfplane(-P, -V, 0.5, TAU, DT, False)
    np.testing.assert_allclose(u2, -u1, atol=1e-12)
    np.testing.assert_allclose(n2, -n1, atol=1e-12)


def test_u_continuous_across_arc_leg_switch(oracle_lib):
    P = np.array([3.0, 0.4])
    codes, us = [], []
    # sweep V along a line that passes from the leg region into the arc region
    for s in np.linspace(-1.5, 1.5, 30001):
        V = np.array([0.2, s])
        c, u, _ = oracle_lib.halfplane(P, V, R_PAIR, TAU, DT, True)
        codes.append(c)
        us.append(u)
    us = np.array(us)
    jumps = np.linalg.norm(np.diff(us, axis=0), axis=1)
    assert len(set(codes)) >= 2
    assert jumps.max() < 1e-3
