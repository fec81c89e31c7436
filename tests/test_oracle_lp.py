"""Pins of the reference velocity choice (section 3: linear program; infeasible case).

The reference enumerates candidate points.  These tests check its answers by
routes that share nothing with that enumeration:
  * KKT certificate: the projection of vhat onto disc ∩ half-planes is optimal
    iff vhat - v lies in the normal cone of the set at v; the multipliers are
    recovered with non-negative least squares;
  * brute force: no feasible point of a dense polar grid is closer to vhat;
  * closed forms: vhat already permitted; one half-plane;
  * least penetration d*: bracketed by scipy's LP solver (HiGHS) on polygons
    inscribed in and circumscribed about the speed disc;
  * fallback closed forms: one half-plane beyond the disc, two facing
    half-planes with a gap (the ring pattern).
"""
import numpy as np
import pytest
from scipy.optimize import linprog, nnls

DELTA = 1e-5


def random_problem(rng, m, vmax=1.5, spread=1.0):
    ang = rng.uniform(0, 2 * np.pi, m)
    n = np.stack([np.cos(ang), np.sin(ang)], 1)
    q = rng.normal(size=(m, 2)) * spread
    vhat = rng.normal(size=2) * 1.2
    return q, n, vmax, vhat


def kkt_residual(q, n, vmax, vhat, v, shift=0.0, tol=1e-7):
    """Residual of vhat - v = sum_k lam_k (-n_k) + mu v with lam, mu >= 0 on the active set."""
    cols = []
    for k in range(len(q)):
        if abs(n[k] @ (v - q[k]) + shift) < tol:
            cols.append(-n[k])
    if abs(np.linalg.norm(v) - vmax) < tol:
        cols.append(v / np.linalg.norm(v))
    g = vhat - v
    if not cols:
        return np.linalg.norm(g)
    A = np.stack(cols, 1)
    _, res = nnls(A, g)
    return res


@pytest.mark.parametrize("seed", range(300))
def test_projection_kkt_and_feasible(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(0, 17))
    q, n, vmax, vhat = random_problem(rng, m, spread=0.6)
    v = oracle_lib.project(q, n, vmax, vhat)
    if v is None:
        # empty: the least-penetration value must then be positive
        d, _ = oracle_lib.min_max(q, n, vmax)
        assert d > -1e-9
        return
    assert np.linalg.norm(v) <= vmax + 1e-9
    for k in range(m):
        assert n[k] @ (v - q[k]) >= -1e-9
    assert kkt_residual(q, n, vmax, vhat, v) < 1e-7


@pytest.mark.parametrize("seed", range(40))
def test_projection_vs_polar_grid(oracle_lib, seed):
    rng = np.random.default_rng(500 + seed)
    m = int(rng.integers(1, 6))
    q, n, vmax, vhat = random_problem(rng, m, spread=0.4)
    v = oracle_lib.project(q, n, vmax, vhat)
    r = np.linspace(0, vmax, 600)
    a = np.linspace(0, 2 * np.pi, 1800, endpoint=False)
    G = (r[:, None, None] * np.stack([np.cos(a), np.sin(a)], -1)[None]).reshape(-1, 2)
    viol = np.einsum("kd,gkd->gk", n, G[:, None, :] - q[None])
    feas = np.all(viol >= 0, axis=1)
    if v is None:
        assert not feas.any()
        return
    if feas.any():
        dmin = np.linalg.norm(G[feas] - vhat, axis=1).min()
        assert np.linalg.norm(v - vhat) <= dmin + 1e-12
        # and the grid gets within its resolution of the answer
        assert dmin - np.linalg.norm(v - vhat) < 2 * vmax * np.pi / 1800 + vmax / 600


def test_permitted_vhat_is_returned(oracle_lib):
    q = np.array([[0.0, -2.0], [-2.0, 0.0]])
    n = np.array([[0.0, 1.0], [1.0, 0.0]])
    vhat = np.array([0.3, 0.2])
    assert np.array_equal(oracle_lib.project(q, n, 1.5, vhat), vhat)


@pytest.mark.parametrize("seed", range(100))
def test_single_halfplane_closed_form(oracle_lib, seed):
    rng = np.random.default_rng(900 + seed)
    a = rng.uniform(0, 2 * np.pi)
    n = np.array([np.cos(a), np.sin(a)])
    c = rng.uniform(-1.4, 1.4)                 # boundary n.v = c crosses the disc
    q = c * n + rng.normal() * np.array([-n[1], n[0]])
    vmax = 1.5
    vhat = rng.normal(size=2) * 1.5
    # textbook: clip to the disc if allowed; else drop onto the line, and if that
    # leaves the disc, take the end of the chord on vhat's side
    if n @ vhat >= c:
        l = np.linalg.norm(vhat)
        want = vhat if l <= vmax else vhat * vmax / l
        if n @ want < c:  # the radial clip fell outside the half-plane
            h = np.sqrt(vmax ** 2 - c ** 2)
            d = np.array([-n[1], n[0]])
            want = c * n + np.sign(d @ vhat) * h * d
    else:
        p = vhat + (c - n @ vhat) * n
        if np.linalg.norm(p) <= vmax:
            want = p
        else:
            h = np.sqrt(vmax ** 2 - c ** 2)
            d = np.array([-n[1], n[0]])
            want = c * n + np.sign(d @ vhat) * h * d
    got = oracle_lib.project([q], [n], vmax, vhat)
    np.testing.assert_allclose(got, want, atol=1e-12)


def polygon_dstar(q, n, vmax, sides, outer):
    """min t s.t. n_k.(q_k - v) <= t, v in a regular polygon (inscribed or circumscribed)."""
    a = np.linspace(0, 2 * np.pi, sides, endpoint=False)
    e = np.stack([np.cos(a), np.sin(a)], 1)
    rad = vmax / np.cos(np.pi / sides) if outer else vmax
    # polygon: e_i . v <= rad cos(pi/sides) for circumscribed / inscribed facets
    h = rad * np.cos(np.pi / sides)
    A = np.concatenate([np.concatenate([-n, -np.ones((len(q), 1))], 1),
                        np.concatenate([e, np.zeros((sides, 1))], 1)])
    b = np.concatenate([-(n * q).sum(1), np.full(sides, h)])
    res = linprog([0, 0, 1], A_ub=A, b_ub=b, bounds=[(None, None)] * 3, method="highs")
    assert res.status == 0
    return res.fun


@pytest.mark.parametrize("seed", range(60))
def test_min_max_bracketed_by_lp(oracle_lib, seed):
    rng = np.random.default_rng(1500 + seed)
    m = int(rng.integers(1, 17))
    q, n, vmax, _ = random_problem(rng, m, spread=1.5)
    d, v = oracle_lib.min_max(q, n, vmax)
    lo = polygon_dstar(q, n, vmax, 4096, outer=True)
    hi = polygon_dstar(q, n, vmax, 4096, outer=False)
    assert lo - 1e-9 <= d <= hi + 1e-9
    assert hi - lo < 1e-5
    # the reported point attains d*
    assert np.linalg.norm(v) <= vmax * (1 + 1e-12) + 1e-12
    assert abs(np.max(np.einsum("kd,kd->k", n, q - v)) - d) < 1e-12


def test_fallback_one_halfplane_beyond_disc(oracle_lib):
    n = np.array([0.6, 0.8])
    q = 2.0 * n + np.array([0.3, -0.225])      # n.q = 2 > vmax
    vmax = 1.5
    vhat = np.array([-1.0, 0.4])
    v, st, d = oracle_lib.solve([q], [n], vmax, vhat)
    assert st == 1
    assert abs(d - (2.0 - vmax)) < 1e-14
    # the permitted cap {n.v >= vmax - delta} is within sqrt(2 vmax delta) of vmax n
    assert np.linalg.norm(v - vmax * n) <= np.sqrt(2 * vmax * DELTA) + 1e-12
    assert n @ v >= vmax - DELTA - 1e-12


@pytest.mark.parametrize("vhat", [(0.0, 1.3), (0.7, -0.2), (-1.4, 0.9)])
def test_fallback_facing_halfplanes(oracle_lib, vhat):
    # v_x >= 1.9 and v_x <= -1.9: gap 3.8, so d* = 1.9 and the middle strip is |v_x| <= delta
    q = np.array([[1.9, 0.0], [-1.9, 0.0]])
    n = np.array([[1.0, 0.0], [-1.0, 0.0]])
    vmax = 1.5
    vhat = np.array(vhat)
    v, st, d = oracle_lib.solve(q, n, vmax, vhat)
    assert st == 1 and abs(d - 1.9) < 1e-14
    vx = np.clip(vhat[0], -DELTA, DELTA)
    want = np.array([vx, vhat[1]])
    if np.linalg.norm(want) > vmax:
        want = np.array([vx, np.sign(vhat[1]) * np.sqrt(vmax ** 2 - vx ** 2)])
    np.testing.assert_allclose(v, want, atol=1e-12)


@pytest.mark.parametrize("seed", range(150))
def test_fallback_second_stage_kkt(oracle_lib, seed):
    rng = np.random.default_rng(2500 + seed)
    m = int(rng.integers(2, 17))
    q, n, vmax, vhat = random_problem(rng, m, spread=2.0)
    v, st, d = oracle_lib.solve(q, n, vmax, vhat)
    if st == 0:
        return
    # v is within d* + delta of every half-plane, inside the disc, and optimal there
    assert np.linalg.norm(v) <= vmax + 1e-9
    assert np.max(np.einsum("kd,kd->k", n, q - v)) <= d + DELTA + 1e-9
    assert kkt_residual(q, n, vmax, vhat, v, shift=d + DELTA) < 1e-7
