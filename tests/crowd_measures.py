"""Crowd measures for the crossing tests (no part of the method: they only
summarise positions and velocities)."""
import numpy as np


def lane_order(pos, present, group, half_width=15.0, band=1.0):
    """Band order parameter of a two-way flow: agents within half_width of the
    centre line are binned into bands of the given height across the flow; each
    band with two or more people scores |n_a - n_b| / (n_a + n_b) for its two
    groups, weighted by its population.  Lanes give values near 1, mixed
    crowds values near 1 / sqrt(people per band)."""
    sel = present & (np.abs(pos[0]) < half_width)
    b = np.floor(pos[1, sel] / band).astype(int)
    g = group[sel]
    acc = tot = 0
    for k in np.unique(b):
        m = b == k
        n = int(m.sum())
        if n >= 2:
            acc += abs(2 * int(g[m].sum()) - n)
            tot += n
    return acc / max(tot, 1)


def turning_speed(pos, vel, present):
    """Mean speed about the origin of the present agents: their angular
    momentum about it over the sum of their distances from it (m/s, positive
    for counter-clockwise turning)."""
    x, y = pos[0, present].astype(np.float64), pos[1, present].astype(np.float64)
    vx, vy = vel[0, present].astype(np.float64), vel[1, present].astype(np.float64)
    return float((x * vy - y * vx).sum() / np.hypot(x, y).sum())
