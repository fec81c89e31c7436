/*
 * orca_oracle_core.h -- the float64 geometry and programs of the CPU
 * reference, written once over a scalar type and included twice by
 * orca_oracle.c (TEST INFRASTRUCTURE ONLY):
 *
 *   REAL = double           FN(x) = x       the reference itself
 *   REAL = double complex   FN(x) = x##_cx  complex-step forward mode: the
 *       inputs carry i*h*tangent, every decision compares real parts (so the
 *       discrete choices are those of the primal), and the imaginary part of
 *       each result is h times its directional derivative.
 *
 * RE(x) is the real part, SQRT the square root of REAL.  For REAL = double
 * these expand to the plain operations, so the reference's arithmetic is
 * unchanged by the second instantiation.
 */

typedef struct {
    REAL qx, qy, nx, ny;
} FN(halfplane_t);

/*
 * Half-plane of one neighbour (section 3, Fig. 1(b)-(c)).  P = x_j - x_i,
 * V = v_i - v_j, R = r_i + r_j.  The velocity obstacle for look-ahead tau is
 * the set of relative velocities that bring the pair closer than R at some
 * t in (0, tau]: a cone from the origin tangent to the disc D(P, R), cut off
 * by the disc D(P/tau, R/tau).  u runs from V to the closest boundary point
 * and n is the outward normal there.  Pairs already closer than R use dt in
 * place of tau (they must separate within one step).  Returns the branch code.
 */
static int FN(obstacle)(REAL Px, REAL Py, REAL Vx, REAL Vy, REAL R, REAL tau, REAL dt,
                        int i_before_j, REAL *ux, REAL *uy, REAL *nx, REAL *ny)
{
    REAL dist2 = Px * Px + Py * Py;
    REAL R2 = R * R;
    if (RE(dist2) > RE(R2)) {
        /* w: from the centre of the cut-off disc to V */
        REAL wx = Vx - Px / tau, wy = Vy - Py / tau;
        REAL w2 = wx * wx + wy * wy;
        REAL wP = wx * Px + wy * Py;
        if (RE(wP) < 0.0 && RE(wP * wP) > RE(R2 * w2)) {
            /* V faces the cut-off arc: nearest boundary point is on the circle */
            REAL wl = SQRT(w2);
            *nx = wx / wl;
            *ny = wy / wl;
            *ux = (R / tau - wl) * *nx;
            *uy = (R / tau - wl) * *ny;
            return ORC_ARC;
        }
        /* otherwise the nearest boundary point is on one of the two tangent legs */
        REAL L = SQRT(dist2 - R2);
        REAL lx, ly;
        int code;
        if (RE(Px * wy - Py * wx) > 0.0) {
            /* left leg: P's direction turned counter-clockwise by asin(R/|P|) */
            lx = (Px * L - Py * R) / dist2;
            ly = (Px * R + Py * L) / dist2;
            *nx = -ly;
            *ny = lx;
            code = ORC_LEFT;
        } else {
            /* right leg: turned clockwise */
            lx = (Px * L + Py * R) / dist2;
            ly = (-Px * R + Py * L) / dist2;
            *nx = ly;
            *ny = -lx;
            code = ORC_RIGHT;
        }
        /* u = (closest point of the leg line to V) - V */
        REAL s = Vx * lx + Vy * ly;
        *ux = s * lx - Vx;
        *uy = s * ly - Vy;
        return code;
    }
    /* already in contact: cut-off disc D(P/dt, R/dt) */
    REAL wx = Vx - Px / dt, wy = Vy - Py / dt;
    REAL wl = SQRT(wx * wx + wy * wy);
    if (RE(wl) > 0.0) {
        *nx = wx / wl;
        *ny = wy / wl;
    } else if (RE(dist2) > 0.0) {
        REAL pl = SQRT(dist2);
        *nx = -Px / pl;
        *ny = -Py / pl;
    } else {
        *nx = i_before_j ? 1.0 : -1.0;
        *ny = 0.0;
    }
    *ux = (R / dt - wl) * *nx;
    *uy = (R / dt - wl) * *ny;
    return ORC_OVERLAP;
}

/* Feasible for every half-plane n.(v - q) >= -shift and inside the disc. */
static int FN(feasible)(int m, const FN(halfplane_t) *h, REAL shift, REAL vmax, REAL vx, REAL vy)
{
    if (RE(vx * vx + vy * vy) > RE(vmax * vmax) * (1.0 + 1e-12) + 1e-12) return 0;
    for (int k = 0; k < m; ++k) {
        REAL s = h[k].nx * (vx - h[k].qx) + h[k].ny * (vy - h[k].qy);
        if (RE(s) < -RE(shift) - ORC_TOL) return 0;
    }
    return 1;
}

typedef struct {
    int found;
    REAL bx, by;
    double bd;
    int code; /* which candidate won (a discrete choice; see project()) */
} FN(best_t);

static void FN(consider)(FN(best_t) *b, int m, const FN(halfplane_t) *h, REAL shift, REAL vmax,
                         REAL px, REAL py, REAL vhx, REAL vhy, int code)
{
    if (!isfinite(RE(px)) || !isfinite(RE(py))) return;
    if (!FN(feasible)(m, h, shift, vmax, px, py)) return;
    double d = RE((px - vhx) * (px - vhx) + (py - vhy) * (py - vhy));
    if (!b->found || d < b->bd) { b->found = 1; b->bx = px; b->by = py; b->bd = d; b->code = code; }
}

/*
 * argmin |v - vhat| over the disc |v| <= vmax and the half-planes
 * n_k.(v - q_k) >= -shift (section 3: the permitted velocity closest to the
 * preferred one).  The minimiser of a strictly convex function over this set
 * is vhat itself, the radial clip of vhat, the projection of vhat onto one
 * boundary line, a line-circle crossing, or a line-line crossing; all of them
 * are tried.  Returns 1 and writes the minimiser if the set is non-empty,
 * else 0.  *which (nullable) names the candidate that won: 0 vhat, 1 its
 * clip, 2 + 4k the foot on line k, 3 + 4k and 4 + 4k its circle crossings,
 * 100000 + 64k + l the crossing of lines k < l; -1 when empty.
 */
static int FN(project)(int m, const FN(halfplane_t) *h, REAL shift, REAL vmax, REAL vhx, REAL vhy,
                       REAL *ox, REAL *oy, int *which)
{
    FN(best_t) b;
    b.found = 0;
    b.bd = 0.0;
    b.code = -1;
    FN(consider)(&b, m, h, shift, vmax, vhx, vhy, vhx, vhy, 0);
    REAL vl = SQRT(vhx * vhx + vhy * vhy);
    if (RE(vl) > 0.0)
        FN(consider)(&b, m, h, shift, vmax, vmax * vhx / vl, vmax * vhy / vl, vhx, vhy, 1);
    for (int k = 0; k < m; ++k) {
        /* boundary line: n_k.v = c_k */
        REAL c = h[k].nx * h[k].qx + h[k].ny * h[k].qy - shift;
        REAL t = c - (h[k].nx * vhx + h[k].ny * vhy);
        FN(consider)(&b, m, h, shift, vmax, vhx + t * h[k].nx, vhy + t * h[k].ny, vhx, vhy,
                     2 + 4 * k);
        REAL hh = vmax * vmax - c * c;
        if (RE(hh) >= 0.0) {
            REAL r = SQRT(hh);
            REAL dx = -h[k].ny, dy = h[k].nx;
            FN(consider)(&b, m, h, shift, vmax, c * h[k].nx + r * dx, c * h[k].ny + r * dy, vhx,
                         vhy, 3 + 4 * k);
            FN(consider)(&b, m, h, shift, vmax, c * h[k].nx - r * dx, c * h[k].ny - r * dy, vhx,
                         vhy, 4 + 4 * k);
        }
    }
    for (int k = 0; k < m; ++k) {
        REAL ck = h[k].nx * h[k].qx + h[k].ny * h[k].qy - shift;
        for (int l = k + 1; l < m; ++l) {
            REAL cl = h[l].nx * h[l].qx + h[l].ny * h[l].qy - shift;
            REAL det = h[k].nx * h[l].ny - h[k].ny * h[l].nx;
            if (RE(det) == 0.0) continue;
            REAL px = (ck * h[l].ny - cl * h[k].ny) / det;
            REAL py = (h[k].nx * cl - h[l].nx * ck) / det;
            FN(consider)(&b, m, h, shift, vmax, px, py, vhx, vhy, 100000 + 64 * k + l);
        }
    }
    if (which) *which = b.code;
    if (!b.found) return 0;
    *ox = b.bx;
    *oy = b.by;
    return 1;
}

/* largest violation max_k n_k.(q_k - v) */
static REAL FN(max_violation)(int m, const FN(halfplane_t) *h, REAL vx, REAL vy)
{
    REAL f = -INFINITY;
    for (int k = 0; k < m; ++k) {
        REAL s = h[k].nx * (h[k].qx - vx) + h[k].ny * (h[k].qy - vy);
        if (RE(s) > RE(f)) f = s;
    }
    return f;
}

static void FN(consider_mm)(int m, const FN(halfplane_t) *h, REAL vmax, REAL vx, REAL vy,
                            int *found, REAL *bf, REAL *bx, REAL *by, int code, int *bcode)
{
    if (!isfinite(RE(vx)) || !isfinite(RE(vy))) return;
    if (RE(vx * vx + vy * vy) > RE(vmax * vmax) * (1.0 + 1e-12) + 1e-12) return;
    REAL f = FN(max_violation)(m, h, vx, vy);
    if (!*found || RE(f) < RE(*bf)) { *found = 1; *bf = f; *bx = vx; *by = vy; *bcode = code; }
}

/*
 * d* = min over |v| <= vmax of max_k n_k.(q_k - v) (section 3: the velocity
 * that least penetrates the half-planes).  The minimum of this convex
 * piecewise-linear function over the disc sits where three pieces are equal,
 * where two pieces are equal on the circle, or on the circle at the point
 * that maximises a single n_k.v (v = vmax n_k); all are tried.  *which
 * (nullable) names the candidate that won: k for vmax n_k, 1000 + 2(64k + l)
 * (+1) for the two circle points of rows k < l, 1000000 + 64(64k + l) + p for
 * the triple k < l < p; -1 when m = 0.
 */
static REAL FN(min_max)(int m, const FN(halfplane_t) *h, REAL vmax, REAL *ox, REAL *oy,
                        int *which)
{
    int found = 0, code = -1;
    REAL bf = 0.0, bx = 0.0, by = 0.0;
    for (int k = 0; k < m; ++k)
        FN(consider_mm)(m, h, vmax, vmax * h[k].nx, vmax * h[k].ny, &found, &bf, &bx, &by, k,
                        &code);
    for (int k = 0; k < m; ++k) {
        REAL ck = h[k].nx * h[k].qx + h[k].ny * h[k].qy;
        for (int l = k + 1; l < m; ++l) {
            REAL cl = h[l].nx * h[l].qx + h[l].ny * h[l].qy;
            /* equal violation: (n_k - n_l).v = c_k - c_l */
            REAL ax = h[k].nx - h[l].nx, ay = h[k].ny - h[l].ny, c = ck - cl;
            REAL a2 = ax * ax + ay * ay;
            if (RE(a2) == 0.0) continue;
            REAL px = c * ax / a2, py = c * ay / a2;
            REAL hh = vmax * vmax - (px * px + py * py);
            if (RE(hh) < 0.0) continue;
            REAL r = SQRT(hh / a2);
            FN(consider_mm)(m, h, vmax, px - r * ay, py + r * ax, &found, &bf, &bx, &by,
                            1000 + 2 * (64 * k + l), &code);
            FN(consider_mm)(m, h, vmax, px + r * ay, py - r * ax, &found, &bf, &bx, &by,
                            1001 + 2 * (64 * k + l), &code);
            for (int p = l + 1; p < m; ++p) {
                REAL cp = h[p].nx * h[p].qx + h[p].ny * h[p].qy;
                /* n.v + t = c for the three pieces (Cramer's rule) */
                REAL a11 = h[k].nx, a12 = h[k].ny;
                REAL a21 = h[l].nx, a22 = h[l].ny;
                REAL a31 = h[p].nx, a32 = h[p].ny;
                REAL det = a11 * (a22 - a32) - a12 * (a21 - a31) + (a21 * a32 - a22 * a31);
                if (RE(det) == 0.0) continue;
                REAL dxn = ck * (a22 - a32) - a12 * (cl - cp) + (cl * a32 - a22 * cp);
                REAL dyn = a11 * (cl - cp) - ck * (a21 - a31) + (a21 * cp - cl * a31);
                FN(consider_mm)(m, h, vmax, dxn / det, dyn / det, &found, &bf, &bx, &by,
                                1000000 + 64 * (64 * k + l) + p, &code);
            }
        }
    }
    if (which) *which = code;
    *ox = bx;
    *oy = by;
    return found ? bf : (REAL)(-INFINITY);
}

/*
 * The velocity choice of one agent from its neighbours' relative positions
 * P[t] = x_j - x_i and velocities V[t] = v_i - v_j (section 3): build the
 * half-planes through v_i + u/2, project vhat; if nothing is permitted, find
 * the least penetration d* and project onto the half-planes relaxed by
 * d* + delta.  Returns 0 (projection feasible) or 1 (fallback).
 */
static int FN(choose)(int m, const REAL *Px, const REAL *Py, const REAL *Vx, const REAL *Vy,
                      const REAL *Rs, const int *first, REAL vix, REAL viy, REAL tau, REAL dt,
                      REAL vmax, REAL vhx, REAL vhy, REAL *ox, REAL *oy, REAL *dstar,
                      FN(halfplane_t) *h, int32_t *branch, int *codes)
{
    /* codes (nullable, 3): the winning candidate of the projection, of the
     * least penetration and of the relaxed projection (-1: not run) */
    int c0 = -1, c1 = -1, c2 = -1;
    for (int t = 0; t < m; ++t) {
        REAL ux, uy, nx, ny;
        int code = FN(obstacle)(Px[t], Py[t], Vx[t], Vy[t], Rs[t], tau, dt, first[t], &ux, &uy,
                                &nx, &ny);
        if (branch) branch[t] = code;
        h[t].qx = vix + 0.5 * ux;
        h[t].qy = viy + 0.5 * uy;
        h[t].nx = nx;
        h[t].ny = ny;
    }
    if (FN(project)(m, h, 0.0, vmax, vhx, vhy, ox, oy, &c0)) {
        if (dstar) *dstar = NAN;
        if (codes) { codes[0] = c0; codes[1] = c1; codes[2] = c2; }
        return 0;
    }
    REAL mx, my;
    REAL d = FN(min_max)(m, h, vmax, &mx, &my, &c1);
    if (dstar) *dstar = d;
    if (!FN(project)(m, h, d + ORC_DELTA, vmax, vhx, vhy, ox, oy, &c2)) {
        *ox = mx;
        *oy = my;
    }
    if (codes) { codes[0] = c0; codes[1] = c1; codes[2] = c2; }
    return 1;
}
