/*
 * orca_oracle.c -- plain, slow CPU reference for the ORCA velocity-selection step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's library.  The GPU library
 * shares no code with it.
 *
 * Everything is double precision except the neighbour-selection distance,
 * which is taken in float32 exactly as the GPU kernel takes it (a floating-point
 * value decides an integer set there, so both sides decide in the same
 * precision).  Inputs are float32 arrays converted exactly to double.
 *
 * What each part follows (Charlton et al., "Fast Simulation of Crowd Collision
 * Avoidance"):
 *   - neighbours: section 3, Fig. 2 -- people read messages from their own and
 *     neighbouring spatial bins and keep those inside the observation radius;
 *     the neighbour cap K is the memory remedy named in section 5.  Two
 *     versions: the definition (scan all agents) and the paper's binned read.
 *   - half-plane: section 3, Fig. 1(b)-(c) -- the velocity obstacle for
 *     look-ahead tau, the shortest vector u from the relative velocity to its
 *     boundary, and the half-plane ORCA through v_opt + u/2 with normal along u
 *     (each agent takes half of the avoidance, section 2 on reciprocal models).
 *   - 2D LP: section 3 -- the permitted velocity closest to the preferred one,
 *     inside the max-speed disc.  This is the Euclidean projection onto
 *     disc ∩ half-planes, written out by its definition: enumerate every point
 *     where the optimum can sit and keep the closest feasible one.
 *   - fallback: section 3 -- when the half-planes leave no velocity, pick the
 *     one that least penetrates them: d* = min over the disc of the largest
 *     violation; then, among velocities within d* + delta of that, the one
 *     closest to the preferred velocity.
 *   - step: synchronous update of all agents, then x += dt v'; goal steering
 *     points the preferred velocity at the goal at walking speed (section 4).
 *
 * Parity status: the overlap branch (pairs already in contact use dt in place
 * of tau) and the lexicographic fallback are readings of passages the paper
 * leaves open; no printed number fixes them ("parity unpinned" for those two
 * choices, pinned only by the invariants they satisfy).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_ARC 0
#define ORC_LEFT 1
#define ORC_RIGHT 2
#define ORC_OVERLAP 3

/* second-stage relaxation of the least-penetration fallback (m/s) */
#define ORC_DELTA 1e-5
/* feasibility tolerance of the enumerated candidates (m/s) */
#define ORC_TOL 1e-10

typedef struct {
    float radius, max_speed, neighbor_dist, time_horizon, dt, pref_speed;
    int32_t max_neighbors, pad;
} oracle_params;

typedef struct {
    double qx, qy, nx, ny;
} halfplane;

/* Threads the parallel loops use. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Neighbour selection                                                 */
/* ------------------------------------------------------------------ */

/* Squared distance in float32, every operation rounded on its own. */
float oracle_dist2_f32(float xi, float yi, float xj, float yj)
{
    float dx = xj - xi;
    float dy = yj - yi;
    float sx = dx * dx;
    float sy = dy * dy;
    return sx + sy;
}

typedef struct {
    float d2;
    int64_t id;
} cand_t;

static int cand_cmp(const void *a, const void *b)
{
    const cand_t *x = (const cand_t *)a, *y = (const cand_t *)b;
    if (x->d2 < y->d2) return -1;
    if (x->d2 > y->d2) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

/* Definition: all j != i of [lo,hi) with d2 < nd^2, ascending by (d2, j), first K. */
int oracle_knn_brute(int64_t n_total, const float *pos, int64_t lo, int64_t hi, int64_t i,
                     float nd, int32_t k, int64_t *ids, float *d2s)
{
    const float *x = pos, *y = pos + n_total;
    float nd2 = nd * nd;
    int64_t cap = 64, m = 0;
    cand_t *c = (cand_t *)malloc(sizeof(cand_t) * cap);
    for (int64_t j = lo; j < hi; ++j) {
        if (j == i) continue;
        float d2 = oracle_dist2_f32(x[i], y[i], x[j], y[j]);
        if (d2 < nd2) {
            if (m == cap) { cap *= 2; c = (cand_t *)realloc(c, sizeof(cand_t) * cap); }
            c[m].d2 = d2; c[m].id = j; ++m;
        }
    }
    qsort(c, (size_t)m, sizeof(cand_t), cand_cmp);
    int32_t out = (int32_t)(m < k ? m : k);
    for (int32_t t = 0; t < out; ++t) { ids[t] = c[t].id; if (d2s) d2s[t] = c[t].d2; }
    free(c);
    return out;
}

/* The paper's message binning: square bins of side >= nd, one list per bin. */
typedef struct {
    double x0, y0, cell;
    int64_t nx, ny;
    int64_t *start; /* nx*ny + 1 */
    int64_t *items; /* agent ids grouped by bin */
} bins_t;

static void bins_build(bins_t *b, int64_t n_total, const float *pos, int64_t lo, int64_t hi,
                       float nd)
{
    const float *x = pos, *y = pos + n_total;
    double mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
    for (int64_t j = lo; j < hi; ++j) {
        if (x[j] < mnx) mnx = x[j];
        if (x[j] > mxx) mxx = x[j];
        if (y[j] < mny) mny = y[j];
        if (y[j] > mxy) mxy = y[j];
    }
    if (hi <= lo) { mnx = mny = 0; mxx = mxy = 0; }
    b->cell = (double)nd * 1.001; /* a bin slightly wider than the radius */
    b->x0 = mnx; b->y0 = mny;
    b->nx = (int64_t)floor((mxx - mnx) / b->cell) + 1;
    b->ny = (int64_t)floor((mxy - mny) / b->cell) + 1;
    int64_t nc = b->nx * b->ny;
    b->start = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
    b->items = (int64_t *)malloc(sizeof(int64_t) * (size_t)(hi - lo + 1));
    int64_t *cellof = (int64_t *)malloc(sizeof(int64_t) * (size_t)(hi - lo + 1));
    for (int64_t j = lo; j < hi; ++j) {
        int64_t cx = (int64_t)floor(((double)x[j] - b->x0) / b->cell);
        int64_t cy = (int64_t)floor(((double)y[j] - b->y0) / b->cell);
        if (cx >= b->nx) cx = b->nx - 1;
        if (cy >= b->ny) cy = b->ny - 1;
        cellof[j - lo] = cy * b->nx + cx;
        b->start[cellof[j - lo] + 1]++;
    }
    for (int64_t c = 0; c < nc; ++c) b->start[c + 1] += b->start[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nc + 1));
    memcpy(fill, b->start, sizeof(int64_t) * (size_t)(nc + 1));
    for (int64_t j = lo; j < hi; ++j) b->items[fill[cellof[j - lo]]++] = j;
    free(fill);
    free(cellof);
}

static void bins_free(bins_t *b)
{
    free(b->start);
    free(b->items);
}

static int32_t knn_binned(const bins_t *b, int64_t n_total, const float *pos, int64_t i,
                          float nd, int32_t k, int64_t *ids, float *d2s)
{
    const float *x = pos, *y = pos + n_total;
    float nd2 = nd * nd;
    int64_t cx = (int64_t)floor(((double)x[i] - b->x0) / b->cell);
    int64_t cy = (int64_t)floor(((double)y[i] - b->y0) / b->cell);
    if (cx >= b->nx) cx = b->nx - 1;
    if (cy >= b->ny) cy = b->ny - 1;
    int64_t cap = 64, m = 0;
    cand_t *c = (cand_t *)malloc(sizeof(cand_t) * cap);
    for (int64_t by = cy - 1; by <= cy + 1; ++by) {
        if (by < 0 || by >= b->ny) continue;
        for (int64_t bx = cx - 1; bx <= cx + 1; ++bx) {
            if (bx < 0 || bx >= b->nx) continue;
            int64_t cell = by * b->nx + bx;
            for (int64_t t = b->start[cell]; t < b->start[cell + 1]; ++t) {
                int64_t j = b->items[t];
                if (j == i) continue;
                float d2 = oracle_dist2_f32(x[i], y[i], x[j], y[j]);
                if (d2 < nd2) {
                    if (m == cap) { cap *= 2; c = (cand_t *)realloc(c, sizeof(cand_t) * cap); }
                    c[m].d2 = d2; c[m].id = j; ++m;
                }
            }
        }
    }
    qsort(c, (size_t)m, sizeof(cand_t), cand_cmp);
    int32_t out = (int32_t)(m < k ? m : k);
    for (int32_t t = 0; t < out; ++t) { ids[t] = c[t].id; if (d2s) d2s[t] = c[t].d2; }
    free(c);
    return out;
}

/* Binned neighbour lists of every agent of one scene: ids [hi-lo, k], -1 padded. */
void oracle_knn_binned_scene(int64_t n_total, const float *pos, int64_t lo, int64_t hi,
                             float nd, int32_t k, int64_t *ids)
{
    bins_t b;
    bins_build(&b, n_total, pos, lo, hi, nd);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = lo; i < hi; ++i) {
        int64_t *row = ids + (i - lo) * k;
        int32_t got = knn_binned(&b, n_total, pos, i, nd, k, row, NULL);
        for (int32_t t = got; t < k; ++t) row[t] = -1;
    }
    bins_free(&b);
}

/* ------------------------------------------------------------------ */
/* Half-plane of one neighbour (Fig. 1)                                */
/* ------------------------------------------------------------------ */

/*
 * P = x_j - x_i, V = v_i - v_j, R = r_i + r_j.  The velocity obstacle for
 * look-ahead tau is the set of relative velocities that bring the pair closer
 * than R at some t in (0, tau]: a cone from the origin tangent to the disc
 * D(P, R), cut off by the disc D(P/tau, R/tau).  u runs from V to the closest
 * boundary point and n is the outward normal there.  Pairs already closer
 * than R use dt in place of tau (they must separate within one step).
 * Returns the branch code.
 */
int oracle_halfplane(double Px, double Py, double Vx, double Vy, double R, double tau,
                     double dt, int i_before_j, double *ux, double *uy, double *nx,
                     double *ny)
{
    double dist2 = Px * Px + Py * Py;
    double R2 = R * R;
    if (dist2 > R2) {
        /* w: from the centre of the cut-off disc to V */
        double wx = Vx - Px / tau, wy = Vy - Py / tau;
        double w2 = wx * wx + wy * wy;
        double wP = wx * Px + wy * Py;
        if (wP < 0.0 && wP * wP > R2 * w2) {
            /* V faces the cut-off arc: nearest boundary point is on the circle */
            double wl = sqrt(w2);
            *nx = wx / wl;
            *ny = wy / wl;
            *ux = (R / tau - wl) * *nx;
            *uy = (R / tau - wl) * *ny;
            return ORC_ARC;
        }
        /* otherwise the nearest boundary point is on one of the two tangent legs */
        double L = sqrt(dist2 - R2);
        double lx, ly;
        int code;
        if (Px * wy - Py * wx > 0.0) {
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
        double s = Vx * lx + Vy * ly;
        *ux = s * lx - Vx;
        *uy = s * ly - Vy;
        return code;
    }
    /* already in contact: cut-off disc D(P/dt, R/dt) */
    double wx = Vx - Px / dt, wy = Vy - Py / dt;
    double wl = sqrt(wx * wx + wy * wy);
    if (wl > 0.0) {
        *nx = wx / wl;
        *ny = wy / wl;
    } else if (dist2 > 0.0) {
        double pl = sqrt(dist2);
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

/* ------------------------------------------------------------------ */
/* 2D LP by enumeration                                                */
/* ------------------------------------------------------------------ */

/* Feasible for every half-plane n.(v - q) >= -shift and inside the disc. */
static int feasible(int m, const halfplane *h, double shift, double vmax, double vx, double vy)
{
    if (vx * vx + vy * vy > vmax * vmax * (1.0 + 1e-12) + 1e-12) return 0;
    for (int k = 0; k < m; ++k) {
        double s = h[k].nx * (vx - h[k].qx) + h[k].ny * (vy - h[k].qy);
        if (s < -shift - ORC_TOL) return 0;
    }
    return 1;
}

typedef struct {
    int found;
    double bx, by, bd;
} best_t;

static void consider(best_t *b, int m, const halfplane *h, double shift, double vmax, double px,
                     double py, double vhx, double vhy)
{
    if (!isfinite(px) || !isfinite(py)) return;
    if (!feasible(m, h, shift, vmax, px, py)) return;
    double d = (px - vhx) * (px - vhx) + (py - vhy) * (py - vhy);
    if (!b->found || d < b->bd) { b->found = 1; b->bx = px; b->by = py; b->bd = d; }
}

/*
 * argmin |v - vhat| over the disc |v| <= vmax and the half-planes
 * n_k.(v - q_k) >= -shift.  The minimiser of a strictly convex function over
 * this set is vhat itself, the radial clip of vhat, the projection of vhat
 * onto one boundary line, a line-circle crossing, or a line-line crossing;
 * all of them are tried.  Returns 1 and writes the minimiser if the set is
 * non-empty, else 0.
 */
int oracle_project(int m, const halfplane *h, double shift, double vmax, double vhx, double vhy,
                   double *ox, double *oy)
{
    best_t b = {0, 0.0, 0.0, 0.0};
    consider(&b, m, h, shift, vmax, vhx, vhy, vhx, vhy);
    double vl = sqrt(vhx * vhx + vhy * vhy);
    if (vl > 0.0) consider(&b, m, h, shift, vmax, vmax * vhx / vl, vmax * vhy / vl, vhx, vhy);
    for (int k = 0; k < m; ++k) {
        /* boundary line: n_k.v = c_k */
        double c = h[k].nx * h[k].qx + h[k].ny * h[k].qy - shift;
        double t = c - (h[k].nx * vhx + h[k].ny * vhy);
        consider(&b, m, h, shift, vmax, vhx + t * h[k].nx, vhy + t * h[k].ny, vhx, vhy);
        double hh = vmax * vmax - c * c;
        if (hh >= 0.0) {
            double r = sqrt(hh);
            double dx = -h[k].ny, dy = h[k].nx;
            consider(&b, m, h, shift, vmax, c * h[k].nx + r * dx, c * h[k].ny + r * dy, vhx, vhy);
            consider(&b, m, h, shift, vmax, c * h[k].nx - r * dx, c * h[k].ny - r * dy, vhx, vhy);
        }
    }
    for (int k = 0; k < m; ++k) {
        double ck = h[k].nx * h[k].qx + h[k].ny * h[k].qy - shift;
        for (int l = k + 1; l < m; ++l) {
            double cl = h[l].nx * h[l].qx + h[l].ny * h[l].qy - shift;
            double det = h[k].nx * h[l].ny - h[k].ny * h[l].nx;
            if (det == 0.0) continue;
            double px = (ck * h[l].ny - cl * h[k].ny) / det;
            double py = (h[k].nx * cl - h[l].nx * ck) / det;
            consider(&b, m, h, shift, vmax, px, py, vhx, vhy);
        }
    }
    if (!b.found) return 0;
    *ox = b.bx;
    *oy = b.by;
    return 1;
}

/* largest violation max_k n_k.(q_k - v) */
static double max_violation(int m, const halfplane *h, double vx, double vy)
{
    double f = -INFINITY;
    for (int k = 0; k < m; ++k) {
        double s = h[k].nx * (h[k].qx - vx) + h[k].ny * (h[k].qy - vy);
        if (s > f) f = s;
    }
    return f;
}

static void consider_mm(int m, const halfplane *h, double vmax, double vx, double vy, int *found,
                        double *bf, double *bx, double *by)
{
    if (!isfinite(vx) || !isfinite(vy)) return;
    if (vx * vx + vy * vy > vmax * vmax * (1.0 + 1e-12) + 1e-12) return;
    double f = max_violation(m, h, vx, vy);
    if (!*found || f < *bf) { *found = 1; *bf = f; *bx = vx; *by = vy; }
}

/*
 * d* = min over |v| <= vmax of max_k n_k.(q_k - v).  The minimum of this
 * convex piecewise-linear function over the disc sits where three pieces are
 * equal, where two pieces are equal on the circle, or on the circle at the
 * point that maximises a single n_k.v (v = vmax n_k); all are tried.
 */
double oracle_min_max(int m, const halfplane *h, double vmax, double *ox, double *oy)
{
    int found = 0;
    double bf = 0.0, bx = 0.0, by = 0.0;
    for (int k = 0; k < m; ++k)
        consider_mm(m, h, vmax, vmax * h[k].nx, vmax * h[k].ny, &found, &bf, &bx, &by);
    for (int k = 0; k < m; ++k) {
        double ck = h[k].nx * h[k].qx + h[k].ny * h[k].qy;
        for (int l = k + 1; l < m; ++l) {
            double cl = h[l].nx * h[l].qx + h[l].ny * h[l].qy;
            /* equal violation: (n_k - n_l).v = c_k - c_l */
            double ax = h[k].nx - h[l].nx, ay = h[k].ny - h[l].ny, c = ck - cl;
            double a2 = ax * ax + ay * ay;
            if (a2 == 0.0) continue;
            double px = c * ax / a2, py = c * ay / a2;
            double hh = vmax * vmax - (px * px + py * py);
            if (hh < 0.0) continue;
            double r = sqrt(hh / a2);
            consider_mm(m, h, vmax, px - r * ay, py + r * ax, &found, &bf, &bx, &by);
            consider_mm(m, h, vmax, px + r * ay, py - r * ax, &found, &bf, &bx, &by);
            for (int p = l + 1; p < m; ++p) {
                double cp = h[p].nx * h[p].qx + h[p].ny * h[p].qy;
                /* n.v + t = c for the three pieces (Cramer's rule) */
                double a11 = h[k].nx, a12 = h[k].ny;
                double a21 = h[l].nx, a22 = h[l].ny;
                double a31 = h[p].nx, a32 = h[p].ny;
                double det = a11 * (a22 - a32) - a12 * (a21 - a31) + (a21 * a32 - a22 * a31);
                if (det == 0.0) continue;
                double dxn = ck * (a22 - a32) - a12 * (cl - cp) + (cl * a32 - a22 * cp);
                double dyn = a11 * (cl - cp) - ck * (a21 - a31) + (a21 * cp - cl * a31);
                consider_mm(m, h, vmax, dxn / det, dyn / det, &found, &bf, &bx, &by);
            }
        }
    }
    *ox = bx;
    *oy = by;
    return found ? bf : -INFINITY;
}

/* ------------------------------------------------------------------ */
/* One agent                                                           */
/* ------------------------------------------------------------------ */

/* Preferred velocity toward the goal at walking speed s, stopping on arrival. */
void oracle_steer(double px, double py, double gx, double gy, double s, double dt, double *vx,
                  double *vy)
{
    double ex = gx - px, ey = gy - py;
    double el = sqrt(ex * ex + ey * ey);
    if (el > s * dt) {
        *vx = s * ex / el;
        *vy = s * ey / el;
    } else {
        *vx = ex / dt;
        *vy = ey / dt;
    }
}

/*
 * New velocity of agent i given its neighbour list.  Writes the half-planes
 * (if hp_out), returns status 0 (2D LP feasible) or 1 (fallback).
 */
int oracle_agent_velocity(int64_t n_total, const float *pos, const float *vel, const float *rad,
                          const oracle_params *p, int64_t i, int32_t m, const int64_t *nbr,
                          double vhx, double vhy, double *ox, double *oy, double *dstar,
                          halfplane *hp_out, int32_t *branch_out)
{
    const float *x = pos, *y = pos + n_total;
    const float *vx = vel, *vy = vel + n_total;
    halfplane hbuf[64];
    halfplane *h = hp_out ? hp_out : hbuf;
    double vmax = p->max_speed;
    for (int32_t t = 0; t < m; ++t) {
        int64_t j = nbr[t];
        double Px = (double)x[j] - (double)x[i], Py = (double)y[j] - (double)y[i];
        double Vx = (double)vx[i] - (double)vx[j], Vy = (double)vy[i] - (double)vy[j];
        double ri = rad ? (double)rad[i] : (double)p->radius;
        double rj = rad ? (double)rad[j] : (double)p->radius;
        double ux, uy, nx, ny;
        int code = oracle_halfplane(Px, Py, Vx, Vy, ri + rj, p->time_horizon, p->dt, i < j,
                                    &ux, &uy, &nx, &ny);
        if (branch_out) branch_out[t] = code;
        h[t].qx = (double)vx[i] + 0.5 * ux;
        h[t].qy = (double)vy[i] + 0.5 * uy;
        h[t].nx = nx;
        h[t].ny = ny;
    }
    if (oracle_project(m, h, 0.0, vmax, vhx, vhy, ox, oy)) {
        if (dstar) *dstar = NAN;
        return 0;
    }
    double mx, my;
    double d = oracle_min_max(m, h, vmax, &mx, &my);
    if (dstar) *dstar = d;
    if (!oracle_project(m, h, d + ORC_DELTA, vmax, vhx, vhy, ox, oy)) {
        *ox = mx;
        *oy = my;
    }
    return 1;
}

static int scene_of(int32_t n_scenes, const int64_t *off, int64_t i)
{
    int lo = 0, hi = n_scenes - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

/*
 * New velocities of the listed agents from one state.  neighbor_mode 0 scans
 * every agent of the scene (the definition), 1 reads the 3x3 bins.
 * Outputs per listed agent: new_vel [n_agents,2], vhat [n_agents,2],
 * nbr [n_agents,kcap] (-1 padded), n_nbr, status, dstar.
 */
void oracle_velocities(int64_t n_total, const float *pos, const float *vel, const float *pref,
                       const float *goals, const float *rad, int32_t n_scenes,
                       const int64_t *offsets, const oracle_params *params,
                       const int64_t *agents, int64_t n_agents, int32_t neighbor_mode,
                       int32_t kcap, double *new_vel, double *vhat, int64_t *nbr,
                       int32_t *n_nbr, uint8_t *status, double *dstar)
{
    bins_t *bins = NULL;
    if (neighbor_mode == 1) {
        bins = (bins_t *)calloc((size_t)n_scenes, sizeof(bins_t));
        for (int s = 0; s < n_scenes; ++s)
            bins_build(&bins[s], n_total, pos, offsets[s], offsets[s + 1],
                       params[s].neighbor_dist);
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t a = 0; a < n_agents; ++a) {
        int64_t i = agents ? agents[a] : a;
        int s = scene_of(n_scenes, offsets, i);
        const oracle_params *p = &params[s];
        int64_t ids[64];
        int32_t m;
        if (neighbor_mode == 1)
            m = knn_binned(&bins[s], n_total, pos, i, p->neighbor_dist, p->max_neighbors, ids,
                           NULL);
        else
            m = oracle_knn_brute(n_total, pos, offsets[s], offsets[s + 1], i, p->neighbor_dist,
                                 p->max_neighbors, ids, NULL);
        double vhx, vhy;
        if (goals)
            oracle_steer(pos[i], pos[n_total + i], goals[i], goals[n_total + i], p->pref_speed,
                         p->dt, &vhx, &vhy);
        else {
            vhx = pref[i];
            vhy = pref[n_total + i];
        }
        double ox, oy, d;
        int st = oracle_agent_velocity(n_total, pos, vel, rad, p, i, m, ids, vhx, vhy, &ox, &oy,
                                       &d, NULL, NULL);
        new_vel[2 * a] = ox;
        new_vel[2 * a + 1] = oy;
        if (vhat) { vhat[2 * a] = vhx; vhat[2 * a + 1] = vhy; }
        if (nbr)
            for (int32_t t = 0; t < kcap; ++t) nbr[a * kcap + t] = t < m ? ids[t] : -1;
        if (n_nbr) n_nbr[a] = m;
        if (status) status[a] = (uint8_t)st;
        if (dstar) dstar[a] = d;
    }
    if (bins) {
        for (int s = 0; s < n_scenes; ++s) bins_free(&bins[s]);
        free(bins);
    }
}

/*
 * n_steps synchronous steps of every agent, state in float32 as the GPU keeps
 * it: v' from the current state, then x <- f32(x + dt v'), v <- f32(v').  With
 * goals the preferred velocity is re-aimed at the goal at the start of every
 * step (and written to pref); without, pref is held fixed.
 */
void oracle_step(int64_t n_total, float *pos, float *vel, float *pref, const float *goals,
                 const float *rad, int32_t n_scenes, const int64_t *offsets,
                 const oracle_params *params, int32_t n_steps, uint8_t *status_last)
{
    double *nv = (double *)malloc(sizeof(double) * 2 * (size_t)n_total);
    double *vh = (double *)malloc(sizeof(double) * 2 * (size_t)n_total);
    for (int32_t step = 0; step < n_steps; ++step) {
        oracle_velocities(n_total, pos, vel, pref, goals, rad, n_scenes, offsets, params, NULL,
                          n_total, 1, 1, nv, vh, NULL, NULL,
                          step == n_steps - 1 ? status_last : NULL, NULL);
        for (int64_t i = 0; i < n_total; ++i) {
            int s = scene_of(n_scenes, offsets, i);
            double dt = params[s].dt;
            pos[i] = (float)((double)pos[i] + dt * nv[2 * i]);
            pos[n_total + i] = (float)((double)pos[n_total + i] + dt * nv[2 * i + 1]);
            vel[i] = (float)nv[2 * i];
            vel[n_total + i] = (float)nv[2 * i + 1];
            if (goals) {
                pref[i] = (float)vh[2 * i];
                pref[n_total + i] = (float)vh[2 * i + 1];
            }
        }
    }
    free(nv);
    free(vh);
}
