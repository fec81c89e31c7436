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
#include <complex.h>
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

/*
 * Optional per-agent properties (section 4, the crossing whose people differ
 * in size and speed): radius, max speed and walking speed, each an array over
 * all agents or NULL for the scene's value.  A pair's combined radius is
 * r_i + r_j.
 */
typedef struct {
    const float *radius, *max_speed, *pref_speed;
    const uint8_t *present; /* 0: the agent is not in the simulation (not spawned or removed) */
} oracle_agents;

static int ag_present(const oracle_agents *ag, int64_t j)
{
    return !(ag && ag->present) || ag->present[j] != 0;
}

static double ag_radius(const oracle_agents *ag, const oracle_params *p, int64_t i)
{
    return ag && ag->radius ? (double)ag->radius[i] : (double)p->radius;
}

static double ag_vmax(const oracle_agents *ag, const oracle_params *p, int64_t i)
{
    return ag && ag->max_speed ? (double)ag->max_speed[i] : (double)p->max_speed;
}

static double ag_speed(const oracle_agents *ag, const oracle_params *p, int64_t i)
{
    return ag && ag->pref_speed ? (double)ag->pref_speed[i] : (double)p->pref_speed;
}


/* Threads the parallel loops use. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Use n threads in later calls from this thread (n <= 0: one per processor). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
    (void)n;
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

/* Definition: all present j != i of [lo,hi) with d2 < nd^2, ascending by (d2, j), first K. */
static int knn_brute_mask(int64_t n_total, const float *pos, int64_t lo, int64_t hi, int64_t i,
                          float nd, int32_t k, int64_t *ids, float *d2s, const uint8_t *present)
{
    const float *x = pos, *y = pos + n_total;
    float nd2 = nd * nd;
    int64_t cap = 64, m = 0;
    cand_t *c = (cand_t *)malloc(sizeof(cand_t) * cap);
    for (int64_t j = lo; j < hi; ++j) {
        if (j == i || (present && !present[j])) continue;
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

int oracle_knn_brute(int64_t n_total, const float *pos, int64_t lo, int64_t hi, int64_t i,
                     float nd, int32_t k, int64_t *ids, float *d2s)
{
    return knn_brute_mask(n_total, pos, lo, hi, i, nd, k, ids, d2s, NULL);
}

/* The paper's message binning: square bins of side >= nd, one list per bin. */
typedef struct {
    double x0, y0, cell;
    int64_t nx, ny;
    int64_t *start; /* nx*ny + 1 */
    int64_t *items; /* agent ids grouped by bin */
} bins_t;

static void bins_build(bins_t *b, int64_t n_total, const float *pos, int64_t lo, int64_t hi,
                       float nd, const uint8_t *present)
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
        if (present && !present[j]) { cellof[j - lo] = -1; continue; }
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
    for (int64_t j = lo; j < hi; ++j)
        if (cellof[j - lo] >= 0) b->items[fill[cellof[j - lo]]++] = j;
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
    bins_build(&b, n_total, pos, lo, hi, nd, NULL);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = lo; i < hi; ++i) {
        int64_t *row = ids + (i - lo) * k;
        int32_t got = knn_binned(&b, n_total, pos, i, nd, k, row, NULL);
        for (int32_t t = got; t < k; ++t) row[t] = -1;
    }
    bins_free(&b);
}

/* ------------------------------------------------------------------ */
/* Geometry and programs: the core, once in double, once complex-step  */
/* ------------------------------------------------------------------ */

#define REAL double
#define FN(x) x
#define RE(x) (x)
#define SQRT(x) sqrt(x)
#include "orca_oracle_core.h"
#undef REAL
#undef FN
#undef RE
#undef SQRT

#define REAL double complex
#define FN(x) x##_cx
#define RE(x) creal(x)
#define SQRT(x) csqrt(x)
#include "orca_oracle_core.h"
#undef REAL
#undef FN
#undef RE
#undef SQRT

typedef halfplane_t halfplane;

/* Half-plane of one neighbour; see obstacle() in orca_oracle_core.h. */
int oracle_halfplane(double Px, double Py, double Vx, double Vy, double R, double tau,
                     double dt, int i_before_j, double *ux, double *uy, double *nx,
                     double *ny)
{
    return obstacle(Px, Py, Vx, Vy, R, tau, dt, i_before_j, ux, uy, nx, ny);
}

/* The 2D program by enumeration; see project(). */
int oracle_project(int m, const halfplane *h, double shift, double vmax, double vhx, double vhy,
                   double *ox, double *oy)
{
    return project(m, h, shift, vmax, vhx, vhy, ox, oy, NULL);
}

/* The least penetration by enumeration; see min_max(). */
double oracle_min_max(int m, const halfplane *h, double vmax, double *ox, double *oy)
{
    return min_max(m, h, vmax, ox, oy, NULL);
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
int oracle_agent_velocity(int64_t n_total, const float *pos, const float *vel,
                          const oracle_agents *ag, const oracle_params *p, int64_t i, int32_t m,
                          const int64_t *nbr,
                          double vhx, double vhy, double *ox, double *oy, double *dstar,
                          halfplane *hp_out, int32_t *branch_out)
{
    const float *x = pos, *y = pos + n_total;
    const float *vx = vel, *vy = vel + n_total;
    halfplane hbuf[64];
    double Px[64], Py[64], Vx[64], Vy[64], Rs[64];
    int first[64];
    for (int32_t t = 0; t < m; ++t) {
        int64_t j = nbr[t];
        Px[t] = (double)x[j] - (double)x[i];
        Py[t] = (double)y[j] - (double)y[i];
        Vx[t] = (double)vx[i] - (double)vx[j];
        Vy[t] = (double)vy[i] - (double)vy[j];
        Rs[t] = ag_radius(ag, p, i) + ag_radius(ag, p, j);
        first[t] = i < j;
    }
    return choose(m, Px, Py, Vx, Vy, Rs, first, (double)vx[i], (double)vy[i], p->time_horizon,
                  p->dt, ag_vmax(ag, p, i), vhx, vhy, ox, oy, dstar, hp_out ? hp_out : hbuf,
                  branch_out, NULL);
}

/*
 * One agent's choice and its directional derivative (complex step, h =
 * 1e-30) along tangents of the neighbours' relative positions P [m,2] and
 * velocities V [m,2], the agent's own velocity, tau, vmax and vhat.  Combined
 * radii Rs [m] and index order first [m] are fixed.  out: v' (2), dv' (2),
 * d* (1), dd* (1).  Returns the status (0 projection, 1 fallback).
 */
int oracle_choice_jvp(int m, const double *P, const double *dP, const double *V, const double *dV,
                      const double *Rs, const int *first, double vix, double viy, double dvix,
                      double dviy, double tau, double dtau, double dt, double vmax, double dvmax,
                      double vhx, double vhy, double dvhx, double dvhy, double *out)
{
    const double h = 1e-30;
    double complex Px[64], Py[64], Vx[64], Vy[64], Rc[64];
    halfplane_t_cx hb[64];
    for (int t = 0; t < m; ++t) {
        Px[t] = P[2 * t] + I * h * dP[2 * t];
        Py[t] = P[2 * t + 1] + I * h * dP[2 * t + 1];
        Vx[t] = V[2 * t] + I * h * dV[2 * t];
        Vy[t] = V[2 * t + 1] + I * h * dV[2 * t + 1];
        Rc[t] = Rs[t];
    }
    double complex ox, oy, d;
    int st = choose_cx(m, Px, Py, Vx, Vy, Rc, first, vix + I * h * dvix, viy + I * h * dviy,
                       tau + I * h * dtau, dt, vmax + I * h * dvmax, vhx + I * h * dvhx,
                       vhy + I * h * dvhy, &ox, &oy, &d, hb, NULL, NULL);
    out[0] = creal(ox);
    out[1] = creal(oy);
    out[2] = cimag(ox) / h;
    out[3] = cimag(oy) / h;
    out[4] = creal(d);
    out[5] = st ? cimag(d) / h : 0.0;
    return st;
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
                       const float *goals, const oracle_agents *ag, int32_t n_scenes,
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
                       params[s].neighbor_dist, ag ? ag->present : NULL);
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t a = 0; a < n_agents; ++a) {
        int64_t i = agents ? agents[a] : a;
        int s = scene_of(n_scenes, offsets, i);
        const oracle_params *p = &params[s];
        int64_t ids[64];
        int32_t m;
        if (!ag_present(ag, i)) {
            /* not in the simulation: no velocity, status 2 */
            new_vel[2 * a] = new_vel[2 * a + 1] = 0.0;
            if (vhat) { vhat[2 * a] = vhat[2 * a + 1] = 0.0; }
            if (nbr)
                for (int32_t t = 0; t < kcap; ++t) nbr[a * kcap + t] = -1;
            if (n_nbr) n_nbr[a] = 0;
            if (status) status[a] = 2;
            if (dstar) dstar[a] = 0.0;
            continue;
        }
        if (neighbor_mode == 1)
            m = knn_binned(&bins[s], n_total, pos, i, p->neighbor_dist, p->max_neighbors, ids,
                           NULL);
        else
            m = knn_brute_mask(n_total, pos, offsets[s], offsets[s + 1], i, p->neighbor_dist,
                               p->max_neighbors, ids, NULL, ag ? ag->present : NULL);
        double vhx, vhy;
        if (goals)
            oracle_steer(pos[i], pos[n_total + i], goals[i], goals[n_total + i],
                         ag_speed(ag, p, i), p->dt, &vhx, &vhy);
        else {
            vhx = pref[i];
            vhy = pref[n_total + i];
        }
        double ox, oy, d;
        int st = oracle_agent_velocity(n_total, pos, vel, ag, p, i, m, ids, vhx, vhy, &ox, &oy,
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
                 const oracle_agents *ag, int32_t n_scenes, const int64_t *offsets,
                 const oracle_params *params, int32_t n_steps, uint8_t *status_last)
{
    double *nv = (double *)malloc(sizeof(double) * 2 * (size_t)n_total);
    double *vh = (double *)malloc(sizeof(double) * 2 * (size_t)n_total);
    for (int32_t step = 0; step < n_steps; ++step) {
        oracle_velocities(n_total, pos, vel, pref, goals, ag, n_scenes, offsets, params, NULL,
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

/*
 * Steps with spawning and removal (section 4: people enter their start
 * region at a spawn time and are removed once they reach their goal).  At
 * step t (t0, t0 + 1, ...) agent i is in the simulation if spawn_step[i] <= t
 * and state[i] == 0; only those agents see each other, move and are steered.
 * After the step an agent whose goal lies within its own radius of its new
 * float32 position is removed (state 1).  The decision is taken in float64 on
 * the float32 coordinates, each operation rounded on its own.
 */
void oracle_life_step(int64_t n_total, float *pos, float *vel, float *pref, const float *goals,
                      const oracle_agents *ag_in, int32_t n_scenes, const int64_t *offsets,
                      const oracle_params *params, int32_t n_steps, const int32_t *spawn_step,
                      uint8_t *state, int32_t t0, uint8_t *status_last)
{
    uint8_t *present = (uint8_t *)malloc((size_t)(n_total ? n_total : 1));
    double *nv = (double *)malloc(sizeof(double) * 2 * (size_t)(n_total ? n_total : 1));
    double *vh = (double *)malloc(sizeof(double) * 2 * (size_t)(n_total ? n_total : 1));
    oracle_agents ag = {NULL, NULL, NULL, present};
    if (ag_in) {
        ag.radius = ag_in->radius;
        ag.max_speed = ag_in->max_speed;
        ag.pref_speed = ag_in->pref_speed;
    }
    for (int32_t step = 0; step < n_steps; ++step) {
        const int32_t t = t0 + step;
        for (int64_t i = 0; i < n_total; ++i)
            present[i] = (uint8_t)(spawn_step[i] <= t && state[i] == 0);
        oracle_velocities(n_total, pos, vel, pref, goals, &ag, n_scenes, offsets, params, NULL,
                          n_total, 1, 1, nv, vh, NULL, NULL,
                          step == n_steps - 1 ? status_last : NULL, NULL);
        for (int64_t i = 0; i < n_total; ++i) {
            if (!present[i]) continue;
            const int s = scene_of(n_scenes, offsets, i);
            const oracle_params *p = &params[s];
            const double dt = p->dt;
            pos[i] = (float)((double)pos[i] + dt * nv[2 * i]);
            pos[n_total + i] = (float)((double)pos[n_total + i] + dt * nv[2 * i + 1]);
            vel[i] = (float)nv[2 * i];
            vel[n_total + i] = (float)nv[2 * i + 1];
            pref[i] = (float)vh[2 * i];
            pref[n_total + i] = (float)vh[2 * i + 1];
            const double ex = (double)goals[i] - (double)pos[i];
            const double ey = (double)goals[n_total + i] - (double)pos[n_total + i];
            const double sx = ex * ex;
            const double sy = ey * ey;
            const double r = ag_radius(&ag, p, i);
            if (sx + sy <= r * r) state[i] = 1;
        }
    }
    free(present);
    free(nv);
    free(vh);
}

/* ------------------------------------------------------------------ */
/* Gradients (forward mode by complex step) and float64 trajectories   */
/* ------------------------------------------------------------------ */

/*
 * One synchronous step of every agent in REAL arithmetic: fixed preferred
 * velocities pref, per-scene vmax_s and tau_s (REAL leaves), neighbours from
 * the binned read of float32(RE(pos)) (the float32 decision the GPU takes).
 * x <- x + dt v', v <- v'.  Written out for both scalar types below.
 */
#define DEFINE_TRAJ_STEP(R_T, SUF, RE_, FIRST_CHOOSE)                                           \
    static void traj_step##SUF(int64_t n, R_T *pos, R_T *vel, const R_T *pref, int32_t n_scenes,  \
                               const int64_t *off, const oracle_params *par, const R_T *vmax_s,   \
                               const R_T *tau_s, const oracle_agents *ag, uint64_t *ahash)        \
    {                                                                                             \
        float *p32 = (float *)malloc(sizeof(float) * 2 * (size_t)(n ? n : 1));                   \
        R_T *nv = (R_T *)malloc(sizeof(R_T) * 2 * (size_t)(n ? n : 1));                           \
        for (int64_t i = 0; i < 2 * n; ++i) p32[i] = (float)RE_(pos[i]);                          \
        bins_t *bins = (bins_t *)calloc((size_t)n_scenes, sizeof(bins_t));                        \
        for (int s = 0; s < n_scenes; ++s)                                                        \
            bins_build(&bins[s], n, p32, off[s], off[s + 1], par[s].neighbor_dist, NULL);         \
        _Pragma("omp parallel for schedule(dynamic, 16)")                                         \
        for (int64_t i = 0; i < n; ++i) {                                                         \
            int s = scene_of(n_scenes, off, i);                                                   \
            const oracle_params *p = &par[s];                                                     \
            int64_t ids[64];                                                                      \
            int32_t m = knn_binned(&bins[s], n, p32, i, p->neighbor_dist, p->max_neighbors, ids,  \
                                   NULL);                                                         \
            R_T Px[64], Py[64], Vx[64], Vy[64], Rs[64];                                           \
            int first[64];                                                                        \
            for (int32_t t = 0; t < m; ++t) {                                                     \
                int64_t j = ids[t];                                                               \
                Px[t] = pos[j] - pos[i];                                                          \
                Py[t] = pos[n + j] - pos[n + i];                                                  \
                Vx[t] = vel[i] - vel[j];                                                          \
                Vy[t] = vel[n + i] - vel[n + j];                                                  \
                Rs[t] = ag_radius(ag, p, i) + ag_radius(ag, p, j);                                \
                first[t] = i < j;                                                                 \
            }                                                                                     \
            /* a per-agent max speed is a constant; the scene's is the leaf */                    \
            const R_T vmax_i = ag && ag->max_speed ? (R_T)ag->max_speed[i] : vmax_s[s];           \
            int32_t branch[64];                                                                   \
            int codes[3];                                                                         \
            int status;                                                                           \
            FIRST_CHOOSE;                                                                         \
            if (ahash) ahash[i] = decisions_hash(m, ids, branch, status, codes);                  \
        }                                                                                         \
        for (int64_t i = 0; i < n; ++i) {                                                         \
            double dt = par[scene_of(n_scenes, off, i)].dt;                                       \
            pos[i] = pos[i] + dt * nv[2 * i];                                                     \
            pos[n + i] = pos[n + i] + dt * nv[2 * i + 1];                                         \
            vel[i] = nv[2 * i];                                                                   \
            vel[n + i] = nv[2 * i + 1];                                                           \
        }                                                                                         \
        for (int s = 0; s < n_scenes; ++s) bins_free(&bins[s]);                                   \
        free(bins);                                                                               \
        free(nv);                                                                                 \
        free(p32);                                                                                \
    }

/*
 * Every discrete decision of one agent's step, folded into 64 bits: the
 * neighbour list, each half-plane's branch, feasibility and the candidate
 * that won each program.  Two steps whose hashes agree took the same branch
 * of the piecewise-smooth step map (up to a hash collision).
 */
static uint64_t tape_mix(uint64_t h, uint64_t x)
{
    uint64_t z = h ^ (x * 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

static uint64_t decisions_hash(int32_t m, const int64_t *ids, const int32_t *branch, int status,
                               const int *codes)
{
    uint64_t h = tape_mix(0x243f6a8885a308d3ull, (uint64_t)m);
    for (int32_t t = 0; t < m; ++t)
        h = tape_mix(h, ((uint64_t)ids[t] << 8) | (uint64_t)(branch[t] & 0xff));
    h = tape_mix(h, (uint64_t)status);
    for (int c = 0; c < 3; ++c) h = tape_mix(h, (uint64_t)(int64_t)codes[c]);
    return h;
}

DEFINE_TRAJ_STEP(double, _d, (double), {
    halfplane hb[64];
    status = choose(m, Px, Py, Vx, Vy, Rs, first, vel[i], vel[n + i], tau_s[s], p->dt, vmax_i,
                    pref[i], pref[n + i], &nv[2 * i], &nv[2 * i + 1], NULL, hb, branch, codes);
})

DEFINE_TRAJ_STEP(double complex, _c, creal, {
    halfplane_t_cx hb[64];
    status = choose_cx(m, Px, Py, Vx, Vy, Rs, first, vel[i], vel[n + i], tau_s[s], p->dt,
                       vmax_i, pref[i], pref[n + i], &nv[2 * i], &nv[2 * i + 1], NULL, hb, branch,
                       codes);
})

/*
 * Loss L = sum_i |x_i(T) - y_i|^2 after n_steps float64 steps from
 * (pos0, vel0) with fixed preferred velocities pref and per-scene vmax_s,
 * tau_s.  Used for central finite differences.
 */
double oracle_traj_loss(int64_t n, const double *pos0, const double *vel0, const double *pref,
                        int32_t n_scenes, const int64_t *off, const oracle_params *par,
                        const double *vmax_s, const double *tau_s, int32_t n_steps,
                        const double *targets, const oracle_agents *ag)
{
    double *pos = (double *)malloc(sizeof(double) * 2 * (size_t)n);
    double *vel = (double *)malloc(sizeof(double) * 2 * (size_t)n);
    memcpy(pos, pos0, sizeof(double) * 2 * (size_t)n);
    memcpy(vel, vel0, sizeof(double) * 2 * (size_t)n);
    for (int32_t t = 0; t < n_steps; ++t)
        traj_step_d(n, pos, vel, pref, n_scenes, off, par, vmax_s, tau_s, ag, NULL);
    double L = 0.0;
    for (int64_t i = 0; i < 2 * n; ++i) L += (pos[i] - targets[i]) * (pos[i] - targets[i]);
    free(pos);
    free(vel);
    return L;
}

/*
 * The same loss and its directional derivative along (dpref, dvmax, dtau) by
 * complex step (h = 1e-30): the discrete choices are those of the primal.
 * With f32_state the primal state is rounded to float32 after every step
 * (the tangent is not), which is the trajectory a float32-state step takes.
 */
void oracle_traj_jvp(int64_t n, const double *pos0, const double *vel0, const double *pref,
                     int32_t n_scenes, const int64_t *off, const oracle_params *par,
                     const double *vmax_s, const double *tau_s, int32_t n_steps,
                     const double *targets, const double *dpref, const double *dvmax,
                     const double *dtau, int32_t f32_state, const oracle_agents *ag,
                     double *loss, double *dloss)
{
    const double h = 1e-30;
    double complex *pos = (double complex *)malloc(sizeof(double complex) * 2 * (size_t)n);
    double complex *vel = (double complex *)malloc(sizeof(double complex) * 2 * (size_t)n);
    double complex *pr = (double complex *)malloc(sizeof(double complex) * 2 * (size_t)n);
    double complex *vm = (double complex *)malloc(sizeof(double complex) * (size_t)n_scenes);
    double complex *ta = (double complex *)malloc(sizeof(double complex) * (size_t)n_scenes);
    for (int64_t i = 0; i < 2 * n; ++i) {
        pos[i] = pos0[i];
        vel[i] = vel0[i];
        pr[i] = pref[i] + I * h * (dpref ? dpref[i] : 0.0);
    }
    for (int s = 0; s < n_scenes; ++s) {
        vm[s] = vmax_s[s] + I * h * (dvmax ? dvmax[s] : 0.0);
        ta[s] = tau_s[s] + I * h * (dtau ? dtau[s] : 0.0);
    }
    for (int32_t t = 0; t < n_steps; ++t) {
        traj_step_c(n, pos, vel, pr, n_scenes, off, par, vm, ta, ag, NULL);
        if (f32_state) /* keep the primal on float32 states (as the GPU stores them) */
            for (int64_t i = 0; i < 2 * n; ++i) {
                pos[i] = (double)(float)creal(pos[i]) + I * cimag(pos[i]);
                vel[i] = (double)(float)creal(vel[i]) + I * cimag(vel[i]);
            }
    }
    double complex L = 0.0;
    for (int64_t i = 0; i < 2 * n; ++i) L += (pos[i] - targets[i]) * (pos[i] - targets[i]);
    *loss = creal(L);
    *dloss = cimag(L) / h;
    free(pos);
    free(vel);
    free(pr);
    free(vm);
    free(ta);
}

/*
 * Tangent of one step from a float32 state along (dpos, dvel, dpref, dvmax,
 * dtau): dpos_out, dvel_out [2, n] (complex step).  The step is the float64
 * map x' = x + dt v', v' (no float32 rounding of the result).
 */
void oracle_step_jvp(int64_t n, const float *pos, const float *vel, const float *pref,
                     int32_t n_scenes, const int64_t *off, const oracle_params *par,
                     const double *dpos, const double *dvel, const double *dpref,
                     const double *dvmax, const double *dtau, const oracle_agents *ag,
                     double *dpos_out, double *dvel_out)
{
    const double h = 1e-30;
    double complex *p = (double complex *)malloc(sizeof(double complex) * 2 * (size_t)n);
    double complex *v = (double complex *)malloc(sizeof(double complex) * 2 * (size_t)n);
    double complex *pr = (double complex *)malloc(sizeof(double complex) * 2 * (size_t)n);
    double complex *vm = (double complex *)malloc(sizeof(double complex) * (size_t)n_scenes);
    double complex *ta = (double complex *)malloc(sizeof(double complex) * (size_t)n_scenes);
    for (int64_t i = 0; i < 2 * n; ++i) {
        p[i] = (double)pos[i] + I * h * dpos[i];
        v[i] = (double)vel[i] + I * h * dvel[i];
        pr[i] = (double)pref[i] + I * h * dpref[i];
    }
    for (int s = 0; s < n_scenes; ++s) {
        vm[s] = (double)par[s].max_speed + I * h * dvmax[s];
        ta[s] = (double)par[s].time_horizon + I * h * dtau[s];
    }
    traj_step_c(n, p, v, pr, n_scenes, off, par, vm, ta, ag, NULL);
    for (int64_t i = 0; i < 2 * n; ++i) {
        dpos_out[i] = cimag(p[i]) / h;
        dvel_out[i] = cimag(v[i]) / h;
    }
    free(p);
    free(v);
    free(pr);
    free(vm);
    free(ta);
}

/*
 * A float64 trajectory from (pos0, vel0) with fixed preferred velocities,
 * step by step: loss_t[t] = sum_i |x_i - y_i|^2 after t + 1 steps and
 * tape_t[t] = the hash of every decision step t took (in agent order).  With
 * a tangent (dpref, dvmax, dtau, any of them non-NULL) the trajectory runs by
 * complex step and dloss_t[t] is the loss's directional derivative after
 * t + 1 steps along that tangent; the decisions are the primal's.  With
 * f32_state the primal state is rounded to float32 after every step, as in
 * oracle_traj_jvp (the trajectory a float32-state step takes).  Used to
 * count central differences only where no decision switches.
 */
void oracle_traj_curve(int64_t n, const double *pos0, const double *vel0, const double *pref,
                       int32_t n_scenes, const int64_t *off, const oracle_params *par,
                       const double *vmax_s, const double *tau_s, int32_t n_steps,
                       const double *targets, const double *dpref, const double *dvmax,
                       const double *dtau, int32_t f32_state, const oracle_agents *ag,
                       double *loss_t, double *dloss_t, uint64_t *tape_t)
{
    uint64_t *ah = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n ? n : 1));
    const int tangent = dpref || dvmax || dtau;
    if (!tangent) {
        double *pos = (double *)malloc(sizeof(double) * 2 * (size_t)(n ? n : 1));
        double *vel = (double *)malloc(sizeof(double) * 2 * (size_t)(n ? n : 1));
        memcpy(pos, pos0, sizeof(double) * 2 * (size_t)n);
        memcpy(vel, vel0, sizeof(double) * 2 * (size_t)n);
        for (int32_t t = 0; t < n_steps; ++t) {
            traj_step_d(n, pos, vel, pref, n_scenes, off, par, vmax_s, tau_s, ag, ah);
            if (f32_state)
                for (int64_t i = 0; i < 2 * n; ++i) {
                    pos[i] = (double)(float)pos[i];
                    vel[i] = (double)(float)vel[i];
                }
            /* summed in long double: central differences divide the loss's
             * rounding by 2h, so it must stay far below L */
            long double L = 0.0L;
            for (int64_t i = 0; i < 2 * n; ++i) {
                const double e = pos[i] - targets[i];
                L += (long double)e * (long double)e;
            }
            uint64_t hs = tape_mix(0, (uint64_t)t);
            for (int64_t i = 0; i < n; ++i) hs = tape_mix(hs, ah[i]);
            if (loss_t) loss_t[t] = (double)L;
            if (dloss_t) dloss_t[t] = 0.0;
            if (tape_t) tape_t[t] = hs;
        }
        free(pos);
        free(vel);
        free(ah);
        return;
    }
    const double h = 1e-30;
    double complex *pos = (double complex *)malloc(sizeof(double complex) * 2 * (size_t)(n ? n : 1));
    double complex *vel = (double complex *)malloc(sizeof(double complex) * 2 * (size_t)(n ? n : 1));
    double complex *pr = (double complex *)malloc(sizeof(double complex) * 2 * (size_t)(n ? n : 1));
    double complex *vm = (double complex *)malloc(sizeof(double complex) * (size_t)n_scenes);
    double complex *ta = (double complex *)malloc(sizeof(double complex) * (size_t)n_scenes);
    for (int64_t i = 0; i < 2 * n; ++i) {
        pos[i] = pos0[i];
        vel[i] = vel0[i];
        pr[i] = pref[i] + I * h * (dpref ? dpref[i] : 0.0);
    }
    for (int s = 0; s < n_scenes; ++s) {
        vm[s] = vmax_s[s] + I * h * (dvmax ? dvmax[s] : 0.0);
        ta[s] = tau_s[s] + I * h * (dtau ? dtau[s] : 0.0);
    }
    for (int32_t t = 0; t < n_steps; ++t) {
        traj_step_c(n, pos, vel, pr, n_scenes, off, par, vm, ta, ag, ah);
        if (f32_state)
            for (int64_t i = 0; i < 2 * n; ++i) {
                pos[i] = (double)(float)creal(pos[i]) + I * cimag(pos[i]);
                vel[i] = (double)(float)creal(vel[i]) + I * cimag(vel[i]);
            }
        /* L and its tangent 2 e . e' summed in long double, as above */
        long double Lr = 0.0L, Li = 0.0L;
        for (int64_t i = 0; i < 2 * n; ++i) {
            const double er = creal(pos[i]) - targets[i], ei = cimag(pos[i]) / h;
            Lr += (long double)er * (long double)er;
            Li += 2.0L * (long double)er * (long double)ei;
        }
        uint64_t hs = tape_mix(0, (uint64_t)t);
        for (int64_t i = 0; i < n; ++i) hs = tape_mix(hs, ah[i]);
        if (loss_t) loss_t[t] = (double)Lr;
        if (dloss_t) dloss_t[t] = (double)Li;
        if (tape_t) tape_t[t] = hs;
    }
    free(pos);
    free(vel);
    free(pr);
    free(vm);
    free(ta);
    free(ah);
}
