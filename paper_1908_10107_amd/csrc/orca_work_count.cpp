// orca_work_count.cpp -- host build of the velocity programs of orca_lp.h with
// their work-counting hooks on, for measuring the algorithmic work per agent
// that the roofline of the LP kernels is priced in.
//
// It runs, for each listed agent, what the velocity kernels run for it, in
// the same order and arithmetic: the float64 half-plane of each neighbour
// (Fig. 1), the incremental 2D program (section 3); for an agent whose program
// is empty, the most violated row after the failed one, the stash order of
// its rows and the fallback (least penetration, then the relaxed projection;
// section 3, infeasible case).  Each hooked event is counted per phase: the
// half-planes and 2D program (the LP kernel) and the fallback.
//
// Built with g++ by the tests (no GPU involved); not part of liborca.
#include <stdint.h>
#include <string.h>

namespace orca_count {
enum Event {
    hp_arc, hp_leg, hp_overlap, lp2_check, lp2_line, lp2_inner, fail_row_check,
    plane_check, plane_line, plane_inner, lp3_check, lp3_plane, kEvents
};
thread_local double *sink = nullptr;  // counters of the current phase
}  // namespace orca_count

#define ORCA_COUNT(what) (orca_count::sink[orca_count::what] += 1.0)
#define ORCA_COUNT_N(what, n) (orca_count::sink[orca_count::what] += (double)(n))

#include "orca_lp.h"

namespace {

constexpr int kRows = 16;  // the kernels' register row bound at K <= 16

// Rows of one agent, read with any index (the host has no register files).
struct HostRows {
    double2 n[kRows];
    double b[kRows];
    double2 N(int k) const { return n[k]; }
    double B(int k) const { return b[k]; }
    double2 NL(int k) const { return n[k]; }
    double BL(int k) const { return b[k]; }
};

}  // namespace

extern "C" {

// Event names in counter order (for the caller's table).
const char *orca_work_events(void)
{
    return "hp_arc hp_leg hp_overlap lp2_check lp2_line lp2_inner fail_row_check plane_check "
           "plane_line plane_inner lp3_check lp3_plane";
}

int orca_work_event_count(void) { return orca_count::kEvents; }

// For each of the n_agents listed agents of one scene: pos, vel [2, n]
// float32 (SoA), vhat [n_agents, 2] the preferred velocity in float64 (as the
// kernels compute it), nbr [n_agents, kcap] neighbour ids nearest first
// (ties by id), ncount [n_agents].  Scene parameters: radius, vmax, tau, dt
// (float32, as the kernels read them).  Outputs: counts_lp, counts_fb
// [kEvents] summed over the agents; new_vel [n_agents, 2]; status
// [n_agents] (0 2D program, 1 fallback).  Returns 0, or -1 if a neighbour
// count exceeds the row bound.
int orca_work_count(int64_t n, const float *pos, const float *vel, const int64_t *agents,
                    int64_t n_agents, const double *vhat, const int64_t *nbr,
                    const int32_t *ncount, int32_t kcap, float radius, float vmax_f, float tau_f,
                    float dt_f, double *counts_lp, double *counts_fb, double *new_vel,
                    uint8_t *status)
{
    using namespace orca;
    memset(counts_lp, 0, sizeof(double) * orca_count::kEvents);
    memset(counts_fb, 0, sizeof(double) * orca_count::kEvents);
    const double tau = (double)tau_f, dt = (double)dt_f;
    const double inv_tau = 1.0 / tau, inv_dt = 1.0 / dt;
    const double R = (double)radius + (double)radius;
    const double vmax = (double)vmax_f;
    for (int64_t a = 0; a < n_agents; ++a) {
        const int64_t i = agents[a];
        const int m = ncount[a];
        if (m > kRows) return -1;
        const double xi = pos[i], yi = pos[n + i];
        const double vix = vel[i], viy = vel[n + i];
        const double vhx = vhat[2 * a], vhy = vhat[2 * a + 1];
        double2 rn[kRows];
        double rb[kRows];
        orca_count::sink = counts_lp;
        for (int k = 0; k < kRows; ++k) {
            rn[k] = make_double2(0.0, 0.0);
            rb[k] = 0.0;
            if (k >= m) continue;
            const int64_t j = nbr[a * kcap + k];
            const double Px = (double)pos[j] - xi, Py = (double)pos[n + j] - yi;
            const double Vx = vix - (double)vel[j], Vy = viy - (double)vel[n + j];
            double ux, uy, nx, ny;
            obstacle_exit(Px, Py, Vx, Vy, R, tau, dt, inv_tau, inv_dt, i < j, ux, uy, nx, ny);
            const double qx = vix + 0.5 * ux, qy = viy + 0.5 * uy;
            rn[k] = make_double2(nx, ny);
            rb[k] = nx * qx + ny * qy;
        }
        double vx, vy;
        disc_clip(vmax, vhx, vhy, vx, vy);
        Active act;
        const int fail = lp2_project_regs<kRows>(rn, rb, m, vmax, vhx, vhy, vx, vy, &act);
        if (fail < 0) {
            new_vel[2 * a] = vx;
            new_vel[2 * a + 1] = vy;
            status[a] = 0;
            continue;
        }
        HostRows in;
        for (int k = 0; k < kRows; ++k) {
            in.n[k] = rn[k];
            in.b[k] = rb[k];
        }
        FallbackItem it{};
        it.m = (int8_t)m;
        it.fail = (int8_t)fail;
        it.line = (int8_t)act.line;
        it.src = (int8_t)act.src;
        it.worst = (int8_t)worst_row<kRows>(in, fail, m, vx, vy);
        // the fallback takes the rows in stash order
        HostRows st;
        for (int k = 0; k < kRows; ++k) {
            st.n[k] = make_double2(0.0, 0.0);
            st.b[k] = 0.0;
        }
        for (int k = 0; k < m; ++k) {
            const int q = stash_position(k, it);
            st.n[q] = rn[k];
            st.b[q] = rb[k];
        }
        orca_count::sink = counts_fb;
        int plane = -1;
        Active dact, ract;
        bool ok;
        fallback_velocity<kRows>(st, m, fail, vmax, vhx, vhy, vx, vy, &plane, &dact, &ract, &ok);
        new_vel[2 * a] = vx;
        new_vel[2 * a + 1] = vy;
        status[a] = 1;
    }
    orca_count::sink = nullptr;
    return 0;
}

}  // extern "C"
