// orca_adjoint.h -- vector-Jacobian products of one agent's velocity choice
// (float64), for the adjoint of a recorded step.
//
// The forward step is piecewise smooth: the neighbour set, the branch of each
// half-plane (Fig. 1: cut-off arc, left leg, right leg, contact) and the
// active constraints of the programs (section 3) are discrete choices.  With
// them held fixed, the chosen velocity is an explicit function of the
// half-planes, the preferred velocity and the max speed:
//   projection (relaxation s = 0, or d* + delta in the fallback):
//     no row: vhat, or its radial clip to the disc;
//     one row a:             vhat + (c_a - n_a.vhat) n_a;
//     rows a and b:          the crossing of their lines;
//     row a and the disc:    the crossing of its line with the circle;
//   least penetration (t = d*, the point v3):
//     plane k and the disc:          v3 = vmax n_k,  t = b_k - vmax;
//     planes k, i, j equal:          [n 1] (v3, t) = b for the three rows;
//     planes k, i equal on the circle;
//     planes k, i with antiparallel normals (t does not depend on v3).
// Each function takes the gradient of its result and accumulates gradients
// of the rows' (n, b), of vhat and of vmax.  obstacle_exit_vjp carries row
// gradients back to the relative position, relative velocity and tau.
#pragma once

#include "orca_lp.h"

namespace orca {

// Record of how one agent's velocity was chosen in a recorded step.
struct TapeCode {
    int8_t status;         // 0 projection feasible, 1 fallback
    int8_t p_line, p_src;  // Active of the final projection (relaxed in the fallback)
    int8_t d_plane;        // least penetration: plane of the last accepted step (-1 none)
    int8_t d_line, d_src;  // and the Active of that plane's program
    int8_t relaxed_empty;  // 1: the relaxed projection was empty, v' is the d* point
    int8_t pad;
    double dstar;          // least penetration (fallback only)
};

// Half-plane r of the agent: inputs of obstacle_exit and its results.
struct RowGeom {
    double Px, Py, Vx, Vy;
    int first;
    double ux, uy, nx, ny, b;
};

// inv_tau, inv_dt: 1 / tau and 1 / dt rounded to nearest, as the forward step
// computes them (so the half-plane is the forward's bit for bit).
ORCA_HD inline void row_geom(RowGeom &g, double R, double tau, double dt, double inv_tau,
                             double inv_dt, double vix, double viy)
{
    obstacle_exit(g.Px, g.Py, g.Vx, g.Vy, R, tau, dt, inv_tau, inv_dt, g.first != 0, g.ux,
                  g.uy, g.nx, g.ny);
    const double qx = vix + 0.5 * g.ux, qy = viy + 0.5 * g.uy;
    g.b = g.nx * qx + g.ny * qy;
}

// Gradient of one obstacle_exit call: (gux, guy, gnx, gny) -> P, V, tau.  The
// branch is the one the recorded half-plane took (the case tests below are
// the forward's: w from div_recip with inv_tau / inv_dt = 1 / tau, 1 / dt
// rounded to nearest rounds as the division does); within it, quotients use
// reciprocals, which moves the gradient by rounding only.
ORCA_HD inline void obstacle_exit_vjp(const RowGeom &g, double R, double tau, double dt,
                                      double inv_tau, double inv_dt, double gux, double guy, double gnx, double gny, double &gPx,
                                      double &gPy, double &gVx, double &gVy, double &gtau)
{
    const double Px = g.Px, Py = g.Py, Vx = g.Vx, Vy = g.Vy;
    const double dist2 = Px * Px + Py * Py;
    const double R2 = R * R;
    if (dist2 > R2) {
        const double wx = Vx - div_recip(Px, tau, inv_tau);
        const double wy = Vy - div_recip(Py, tau, inv_tau);
        const double w2 = wx * wx + wy * wy;
        const double wP = wx * Px + wy * Py;
        if (wP < 0.0 && wP * wP > R2 * w2) {
            // u = f n with n = w / |w|, f = R / tau - |w|, w = V - P / tau
            const double wl = sqrt(w2);
            const double iw = 1.0 / wl;
            const double nx = wx * iw, ny = wy * iw;
            const double f = R * inv_tau - wl;
            const double gf = gux * nx + guy * ny;
            const double gtx = gnx + f * gux, gty = gny + f * guy;
            const double nd = nx * gtx + ny * gty;
            const double gwx = (gtx - nx * nd) * iw - gf * nx;
            const double gwy = (gty - ny * nd) * iw - gf * ny;
            gtau += (-gf * R + (gwx * Px + gwy * Py)) * (inv_tau * inv_tau);
            gVx += gwx;
            gVy += gwy;
            gPx += -gwx * inv_tau;
            gPy += -gwy * inv_tau;
            return;
        }
        // leg: l = A / |P|^2 with A = L P +- R J P, J P = (-Py, Px), L = sqrt(|P|^2 - R^2)
        const bool left = Px * wy - Py * wx > 0.0;
        const double L = sqrt(dist2 - R2);
        const double id2 = 1.0 / dist2, iL = 1.0 / L;
        const double sg = left ? 1.0 : -1.0;
        const double Ax = Px * L - sg * Py * R, Ay = sg * Px * R + Py * L;
        const double lx = Ax * id2, ly = Ay * id2;
        double glx, gly;
        if (left) {  // n = (-ly, lx)
            glx = gny;
            gly = -gnx;
        } else {  // n = (ly, -lx)
            glx = -gny;
            gly = gnx;
        }
        // u = s l - V, s = V . l
        const double s = Vx * lx + Vy * ly;
        const double gs = gux * lx + guy * ly;
        glx += s * gux + gs * Vx;
        gly += s * guy + gs * Vy;
        gVx += gs * lx - gux;
        gVy += gs * ly - guy;
        // l = A / d2
        const double gAx = glx * id2, gAy = gly * id2;
        const double gd2 = -(glx * lx + gly * ly) * id2;
        // A = L P + sg R J P:  dA = L dP + sg R J dP + P (P . dP) / L
        const double AP = gAx * Px + gAy * Py;
        gPx += L * gAx + sg * R * gAy + AP * Px * iL + 2.0 * gd2 * Px;
        gPy += L * gAy - sg * R * gAx + AP * Py * iL + 2.0 * gd2 * Py;
        return;
    }
    // contact: the one-step disc D(P/dt, R/dt)
    const double wx = Vx - div_recip(Px, dt, inv_dt);
    const double wy = Vy - div_recip(Py, dt, inv_dt);
    const double wl = sqrt(wx * wx + wy * wy);
    if (wl > 0.0) {
        const double iw = 1.0 / wl;
        const double nx = wx * iw, ny = wy * iw;
        const double f = R * inv_dt - wl;
        const double gf = gux * nx + guy * ny;
        const double gtx = gnx + f * gux, gty = gny + f * guy;
        const double nd = nx * gtx + ny * gty;
        const double gwx = (gtx - nx * nd) * iw - gf * nx;
        const double gwy = (gty - ny * nd) * iw - gf * ny;
        gVx += gwx;
        gVy += gwy;
        gPx += -gwx * inv_dt;
        gPy += -gwy * inv_dt;
    } else if (dist2 > 0.0) {
        // n = -P / |P|, u = (R / dt) n
        const double pl = sqrt(dist2);
        const double ip = 1.0 / pl;
        const double nx = -Px * ip, ny = -Py * ip;
        const double f = R * inv_dt;
        const double gtx = gnx + f * gux, gty = gny + f * guy;
        const double nd = nx * gtx + ny * gty;
        gPx += -(gtx - nx * nd) * ip;
        gPy += -(gty - ny * nd) * ip;
    }
}

// Gradient of row r's (n, b) -> P, V, tau and the agent's own velocity v_i
// (b = n . (v_i + u / 2)).
ORCA_HD inline void row_vjp(const RowGeom &g, double R, double tau, double dt, double inv_tau,
                            double inv_dt, double vix, double viy, double gnx, double gny, double gb,
                            double &gPx, double &gPy, double &gVx, double &gVy, double &gtau,
                            double &gvix, double &gviy)
{
    const double qx = vix + 0.5 * g.ux, qy = viy + 0.5 * g.uy;
    gnx += gb * qx;
    gny += gb * qy;
    const double gqx = gb * g.nx, gqy = gb * g.ny;
    gvix += gqx;
    gviy += gqy;
    obstacle_exit_vjp(g, R, tau, dt, inv_tau, inv_dt, 0.5 * gqx, 0.5 * gqy, gnx, gny, gPx, gPy, gVx, gVy,
                      gtau);
}

// The rows a record refers to, in fixed slots (the caller fetches them):
enum Slot { kSlotLine = 0, kSlotClamp = 1, kSlotPlane = 2, kSlotPlaneLine = 3, kSlotPlaneClamp = 4 };
constexpr int kSlots = 5;

// Gradients of the slots' (n, b).
struct SlotGrads {
    double gnx[kSlots], gny[kSlots], gb[kSlots];
    ORCA_HD inline void clear()
    {
        for (int q = 0; q < kSlots; ++q) gnx[q] = gny[q] = gb[q] = 0.0;
    }
};

// Row index held by each slot of a record (-1: unused).
ORCA_HD inline void slot_rows(const TapeCode &tc, int r[kSlots])
{
    for (int q = 0; q < kSlots; ++q) r[q] = -1;
    if (tc.p_line >= 0) r[kSlotLine] = tc.p_line;
    if (tc.p_line >= 0 && tc.p_src >= 0) r[kSlotClamp] = tc.p_src;
    if (tc.status == 1 && tc.d_plane >= 0) {
        r[kSlotPlane] = tc.d_plane;
        if (tc.d_line >= 0) r[kSlotPlaneLine] = tc.d_line;
        if (tc.d_line >= 0 && tc.d_src >= 0) r[kSlotPlaneClamp] = tc.d_src;
    }
}

// Gradient of a projection's result (relaxation s) given its Active; a is the
// line's row, b the clamping row.
ORCA_HD inline void projection_vjp(const RowGeom &a, const RowGeom &b, int line, int src, double s,
                                   double vmax, double vhx, double vhy, double gx, double gy,
                                   SlotGrads &sg_, double &gvhx, double &gvhy, double &gvmax,
                                   double &gs)
{
    if (line == kLineNone) {
        const double vh2 = vhx * vhx + vhy * vhy;
        if (vh2 > vmax * vmax) {  // v' = vmax vhat / |vhat|
            const double vl = sqrt(vh2);
            const double ux = vhx / vl, uy = vhy / vl;
            const double ug = ux * gx + uy * gy;
            gvhx += vmax / vl * (gx - ux * ug);
            gvhy += vmax / vl * (gy - uy * ug);
            gvmax += ug;
        } else {
            gvhx += gx;
            gvhy += gy;
        }
        return;
    }
    const double ca = a.b - s;
    if (src == kSrcFree) {  // v' = vhat + (c - n.vhat) n
        const double ng = a.nx * gx + a.ny * gy;
        const double coef = ca - (a.nx * vhx + a.ny * vhy);
        gvhx += gx - a.nx * ng;
        gvhy += gy - a.ny * ng;
        sg_.gnx[kSlotLine] += coef * gx - ng * vhx;
        sg_.gny[kSlotLine] += coef * gy - ng * vhy;
        sg_.gb[kSlotLine] += ng;
        gs -= ng;
        return;
    }
    if (src >= 0) {  // crossing of lines a and b: [n_a; n_b] v' = (c_a, c_b)
        const double cb = b.b - s;
        const double det = a.nx * b.ny - a.ny * b.nx;
        if (det == 0.0) return;
        const double vx = (ca * b.ny - cb * a.ny) / det;
        const double vy = (a.nx * cb - b.nx * ca) / det;
        const double za = (gx * b.ny - gy * b.nx) / det;
        const double zb = (a.nx * gy - a.ny * gx) / det;
        sg_.gnx[kSlotLine] += -za * vx;
        sg_.gny[kSlotLine] += -za * vy;
        sg_.gb[kSlotLine] += za;
        sg_.gnx[kSlotClamp] += -zb * vx;
        sg_.gny[kSlotClamp] += -zb * vy;
        sg_.gb[kSlotClamp] += zb;
        gs -= za + zb;
        return;
    }
    // crossing of line a with the circle, on vhat's side of the line's foot
    const double dx = -a.ny, dy = a.nx;
    double h2 = vmax * vmax - ca * ca;
    h2 = h2 > 0.0 ? h2 : 0.0;
    const double sgn = (dx * vhx + dy * vhy) >= 0.0 ? 1.0 : -1.0;
    const double vx = ca * a.nx + sgn * sqrt(h2) * dx, vy = ca * a.ny + sgn * sqrt(h2) * dy;
    // n.dv = dc - v.dn ; v.dv = vmax dvmax
    const double det = a.nx * vy - a.ny * vx;
    if (det == 0.0) return;
    const double z0 = (gx * vy - gy * vx) / det;
    const double z1 = (a.nx * gy - a.ny * gx) / det;
    sg_.gnx[kSlotLine] += -z0 * vx;
    sg_.gny[kSlotLine] += -z0 * vy;
    sg_.gb[kSlotLine] += z0;
    gs -= z0;
    gvmax += z1 * vmax;
}

// Solve M^T z = r for a 3x3 M (Cramer's rule); false if singular.
ORCA_HD inline bool solve3_t(const double M[3][3], const double r[3], double z[3])
{
    // columns of M^T are rows of M
    const double a = M[0][0], b = M[1][0], c = M[2][0];
    const double d = M[0][1], e = M[1][1], f = M[2][1];
    const double g = M[0][2], h = M[1][2], k = M[2][2];
    const double det = a * (e * k - f * h) - b * (d * k - f * g) + c * (d * h - e * g);
    if (det == 0.0) return false;
    z[0] = (r[0] * (e * k - f * h) - b * (r[1] * k - f * r[2]) + c * (r[1] * h - e * r[2])) / det;
    z[1] = (a * (r[1] * k - f * r[2]) - r[0] * (d * k - f * g) + c * (d * r[2] - r[1] * g)) / det;
    z[2] = (a * (e * r[2] - r[1] * h) - b * (d * r[2] - r[1] * g) + r[0] * (d * h - e * g)) / det;
    return true;
}

// Gradient of the least-penetration result (t = d*, point v3) given its
// record; gt and (g3x, g3y) are the gradients of t and v3.  k, i, j: the
// rows in the plane, plane-line and plane-clamp slots.
ORCA_HD inline void least_penetration_vjp(const RowGeom &k, const RowGeom &i, const RowGeom &j,
                                          int plane, int line, int src, double vmax, double gt,
                                          double g3x, double g3y, SlotGrads &sg_, double &gvmax)
{
    if (plane < 0) return;  // no accepted step: t = 0 does not move
    if (line == kLineNone) {  // v3 = vmax n_k / |n_k|, t = b_k - vmax |n_k|
        const double ng = k.nx * g3x + k.ny * g3y;
        sg_.gnx[kSlotPlane] += -vmax * gt * k.nx + vmax * (g3x - k.nx * ng);
        sg_.gny[kSlotPlane] += -vmax * gt * k.ny + vmax * (g3y - k.ny * ng);
        sg_.gb[kSlotPlane] += gt;
        gvmax += -gt + ng;
        return;
    }
    if (line < 0 || src == -1) return;  // "t >= 0" active: t = 0
    const double mx = i.nx - k.nx, my = i.ny - k.ny;  // projected row of the line
    const double ci = i.b - k.b;
    if (src == kSrcFree) {
        // objective parallel to the line (antiparallel normals): n_k.v = c_i / alpha,
        // t = b_k - c_i / alpha with alpha = (n_i - n_k).n_k
        const double alpha = mx * k.nx + my * k.ny;
        if (alpha == 0.0) return;
        const double ga = gt * ci / (alpha * alpha);
        sg_.gnx[kSlotPlane] += ga * (i.nx - 2.0 * k.nx);
        sg_.gny[kSlotPlane] += ga * (i.ny - 2.0 * k.ny);
        sg_.gb[kSlotPlane] += gt * (1.0 + 1.0 / alpha);
        sg_.gnx[kSlotPlaneLine] += ga * k.nx;
        sg_.gny[kSlotPlaneLine] += ga * k.ny;
        sg_.gb[kSlotPlaneLine] += -gt / alpha;
        return;
    }
    double M[3][3], v3x, v3y;
    const double r[3] = {g3x, g3y, gt};
    double z[3];
    if (src >= 0) {  // three equal pieces: [n_a 1] (v, t) = b_a
        M[0][0] = k.nx; M[0][1] = k.ny; M[0][2] = 1.0;
        M[1][0] = i.nx; M[1][1] = i.ny; M[1][2] = 1.0;
        M[2][0] = j.nx; M[2][1] = j.ny; M[2][2] = 1.0;
        const double det = k.nx * (i.ny - j.ny) - k.ny * (i.nx - j.nx) + (i.nx * j.ny - i.ny * j.nx);
        if (det == 0.0) return;
        v3x = (k.b * (i.ny - j.ny) - k.ny * (i.b - j.b) + (i.b * j.ny - i.ny * j.b)) / det;
        v3y = (k.nx * (i.b - j.b) - k.b * (i.nx - j.nx) + (i.nx * j.b - i.b * j.nx)) / det;
        if (!solve3_t(M, r, z)) return;
        sg_.gnx[kSlotPlane] += -z[0] * v3x;
        sg_.gny[kSlotPlane] += -z[0] * v3y;
        sg_.gb[kSlotPlane] += z[0];
        sg_.gnx[kSlotPlaneLine] += -z[1] * v3x;
        sg_.gny[kSlotPlaneLine] += -z[1] * v3y;
        sg_.gb[kSlotPlaneLine] += z[1];
        sg_.gnx[kSlotPlaneClamp] += -z[2] * v3x;
        sg_.gny[kSlotPlaneClamp] += -z[2] * v3y;
        sg_.gb[kSlotPlaneClamp] += z[2];
        return;
    }
    // two equal pieces on the circle: the crossing of line (m, c) with |v| = vmax
    const double mm = mx * mx + my * my;
    double disc = vmax * vmax * mm - ci * ci;
    disc = disc > 0.0 ? disc : 0.0;
    const double slope = k.ny * mx - k.nx * my;
    const double sv = (slope >= 0.0 ? 1.0 : -1.0) * sqrt(disc) / mm;
    v3x = ci / mm * mx - sv * my;
    v3y = ci / mm * my + sv * mx;
    M[0][0] = k.nx; M[0][1] = k.ny; M[0][2] = 1.0;
    M[1][0] = i.nx; M[1][1] = i.ny; M[1][2] = 1.0;
    M[2][0] = v3x;  M[2][1] = v3y;  M[2][2] = 0.0;
    if (!solve3_t(M, r, z)) return;
    sg_.gnx[kSlotPlane] += -z[0] * v3x;
    sg_.gny[kSlotPlane] += -z[0] * v3y;
    sg_.gb[kSlotPlane] += z[0];
    sg_.gnx[kSlotPlaneLine] += -z[1] * v3x;
    sg_.gny[kSlotPlaneLine] += -z[1] * v3y;
    sg_.gb[kSlotPlaneLine] += z[1];
    gvmax += z[2] * vmax;
}

// Whole VJP of one agent's choice: given g = dL/dv', accumulate dL/d(slot
// rows) through the least penetration and the projection, dL/dvhat and
// dL/dvmax.  rows: the five slots (unused slots are ignored).
ORCA_HD inline void choice_vjp(const RowGeom rows[kSlots], const TapeCode &tc, double vmax,
                               double vhx, double vhy, double gx, double gy, SlotGrads &sg_,
                               double &gvhx, double &gvhy, double &gvmax)
{
    if (tc.status == 0) {
        double gs = 0.0;
        projection_vjp(rows[kSlotLine], rows[kSlotClamp], tc.p_line, tc.p_src, 0.0, vmax, vhx, vhy,
                       gx, gy, sg_, gvhx, gvhy, gvmax, gs);
        return;
    }
    if (tc.relaxed_empty) {
        least_penetration_vjp(rows[kSlotPlane], rows[kSlotPlaneLine], rows[kSlotPlaneClamp],
                              tc.d_plane, tc.d_line, tc.d_src, vmax, 0.0, gx, gy, sg_, gvmax);
        return;
    }
    double gs = 0.0;
    projection_vjp(rows[kSlotLine], rows[kSlotClamp], tc.p_line, tc.p_src, tc.dstar + kRelax, vmax,
                   vhx, vhy, gx, gy, sg_, gvhx, gvhy, gvmax, gs);
    least_penetration_vjp(rows[kSlotPlane], rows[kSlotPlaneLine], rows[kSlotPlaneClamp], tc.d_plane,
                          tc.d_line, tc.d_src, vmax, gs, 0.0, 0.0, sg_, gvmax);
}

}  // namespace orca
