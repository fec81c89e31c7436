// orca_lp.h -- per-agent geometry and linear programs of the ORCA step
// (float64), used by the velocity kernels.
//
//   obstacle_exit          Fig. 1(b)-(c): shortest exit u from the velocity
//                          obstacle and the outward normal
//   lp2_project            section 3: permitted velocity closest to the
//                          preferred one (incremental 2D program)
//   lp3_least_penetration  section 3, infeasible case: least penetration d*
//                          (incremental 3D program on the plane of each
//                          violated constraint)
#pragma once

#include <math.h>
#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define ORCA_HD __host__ __device__
#else
#define ORCA_HD
struct double2 {
    double x, y;
};
inline double2 make_double2(double x, double y) { return double2{x, y}; }
#endif

// Always inlined: a row store held in registers must not escape into a call.
#define ORCA_HDI ORCA_HD __attribute__((always_inline))

// Work-counting hooks for the host build that counts the programs' work per
// agent (ORCA_COUNT: one event; ORCA_COUNT_N: n events); they compile to
// nothing in the library.
#ifndef ORCA_COUNT
#define ORCA_COUNT(what)
#endif
#ifndef ORCA_COUNT_N
#define ORCA_COUNT_N(what, n)
#endif

namespace orca {

#ifndef ORCA_LP_STRIDE
constexpr int kLpStride = 64;  // lanes per LP block: element k of a lane at [k * kLpStride]
#else
constexpr int kLpStride = ORCA_LP_STRIDE;
#endif

// a / b rounded to nearest, from y = 1 / b rounded to nearest: one residual
// step on a * y (Markstein's correction), exact for operands that neither
// overflow nor underflow on the way.  A zero a keeps its sign.  Cheaper than a
// full division when y serves several quotients.
ORCA_HDI inline double div_recip(double a, double b, double y)
{
    const double q = a * y;
    const double r = fma(fma(-q, b, a), y, q);
    return q == 0.0 ? q : r;
}

// Shortest change u of the relative velocity V = v_i - v_j out of the velocity
// obstacle of neighbour j (relative position P = x_j - x_i, combined radius R,
// look-ahead tau) and the outward normal n at V + u (Fig. 1(b)-(c)).  A pair
// already closer than R uses the one-step disc D(P/dt, R/dt).  inv_tau and
// inv_dt are 1/tau and 1/dt rounded to nearest.  No other fused multiply-add:
// the operations are rounded one by one, each quotient as a division would
// round it.
ORCA_HD inline void obstacle_exit(double Px, double Py, double Vx, double Vy, double R,
                                              double tau, double dt, double inv_tau,
                                              double inv_dt, bool i_first, double &ux,
                                              double &uy, double &nx, double &ny)
{
#pragma clang fp contract(off)
    // The cases share their arithmetic in two groups, so a wave whose lanes
    // fall in different cases runs two paths, not four; each case still does
    // exactly its own operations in its own order:
    //   circle: the cut-off arc (apart, look-ahead tau) or, for a pair
    //           already in contact, the one-step disc (dt in place of tau);
    //   legs:   the left or right tangent leg, mirror images by a sign.
    const double dist2 = Px * Px + Py * Py;
    const double R2 = R * R;
    const bool apart = dist2 > R2;
    const double tc = apart ? tau : dt, ic = apart ? inv_tau : inv_dt;
    const double wx = Vx - div_recip(Px, tc, ic), wy = Vy - div_recip(Py, tc, ic);
    const double w2 = wx * wx + wy * wy;
    const double wP = wx * Px + wy * Py;
    const bool circle = !apart || (wP < 0.0 && wP * wP > R2 * w2);
    if (!apart) {
        ORCA_COUNT(hp_overlap);
    } else if (circle) {
        ORCA_COUNT(hp_arc);
    } else {
        ORCA_COUNT(hp_leg);
    }
    // Each case takes one square root and two quotients by one divisor: |w|
    // and w / |w| on the circle; the leg length L and the leg direction
    // (L P -+ R P_perp) / |P|^2 on a leg (left, sg = +1, if w is left of P).
    // Selecting their arguments first lets a wave with lanes in both cases
    // run them once.
    const double root = sqrt(circle ? w2 : dist2 - R2);
    const double den = circle ? root : dist2;
    const double rec = 1.0 / den;
    const double sg = Px * wy - Py * wx > 0.0 ? 1.0 : -1.0;
    const double q1 = div_recip(circle ? wx : Px * root - sg * (Py * R), den, rec);
    const double q2 = div_recip(circle ? wy : sg * (Px * R) + Py * root, den, rec);
    if (circle) {
        const double wl = root;
        if (wl > 0.0) {
            nx = q1;
            ny = q2;
        } else if (dist2 > 0.0) {
            // in contact and not moving apart: away from the neighbour
            const double pl = sqrt(dist2);
            nx = -Px / pl;
            ny = -Py / pl;
        } else {
            nx = i_first ? 1.0 : -1.0;
            ny = 0.0;
        }
        const double f = div_recip(R, tc, ic) - wl;
        ux = f * nx;
        uy = f * ny;
        return;
    }
    // nearest boundary point on the tangent leg, direction (lx, ly)
    const double lx = q1, ly = q2;
    nx = -sg * ly;
    ny = sg * lx;
    const double sdot = Vx * lx + Vy * ly;
    ux = sdot * lx - Vx;
    uy = sdot * ly - Vy;
}

// Constraint store of one lane in the block's LDS: half-plane k is
// {v : n_k . v >= b_k}; n_k is one 16-byte double2 at [k * kLpStride + lane],
// b_k a double at the same index of a second array.
struct Lane {
    double2 *n;
    double *b;
    ORCA_HD inline double2 N(int k) const { return n[k * kLpStride]; }
    ORCA_HD inline double B(int k) const { return b[k * kLpStride]; }
    ORCA_HD inline double2 NL(int k) const { return n[k * kLpStride]; }
    ORCA_HD inline double BL(int k) const { return b[k * kLpStride]; }
};

// What fixes the final point of an incremental 2D program (kept when a step
// is recorded for the adjoint): the row whose 1D program ran last (line; -1:
// none ran, the start point stands) and what bounds the point on that line
// (src: a row index, kSrcDisc, or kSrcFree when the line's own optimum lies
// inside its interval).  Row -1 of a plane program is "t >= 0".
constexpr int kSrcDisc = -2;
constexpr int kSrcFree = -3;
constexpr int kLineNone = -4;    // Active.line when no 1D program ran
constexpr double kRelax = 1e-5;  // relaxation of the least-penetration second stage (m/s)
struct Active {
    int line, src;
};

// An agent whose projection was empty, with what the fallback needs to
// finish it without touching the agent arrays again: sorted index, id, number
// of half-planes, the row at which the projection failed, the line and bound
// that fix the optimum of the rows before it (an Active, as int8), the most
// violated row from the failed one on, that optimum, the preferred velocity,
// max speed, dt and position.  Rows are numbered as in the neighbour list;
// the stash holds them in the order of stash_position().
struct FallbackItem {
    int32_t s, id;
    int8_t m, fail, line, src;
    int8_t worst, pad8[3];
    double vx, vy, vhx, vhy;
    float vmax, dt, mex, mey;
};
static_assert(sizeof(FallbackItem) == 64, "one fallback record per 64-byte line");

// Order in which the fallback takes an agent's rows (the stash order): the
// rows that fix the projection's last optimum (line, then src) first, the
// other rows before the failed one next, then the most violated row from the
// failed one on, then the rest.  The programs' results do not depend on the
// order, only their cost does: started this way, the least-penetration
// program meets few violations after its first plane.
ORCA_HDI inline int stash_position(int k, const FallbackItem &it)
{
    // selects only: the kernels evaluate it for every row of a wave at once
    const int fail = it.fail, line = it.line, src = it.src, worst = it.worst;
    const int nf = (line >= 0 ? 1 : 0) + (src >= 0 ? 1 : 0);
    int before = nf + k - ((src >= 0 && src < k) ? 1 : 0) - ((line >= 0 && line < k) ? 1 : 0);
    before = k == src ? (line >= 0 ? 1 : 0) : before;
    before = k == line ? 0 : before;
    const int after = k == worst ? fail : k + (k < worst ? 1 : 0);
    return k < fail ? before : after;
}

// Inverse of stash_position (negative codes pass through: they name no row).
ORCA_HDI inline int stash_row(int p, const FallbackItem &it)
{
    const int fail = it.fail, line = it.line, src = it.src, worst = it.worst;
    if (p < 0) return p;
    if (p < fail) {
        const int nf = (line >= 0 ? 1 : 0) + (src >= 0 ? 1 : 0);
        if (p < nf) return p == 0 ? (line >= 0 ? line : src) : src;
        int k = p - nf;
        if (src >= 0 && src <= k) ++k;  // src < line when both are rows
        if (line >= 0 && line <= k) ++k;
        return k;
    }
    if (p == fail) return worst;
    const int k = p - 1;
    return k >= worst ? k + 1 : k;
}

// Feasible interval lo <= s <= hi of a 1D program, each end kept as a
// fraction and compared by cross-multiplication, so adding a constraint costs
// no division.  lo has a non-negative denominator, hi a negative one (as the
// rows that set it come), so neither end is ever negated.  lo_src / hi_src
// name the row that set each end (kSrcDisc for the disc).
struct Interval {
    double lo_n, lo_d, hi_n, hi_d;
    int lo_src, hi_src;
    // -h_n / h_d <= s <= h_n / h_d, h_d > 0
    ORCA_HDI inline void init(double h_n, double h_d)
    {
        lo_n = -h_n;
        lo_d = h_d;
        hi_n = -h_n;
        hi_d = -h_d;
        lo_src = kSrcDisc;
        hi_src = kSrcDisc;
    }
    // add s * den >= num (row src).  A row parallel to the line (den == 0)
    // that excludes it (num > 0) raises the lower end to num / 0 = +infinity
    // (lo_d = 0), which every later row keeps and empty() reports; one that
    // admits it (num <= 0) changes nothing.
    ORCA_HDI inline void add(double den, double num, int src)
    {
        const bool up = den >= 0.0;
        const bool raise = up && num * lo_d > lo_n * den;
        const bool lower = !up && num * hi_d < hi_n * den;  // num/den < hi; den, hi_d < 0
        lo_n = raise ? num : lo_n;
        lo_d = raise ? den : lo_d;
        lo_src = raise ? src : lo_src;
        hi_n = lower ? num : hi_n;
        hi_d = lower ? den : hi_d;
        hi_src = lower ? src : hi_src;
    }
    // lo > hi (lo_d >= 0 > hi_d; lo = +infinity also counts)
    ORCA_HDI inline bool empty() const { return lo_n * hi_d < hi_n * lo_d; }
    // t_n / t_d clamped into the interval (t_d > 0); returns the source that
    // bounds the result (kSrcFree if t was inside); o_n / o_d is the value
    ORCA_HDI inline int clamp(double t_n, double t_d, double &o_n, double &o_d) const
    {
        if (t_n * lo_d < lo_n * t_d) {
            o_n = lo_n;
            o_d = lo_d;
            return lo_src;
        }
        if (t_n * hi_d < hi_n * t_d) {
            o_n = hi_n;
            o_d = hi_d;
            return hi_src;
        }
        o_n = t_n;
        o_d = t_d;
        return kSrcFree;
    }
};

// Incremental 2D LP: the point of the disc |v| <= vmax and of the half-planes
// n_k.v >= b_k - relax closest to vhat, constraints taken from index `from`
// on with (vx, vy) optimal for the ones before.  When the current point
// violates constraint k the new optimum lies on its line, found by a 1D
// program against the disc and constraints 0..k-1.  Returns -1 (feasible, v
// set) or the first k whose 1D program is empty (v = the optimum over
// constraints 0..k-1).  With REC the last line and its bound go to *act.
template <bool REC>
ORCA_HD inline int lp2_project(const Lane &L, int m, int from, double relax, double vmax,
                               double vhx, double vhy, double &vx, double &vy, Active *act)
{
    const double vm2 = vmax * vmax;
    if (REC) {
        act->line = kLineNone;
        act->src = kSrcFree;
    }
    for (int k = from; k < m; ++k) {
        const double2 nk = L.N(k);
        const double bk = L.B(k) - relax;
        ORCA_COUNT(lp2_check);
        if (nk.x * vx + nk.y * vy >= bk) continue;
        ORCA_COUNT(lp2_line);
        double h2 = vm2 - bk * bk;
        if (h2 < 0.0) {
            if (bk > 0.0) return k;  // the line misses the disc on the far side
            h2 = 0.0;
        }
        // line k: p(t) = bk n_k + t d_k with d_k = (-n_k.y, n_k.x)
        Interval iv;
        iv.init(sqrt(h2), 1.0);
        for (int j = 0; j < k; ++j) {
            const double2 nj = L.N(j);
            const double bj = L.B(j) - relax;
            ORCA_COUNT(lp2_inner);
            iv.add(nj.y * nk.x - nj.x * nk.y, bj - bk * (nj.x * nk.x + nj.y * nk.y), j);
        }
        if (iv.empty()) return k;
        double tn, td;
        const int src = iv.clamp(nk.x * vhy - nk.y * vhx, 1.0, tn, td);  // d_k . vhat, clamped
        const double t = tn / td;
        vx = bk * nk.x - t * nk.y;
        vy = bk * nk.y + t * nk.x;
        if (REC) {
            act->line = k;
            act->src = src;
        }
    }
    return -1;
}

// lp2_project from row 0 with no relaxation, for rows held in registers:
// every loop runs to the compile-time bound KMAX (rows at or beyond m are
// skipped), so all row indices are static and nothing goes to LDS.  Same
// steps and arithmetic as lp2_project; the Active is always recorded.
template <int KMAX>
ORCA_HD inline int lp2_project_regs(const double2 (&n)[KMAX], const double (&b)[KMAX], int m,
                                    double vmax, double vhx, double vhy, double &vx, double &vy,
                                    Active *act)
{
    const double vm2 = vmax * vmax;
    act->line = kLineNone;
    act->src = kSrcFree;
    int fail = -1;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        if (k >= m || fail >= 0) continue;
        const double2 nk = n[k];
        const double bk = b[k];
        ORCA_COUNT(lp2_check);
        if (nk.x * vx + nk.y * vy >= bk) continue;
        ORCA_COUNT(lp2_line);
        double h2 = vm2 - bk * bk;
        if (h2 < 0.0) {
            if (bk > 0.0) {
                fail = k;  // the line misses the disc on the far side
                continue;
            }
            h2 = 0.0;
        }
        Interval iv;
        iv.init(sqrt(h2), 1.0);
#pragma unroll
        for (int j = 0; j < k; ++j) {
            const double2 nj = n[j];
            ORCA_COUNT(lp2_inner);
            iv.add(nj.y * nk.x - nj.x * nk.y, b[j] - bk * (nj.x * nk.x + nj.y * nk.y), j);
        }
        if (iv.empty()) {
            fail = k;
            continue;
        }
        double tn, td;
        const int src = iv.clamp(nk.x * vhy - nk.y * vhx, 1.0, tn, td);
        const double t = tn / td;
        vx = bk * nk.x - t * nk.y;
        vy = bk * nk.y + t * nk.x;
        act->line = k;
        act->src = src;
    }
    return fail;
}

// Start of lp2_project: vhat, pulled radially into the disc.
ORCA_HDI inline void disc_clip(double vmax, double vhx, double vhy, double &vx, double &vy)
{
    const double vh2 = vhx * vhx + vhy * vhy;
    if (vh2 > vmax * vmax) {
        const double sc = vmax / sqrt(vh2);
        vx = vhx * sc;
        vy = vhy * sc;
    } else {
        vx = vhx;
        vy = vhy;
    }
}

// The fallback's programs below take a row store RS and a compile-time bound
// KB <= 32 on the number of rows.  N(k), B(k) read row k with an index that is
// the same on every lane of a wave (every such loop runs over fixed bounds, a
// lane outside its own range just skips the body, so a store that keeps the
// rows in registers is indexed statically); NL(k), BL(k) read it with a
// lane's own index.  Each lane walks its own violated rows in order: a pass
// finds every lane's next one, then the 1D (or plane) programs of that pass
// run together whatever rows they are on, so a wave pays for its longest
// sequence of violated rows, not for every row that any of its lanes violates.
// A lane's steps and arithmetic are those of the one-row-at-a-time program.

// Rows 0..m-1 as bits.
ORCA_HDI inline uint32_t rows_below(int m) { return m >= 32 ? ~0u : (1u << m) - 1u; }

// Projected constraint i of the plane-k subproblem: i = -1 is "no negative
// penetration" (-n_k . v >= -b_k), i >= 0 is "constraint i penetrates no more
// than k" ((n_i - n_k) . v >= b_i - b_k).
template <class RS>
ORCA_HDI inline void plane_row(const RS &L, int i, double2 nk, double bk, double &mx, double &my,
                              double &c)
{
    if (i < 0) {
        mx = -nk.x;
        my = -nk.y;
        c = -bk;
    } else {
        const double2 ni = L.N(i);
        mx = ni.x - nk.x;
        my = ni.y - nk.y;
        c = L.B(i) - bk;
    }
}

// The term row (ax, ay, cj) adds to the 1D program on projected line
// (mx, my, ci) with |m|^2 = mm: s (a.d) mm >= c_j mm - c_i (a.m), with
// d = (-my, mx).  Shared by the plane program and its work-unit form, so both
// round alike.
ORCA_HDI inline void plane_term(double ax, double ay, double cj, double mx, double my, double ci,
                                double mm, double &den, double &num)
{
    den = (ay * mx - ax * my) * mm;
    num = cj * mm - ci * (ax * mx + ay * my);
}

// Optimum of n_k . v on the projected line (mx, my, ci) within the
// interval iv of its 1D program; act->src gets what bounds it.
ORCA_HDI inline void plane_point(const Interval &iv, double2 nk, double mx, double my, double ci,
                                 double mm, double &vx, double &vy, Active *act)
{
    const double slope = nk.y * mx - nk.x * my;  // n_k . (-my, mx)
    double sn, sd;
    int src;
    if (slope > 0.0) {
        sn = iv.hi_n;
        sd = iv.hi_d;
        src = iv.hi_src;
    } else if (slope < 0.0) {
        sn = iv.lo_n;
        sd = iv.lo_d;
        src = iv.lo_src;
    } else {
        src = iv.clamp(0.0, 1.0, sn, sd);
    }
    const double s = sn / sd;
    const double c0 = ci / mm;
    vx = c0 * mx - s * my;
    vy = c0 * my + s * mx;
    act->src = src;
}

// Maximise n_k . v over the disc and the projected constraints -1..k-1
// (incremental, as lp2_project but with a linear objective).  Line i is
// p(s) = c_i m_i / |m_i|^2 + s (-m_i.y, m_i.x); each constraint j on it is
// multiplied through by |m_i|^2 > 0 so no division is needed until the end.
// Returns false if the subproblem is empty.  The last line and its bound go
// to *act (line kLineNone: the start point vmax n_k stands).  k and the row
// (nk, bk) are the lane's own.
template <int KB, class RS>
ORCA_HDI inline bool lp2_plane(const RS &L, int k, double2 nk, double bk, double vmax, double &vx,
                              double &vy, Active *act)
{
    const double vm2 = vmax * vmax;
    vx = vmax * nk.x;
    vy = vmax * nk.y;
    act->line = kLineNone;
    act->src = kSrcDisc;
    bool ok = true;
    for (int i = -1; i < KB - 1; ++i) {
        if (!ok || i >= k) continue;
        double mx, my, ci;
        plane_row(L, i, nk, bk, mx, my, ci);
        ORCA_COUNT(plane_check);
        if (mx * vx + my * vy >= ci) continue;
        ORCA_COUNT(plane_line);
        const double mm = mx * mx + my * my;
        if (mm == 0.0) {
            ok = !(ci > 0.0);
            continue;
        }
        const double disc = vm2 * mm - ci * ci;
        if (disc < 0.0) {
            ok = false;
            continue;
        }
        // s in [-sqrt(disc), sqrt(disc)] / mm
        Interval iv;
        iv.init(sqrt(disc), mm);
        for (int j = -1; j < i; ++j) {
            double ax, ay, cj;
            plane_row(L, j, nk, bk, ax, ay, cj);
            ORCA_COUNT(plane_inner);
            // a.(c_i m / mm + s d) >= c_j  ->  s (a.d) mm >= c_j mm - c_i (a.m)
            double den, num;
            plane_term(ax, ay, cj, mx, my, ci, mm, den, num);
            iv.add(den, num, j);
        }
        if (iv.empty()) {
            ok = false;
            continue;
        }
        plane_point(iv, nk, mx, my, ci, mm, vx, vy, act);
        act->line = i;
    }
    return ok;
}

// Least penetration d* = min over the disc of max_k (b_k - n_k . v), by an
// incremental 3D program in (v, t) with t >= 0, starting from a point that
// satisfies rows 0..start-1 (so t = 0 is optimal for them).  When row k is
// violated beyond the current t, the new optimum has t = b_k - n_k . v:
// maximise n_k . v on that plane.  The plane of the last accepted step (-1:
// none) and its program's Active are recorded.
template <int KB, class RS>
ORCA_HDI inline double lp3_least_penetration(const RS &L, int m, int start, double vmax, double &vx,
                                            double &vy, int *plane, Active *act)
{
    static_assert(KB <= 32, "row sets are 32-bit masks");
    double t = 0.0;
    *plane = -1;
    act->line = kLineNone;
    act->src = kSrcDisc;
    uint32_t left = rows_below(m) & ~rows_below(start);  // rows not yet tested
#pragma unroll 1
    for (int pass = 0; pass < KB; ++pass) {
        // the lane's first untested row that (v, t) violates
        int k = KB;
        for (int u = KB - 1; u >= 0; --u) {
            const double2 nu = L.N(u);
            const bool hit = ((left >> u) & 1u) != 0u && !(nu.x * vx + nu.y * vy + t >= L.B(u));
            k = hit ? u : k;
        }
        // a lane on its own tests its untested rows up to the violated one
        ORCA_COUNT_N(lp3_check, __builtin_popcount(left & (k < KB ? rows_below(k + 1) : ~0u)));
        if (k >= KB) break;
        left &= ~rows_below(k + 1);
        ORCA_COUNT(lp3_plane);
        const double2 nk = L.NL(k);
        const double bk = L.BL(k);
        double wx, wy;
        Active pa;
        if (lp2_plane<KB>(L, k, nk, bk, vmax, wx, wy, &pa)) {
            vx = wx;
            vy = wy;
            t = fmax(bk - (nk.x * vx + nk.y * vy), 0.0);
            *plane = k;
            *act = pa;
        }
    }
    return t;
}

// Up to three rows taken ahead of the others: copies of rows of the store,
// with their positions in it (pos < 0: the slot is empty).
struct FrontRows {
    double2 n[3];
    double b[3];
    int pos[3];
};

// lp2_project with the front rows taken first and then the other rows of the
// store in order: the point of the disc and of the half-planes
// n_k.v >= b_k - relax closest to vhat, from the radial clip of vhat.  Returns -1 (v set) or the position of
// the first row whose 1D program is empty.  The Active names rows by their
// position in the store.
template <int KB, class RS>
ORCA_HDI inline int lp2_project_front(const RS &L, int m, const FrontRows &F, double relax,
                                     double vmax, double vhx, double vhy, double &vx, double &vy,
                                     Active *act)
{
    const double vm2 = vmax * vmax;
    act->line = kLineNone;
    act->src = kSrcFree;
    int fail = -1;
    disc_clip(vmax, vhx, vhy, vx, vy);
    // one step of the incremental projection on the violated row (nk, bk),
    // given the rows before it: the filled front slots below nf and store rows
    // 0..nrows-1 (nrows may differ between lanes)
    auto line_step = [&](double2 nk, double bk, int pos, int nf,
                         int nrows) __attribute__((always_inline)) {
        ORCA_COUNT(lp2_line);
        double h2 = vm2 - bk * bk;
        if (h2 < 0.0) {
            if (bk > 0.0) {
                fail = pos;  // the line misses the disc on the far side
                return;
            }
            h2 = 0.0;
        }
        Interval iv;
        iv.init(sqrt(h2), 1.0);
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            if (u < nf && F.pos[u] >= 0) {
                const double2 nj = F.n[u];
                ORCA_COUNT(lp2_inner);
                iv.add(nj.y * nk.x - nj.x * nk.y,
                       (F.b[u] - relax) - bk * (nj.x * nk.x + nj.y * nk.y), F.pos[u]);
            }
        }
        for (int j = 0; j < KB - 1; ++j) {
            if (j >= nrows) continue;
            const double2 nj = L.N(j);
            ORCA_COUNT(lp2_inner);
            iv.add(nj.y * nk.x - nj.x * nk.y, (L.B(j) - relax) - bk * (nj.x * nk.x + nj.y * nk.y),
                   j);
        }
        if (iv.empty()) {
            fail = pos;
            return;
        }
        double tn, td;
        const int src = iv.clamp(nk.x * vhy - nk.y * vhx, 1.0, tn, td);  // d_k . vhat, clamped
        const double t = tn / td;
        vx = bk * nk.x - t * nk.y;
        vy = bk * nk.y + t * nk.x;
        act->line = pos;
        act->src = src;
    };
    static_assert(KB <= 32, "row sets are 32-bit masks");
#pragma unroll
    for (int u = 0; u < 3; ++u) {
        if (F.pos[u] < 0 || fail >= 0) continue;
        const double bu = F.b[u] - relax;
        ORCA_COUNT(lp2_check);
        if (!(F.n[u].x * vx + F.n[u].y * vy >= bu)) line_step(F.n[u], bu, F.pos[u], u, 0);
    }
    // a front row is not taken again: on its own line it would meet itself as
    // a constraint, with a cross term that rounding leaves nonzero
    uint32_t left = rows_below(m);
#pragma unroll
    for (int u = 0; u < 3; ++u)
        if (F.pos[u] >= 0) left &= ~(1u << F.pos[u]);
#pragma unroll 1
    for (int pass = 0; pass < KB && fail < 0; ++pass) {
        // the lane's first untested row that v violates
        int k = KB;
        for (int u = KB - 1; u >= 0; --u) {
            const double2 nu = L.N(u);
            const bool hit = ((left >> u) & 1u) != 0u && !(nu.x * vx + nu.y * vy >= L.B(u) - relax);
            k = hit ? u : k;
        }
        ORCA_COUNT_N(lp2_check, __builtin_popcount(left & (k < KB ? rows_below(k + 1) : ~0u)));
        if (k >= KB) break;
        left &= ~rows_below(k + 1);
        line_step(L.NL(k), L.BL(k) - relax, k, 3, k);
    }
    return fail;
}

// The row most violated at (vx, vy) among rows fail..m-1 of a store (the
// fallback's first plane is taken there); fail if none is.
template <int KB, class RS>
ORCA_HDI inline int worst_row(const RS &rows, int fail, int m, double vx, double vy)
{
    int worst = fail;
    double wv = -1.0e300;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        if (k >= fail && k < m) {
            ORCA_COUNT(fail_row_check);
            const double2 nk = rows.N(k);
            const double viol = rows.B(k) - (nk.x * vx + nk.y * vy);
            if (viol > wv) {
                wv = viol;
                worst = k;
            }
        }
    }
    return worst;
}

// The fallback's choice for one agent (section 3, infeasible case), its rows
// in stash order in store RS and (vx, vy) the projection's last optimum,
// where rows 0..fail-1 hold: d* by the least-penetration program, then the
// point closest to vhat within d* + kRelax of every half-plane, with the rows
// that fix d* taken first (the relaxed optimum lies where they cross, so the
// other rows are rarely violated).  Sets (vx, vy) to the result and returns
// d*; *relaxed_ok is false when the relaxed projection was empty (the
// least-penetration point stands).  plane, dact, ract: what fixed the two
// programs' optima, rows named by stash position.
// The least-penetration program fallback_velocity runs by default.
struct Lp3Plain {
    template <int KB, class RS>
    ORCA_HDI double run(const RS &L, int m, int start, double vmax, double &vx, double &vy,
                        int *plane, Active *act) const
    {
        return lp3_least_penetration<KB>(L, m, start, vmax, vx, vy, plane, act);
    }
};

template <int KB, class RS, class LP3 = Lp3Plain>
ORCA_HDI inline double fallback_velocity(const RS &rows, int m, int fail, double vmax, double vhx,
                                         double vhy, double &vx, double &vy, int *plane,
                                         Active *dact, Active *ract, bool *relaxed_ok,
                                         const LP3 &lp3 = LP3())
{
    const double d = lp3.template run<KB>(rows, m, fail, vmax, vx, vy, plane, dact);
    FrontRows F;
    F.pos[0] = *plane;
    F.pos[1] = dact->line;
    F.pos[2] = dact->src;
#pragma unroll
    for (int u = 0; u < 3; ++u) {
        F.n[u] = make_double2(0.0, 0.0);
        F.b[u] = 0.0;
        if (F.pos[u] < 0) F.pos[u] = -1;
    }
    // copy the rows that fix d*: one pass with the same row index on every
    // lane (a per-lane index would move register-held rows to memory)
#pragma unroll 1
    for (int k = 0; k < KB; ++k) {
        const double2 nk = rows.N(k);
        const double bk = rows.B(k);
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            if (F.pos[u] == k) {
                F.n[u] = nk;
                F.b[u] = bk;
            }
        }
    }
    double wx, wy;
    *relaxed_ok = lp2_project_front<KB>(rows, m, F, d + kRelax, vmax, vhx, vhy, wx, wy, ract) < 0;
    if (*relaxed_ok) {
        vx = wx;
        vy = wy;
    }
    return d;
}

}  // namespace orca
