// orca_adjoint.hip -- adjoint (vector-Jacobian product) of one recorded step.
//
// The step is x' = x + dt v', v_next = v', with v' the velocity choice of
// section 3 made from the state at the step's start.  Given dL/dx' and
// dL/dv_next, k_backward handles each agent i (in the recorded step's cell
// order, so a wave's neighbours and atomics are close together):
//   g = dL/dv'_i = dL/dv_next_i + dt dL/dx'_i;
//   refetch from the tape the (at most five) half-planes that fix v'_i
//   (orca_adjoint.h), push g back through the programs to those half-planes,
//   to vhat_i and to v_max, then through each half-plane to its relative
//   position P = x_j - x_i, relative velocity V = v_i - v_j, v_i (through
//   v_i + u/2) and tau;
//   scatter P and V gradients to neighbours j: within the block's own range
//   of sorted indices into LDS, outside it with float64 atomics into
//   accumulators indexed by the step's sorted index; then store agent i's
//   own share (summed over its rows) plus the block's shares for it beside
//   them.
// k_backward_finish then writes dL/dx = dL/dx' + (scattered part), dL/dv
// (scattered part) by agent id, adds the per-scene v_max and tau gradients,
// and clears the float64 accumulators for the next use.
#include <hip/hip_runtime.h>

#include "orca_internal.h"

namespace orca {

__device__ __forceinline__ double wave_sum_f64(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Held to the registers of three waves per SIMD (a few bytes of spill): the
// kernel waits on its neighbour gathers and float64 chains, which a third
// wave covers better than the unconstrained two.
constexpr int kBackBlock = 256;  // threads (sorted indices) per k_backward block

__global__ __launch_bounds__(kBackBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_backward(
    BackArgs a)
{
    // sorted index, neighbouring tiles on one XCD (the atomics on shared
    // neighbours come from one XCD's waves)
    const int32_t b0 = xcd_tile(blockIdx.x, gridDim.x) * kBackBlock;
    const int32_t s = b0 + threadIdx.x;
    const int32_t n = a.n;
    const bool live = s < n;
    // the shares of neighbours within this block's own sorted range: summed
    // in LDS and stored with each agent's own share, so only neighbours
    // outside the block take global atomics
    __shared__ double lacc[4][kBackBlock];
#pragma unroll
    for (int c = 0; c < 4; ++c) lacc[c][threadIdx.x] = 0.0;
    __syncthreads();
    int32_t sc = 0;
    double gvmax = 0.0, gtau = 0.0;
    double gvix = 0.0, gviy = 0.0, gxi = 0.0, gyi = 0.0;
    if (live) {
        const int32_t i = a.sid[s];
        // a recorded step's scenes keep their index ranges in cell order
        sc = a.agent_scene[s];
        const SceneDev p = a.sp[sc];
        const TapeCode tc = a.codes[s];
        const float4 me = a.state[s];
        const double tau = (double)p.tau, dt = (double)p.dt;
        const double inv_tau = 1.0 / tau, inv_dt = 1.0 / dt;  // as the forward step has them
        const double ri = (double)(a.radius ? a.radius[i] : p.radius);
        const double vmax = (double)(a.max_speed ? a.max_speed[i] : p.vmax);
        const double vix = (double)me.z, viy = (double)me.w;
        double vhx, vhy, gx, gy;
        if (a.pref2) {
            const float2 ph = a.pref2[i];
            vhx = (double)ph.x;
            vhy = (double)ph.y;
        } else {
            vhx = (double)a.pref[i];
            vhy = (double)a.pref[n + i];
        }
        if (a.g_in4) {
            const float4 gn = a.g_in4[i];
            gx = (double)gn.z + dt * (double)gn.x;
            gy = (double)gn.w + dt * (double)gn.y;
        } else {
            gx = (double)a.g_vel_next[i] + dt * (double)a.g_pos_next[i];
            gy = (double)a.g_vel_next[n + i] + dt * (double)a.g_pos_next[n + i];
        }
        int r[kSlots];
        slot_rows(tc, r);
        RowGeom rows[kSlots];
        double Rq[kSlots];
        int32_t js[kSlots];
#pragma unroll
        for (int q = 0; q < kSlots; ++q) {
            js[q] = -1;
            rows[q] = RowGeom{};
            Rq[q] = 0.0;
            if (r[q] >= 0) {
                // sorted index of the neighbour; bit 31: agent i does not come
                // first of the pair
                const int32_t entry = a.nbr[(int64_t)r[q] * a.ld + s];
                const int32_t j = entry & 0x7fffffff;
                const float4 o = a.state[j];
                rows[q].Px = (double)o.x - (double)me.x;
                rows[q].Py = (double)o.y - (double)me.y;
                rows[q].Vx = vix - (double)o.z;
                rows[q].Vy = viy - (double)o.w;
                rows[q].first = entry >= 0;
                Rq[q] = ri + (double)(a.radius ? a.radius[a.sid[j]] : p.radius);
                row_geom(rows[q], Rq[q], tau, dt, inv_tau, inv_dt, vix, viy);
                js[q] = j;
            }
        }
        SlotGrads sg;
        sg.clear();
        double gvhx = 0.0, gvhy = 0.0;
        choice_vjp(rows, tc, vmax, vhx, vhy, gx, gy, sg, gvhx, gvhy, gvmax);
        // agent i's own share is summed over its slots first: four atomics
        // per neighbour outside the block, none for i
#pragma unroll
        for (int q = 0; q < kSlots; ++q) {
            if (js[q] < 0) continue;
            double gPx = 0.0, gPy = 0.0, gVx = 0.0, gVy = 0.0;
            row_vjp(rows[q], Rq[q], tau, dt, inv_tau, inv_dt, vix, viy, sg.gnx[q], sg.gny[q],
                    sg.gb[q], gPx, gPy, gVx, gVy, gtau, gvix, gviy);
            const int32_t j = js[q];
            // P = x_j - x_i, V = v_i - v_j
            const uint32_t lj = (uint32_t)(j - b0);
            if (lj < (uint32_t)kBackBlock) {
                atomicAdd(&lacc[0][lj], gPx);
                atomicAdd(&lacc[1][lj], gPy);
                atomicAdd(&lacc[2][lj], -gVx);
                atomicAdd(&lacc[3][lj], -gVy);
            } else {
                atomicAdd(&a.acc[j], gPx);
                atomicAdd(&a.acc[n + j], gPy);
                atomicAdd(&a.acc[2 * n + j], -gVx);
                atomicAdd(&a.acc[3 * n + j], -gVy);
            }
            gxi -= gPx;
            gyi -= gPy;
            gvix += gVx;
            gviy += gVy;
        }
        if (a.g_pref2) {
            float2 gp = a.g_pref2[i];
            gp.x += (float)gvhx;
            gp.y += (float)gvhy;
            a.g_pref2[i] = gp;
        } else {
            a.g_pref[i] += (float)gvhx;
            a.g_pref[n + i] += (float)gvhy;
        }
        if (a.max_speed) gvmax = 0.0;  // the agent's own max speed is a constant here
    }
    __syncthreads();
    if (live) {
        // the agent's own share and the block's shares for it: each sorted
        // index is written by its own lane only, so plain stores beside the
        // other blocks' atomics
        a.own[s] = gxi + lacc[0][threadIdx.x];
        a.own[n + s] = gyi + lacc[1][threadIdx.x];
        a.own[2 * n + s] = gvix + lacc[2][threadIdx.x];
        a.own[3 * n + s] = gviy + lacc[3][threadIdx.x];
    }
    // per-scene parameters: one atomic per wave when the wave is one scene
    const int32_t sc0 = __shfl(sc, 0, 64);
    const uint64_t same = __ballot(!live || sc == sc0);
    if (same == ~0ull) {
        const double sv = wave_sum_f64(gvmax), st = wave_sum_f64(gtau);
        if ((threadIdx.x & 63) == 0) {
            atomicAdd(&a.acc_scene[sc0], sv);
            atomicAdd(&a.acc_scene[a.n_scenes + sc0], st);
        }
    } else if (live) {
        atomicAdd(&a.acc_scene[sc], gvmax);
        atomicAdd(&a.acc_scene[a.n_scenes + sc], gtau);
    }
}

__global__ __launch_bounds__(256) void k_backward_finish(BackArgs a)
{
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;  // sorted index
    const int32_t n = a.n;
    if (s < n) {
        const int32_t i = a.sid[s];
        double gpx, gpy;
        if (a.g_in4) {
            const float4 gn = a.g_in4[i];
            gpx = (double)gn.x;
            gpy = (double)gn.y;
        } else {
            gpx = (double)a.g_pos_next[i];
            gpy = (double)a.g_pos_next[n + i];
        }
        const float gx = (float)(gpx + (a.own[s] + a.acc[s]));
        const float gy = (float)(gpy + (a.own[n + s] + a.acc[n + s]));
        const float gvx = (float)(a.own[2 * n + s] + a.acc[2 * n + s]);
        const float gvy = (float)(a.own[3 * n + s] + a.acc[3 * n + s]);
        if (a.g_out4) {
            a.g_out4[i] = make_float4(gx, gy, gvx, gvy);
        } else {
            a.g_pos[i] = gx;
            a.g_pos[n + i] = gy;
            a.g_vel[i] = gvx;
            a.g_vel[n + i] = gvy;
        }
        a.acc[s] = 0.0;
        a.acc[n + s] = 0.0;
        a.acc[2 * n + s] = 0.0;
        a.acc[3 * n + s] = 0.0;
    }
    if (s < a.n_scenes) {  // per-scene parameters, scene s
        if (a.g_max_speed) a.g_max_speed[s] += (float)a.acc_scene[s];
        if (a.g_time_horizon) a.g_time_horizon[s] += (float)a.acc_scene[a.n_scenes + s];
        a.acc_scene[s] = 0.0;
        a.acc_scene[a.n_scenes + s] = 0.0;
    }
}

__global__ __launch_bounds__(256) void k_backward_prep(const float *__restrict__ pref,
                                                       float2 *__restrict__ pref2,
                                                       float2 *__restrict__ g_pref2, int32_t n)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    pref2[i] = make_float2(pref[i], pref[n + i]);
    g_pref2[i] = make_float2(0.f, 0.f);
}

__global__ __launch_bounds__(256) void k_backward_post(const float2 *__restrict__ g_pref2,
                                                       float *__restrict__ g_pref, int32_t n)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float2 g = g_pref2[i];
    g_pref[i] += g.x;
    g_pref[n + i] += g.y;
}

hipError_t launch_backward_prep(const float *pref, float2 *pref2, float2 *g_pref2, int32_t n,
                                hipStream_t st)
{
    if (n > 0)
        hipLaunchKernelGGL(k_backward_prep, dim3((n + 255) / 256), dim3(256), 0, st, pref, pref2,
                           g_pref2, n);
    return hipGetLastError();
}

hipError_t launch_backward_post(const float2 *g_pref2, float *g_pref, int32_t n, hipStream_t st)
{
    if (n > 0)
        hipLaunchKernelGGL(k_backward_post, dim3((n + 255) / 256), dim3(256), 0, st, g_pref2,
                           g_pref, n);
    return hipGetLastError();
}

hipError_t launch_backward(const BackArgs &a, hipStream_t st)
{
    if (a.n > 0)
        hipLaunchKernelGGL(k_backward, dim3((a.n + kBackBlock - 1) / kBackBlock), dim3(kBackBlock),
                           0, st, a);
    const int32_t m = a.n > a.n_scenes ? a.n : a.n_scenes;
    if (m > 0) hipLaunchKernelGGL(k_backward_finish, dim3((m + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace orca
