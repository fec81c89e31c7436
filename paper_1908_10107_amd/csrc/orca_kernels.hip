// orca_kernels.hip -- gfx950 kernels of the ORCA crowd step.
//
// One step, in launch order (all on one stream, no host synchronisation):
//   k_bbox        per-scene bounding box of the positions (ordered-int atomics)
//   k_grid        per-scene cell size / origin / dimensions and the cell-key
//                 base of every scene (one block)
//   k_key         cell key of every agent and its rank inside the cell
//                 (histogram by atomic increment); with spawning and removal,
//                 absent agents go to one extra cell sorted after every scene
//   k_scan_sums   per-tile sums of the cell counts
//   k_scan_apply  exclusive scan -> cell_start, counts cleared for the next step
//   k_scatter     counting-sort scatter: agents into cell order (float4 x,y,vx,vy)
//   k_knn         gather over the cells within neighbor_dist (each row over the
//                 disc's chord), K nearest by float32 squared distance held as
//                 packed 64-bit keys in registers
//   k_lp          float64 half-planes in registers (LDS above 16 rows),
//                 incremental 2D LP; feasible agents
//                 write their result, the rest are appended to a fallback list
//   k_fallback    persistent over the fallback list: least-penetration 3D LP,
//                 then the 2D LP on the relaxed half-planes
// Messages: section 3 / Fig. 2 (binning, radius filter); half-planes: Fig. 1;
// LP and its infeasible case: section 3.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "orca_internal.h"

namespace orca {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ uint32_t ord_from_float(float f)
{
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float float_from_ord(uint32_t o)
{
    uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    return __uint_as_float(u);
}

template <typename T>
__device__ __forceinline__ T wave_reduce_min(T v)
{
    for (int o = 32; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_reduce_max(T v)
{
    for (int o = 32; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_reduce_sum_u32(uint32_t v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Squared distance in float32 with every operation rounded on its own (no
// fused multiply-add): the neighbour set is decided by this value.  The
// squares are added as absolute values (input modifiers, no instruction):
// the same value for any finite input, and a NaN from non-finite positions
// comes out with its sign bit clear, so its bit pattern exceeds every
// distance limit.
__device__ __forceinline__ float dist2_f32(float xi, float yi, float xj, float yj)
{
#pragma clang fp contract(off)
    const float dx = xj - xi;
    const float dy = yj - yi;
    const float sx = dx * dx;
    const float sy = dy * dy;
    return fabsf(sx) + fabsf(sy);
}

// ------------------------------------------------------------------ grid

__global__ void k_scene_of_agent(const int32_t *__restrict__ off, int32_t n_scenes,
                                 int32_t *__restrict__ agent_scene, int32_t n)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t lo = 0, hi = n_scenes - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    agent_scene[i] = lo;
}

__global__ void k_reset_bbox(uint32_t *__restrict__ bbox, int32_t n_scenes)
{
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_scenes) return;
    bbox[4 * s + 0] = 0xffffffffu;
    bbox[4 * s + 1] = 0xffffffffu;
    bbox[4 * s + 2] = 0u;
    bbox[4 * s + 3] = 0u;
}

// Bounding box per scene.  Block b reduces chunk b (at most kBboxChunk agents
// of one scene, listed by the host when the scene set changes) in registers
// and LDS, then folds it into its scene with four atomics: a 1M-agent scene
// costs 128 x 4 atomics instead of one set per 256 agents.  Blocks of 1024
// threads keep more of a chunk's loads in flight than 256 (few chunks, so few
// blocks).
// pos4 (resident steps): the positions in the previous step's cell order,
// whose scenes occupy the same index ranges as in agent order.
__global__ __launch_bounds__(kBboxBlock) void k_bbox(const float *__restrict__ pos, int32_t n,
                                              const float4 *__restrict__ pos4,
                                              const int2 *__restrict__ chunks,
                                              const int32_t *__restrict__ off,
                                              uint32_t *__restrict__ bbox)
{
    __shared__ uint32_t red[kBboxBlock / 64][4];
    const int2 ch = chunks[blockIdx.x];  // (scene, first agent)
    const int32_t end = min(ch.y + kBboxChunk, off[ch.x + 1]);
    uint32_t mnx = 0xffffffffu, mny = 0xffffffffu, mxx = 0u, mxy = 0u;
    for (int32_t i = ch.y + threadIdx.x; i < end; i += blockDim.x) {
        float px, py;
        if (pos4) {
            const float2 q = *reinterpret_cast<const float2 *>(&pos4[i]);
            px = q.x;
            py = q.y;
        } else {
            px = pos[i];
            py = pos[n + i];
        }
        const uint32_t ox = ord_from_float(px);
        const uint32_t oy = ord_from_float(py);
        mnx = min(mnx, ox);
        mny = min(mny, oy);
        mxx = max(mxx, ox);
        mxy = max(mxy, oy);
    }
    mnx = wave_reduce_min(mnx);
    mny = wave_reduce_min(mny);
    mxx = wave_reduce_max(mxx);
    mxy = wave_reduce_max(mxy);
    const int32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        red[wave][0] = mnx;
        red[wave][1] = mny;
        red[wave][2] = mxx;
        red[wave][3] = mxy;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int32_t w = 1; w < kBboxBlock / 64; ++w) {
            mnx = min(mnx, red[w][0]);
            mny = min(mny, red[w][1]);
            mxx = max(mxx, red[w][2]);
            mxy = max(mxy, red[w][3]);
        }
        const int32_t s = ch.x;
        atomicMin(&bbox[4 * s + 0], mnx);
        atomicMin(&bbox[4 * s + 1], mny);
        atomicMax(&bbox[4 * s + 2], mxx);
        atomicMax(&bbox[4 * s + 3], mxy);
    }
}

// Grid of every scene.  Cells are square, neighbor_dist * (1 + 2^-10) / c
// wide with c = 2, 3 or 4 cells per neighbor_dist chosen per scene from its
// density and K, so two agents closer than neighbor_dist (also after float32
// rounding of their squared distance) always sit within c cells of each other
// in x and in y (the neighbour search reads the disc's chords over them).  If the
// total number of cells would exceed the budget, all cells are widened by a
// common factor (more candidates per agent, same neighbours).  With spawning
// and removal on (life), one more cell after all scenes' cells takes the
// absent agents.  Also resets the bounding-box accumulators and the fallback
// counter for the next use.
__global__ __launch_bounds__(256) void k_grid(int32_t n_scenes, const int32_t *__restrict__ off,
                                              const SceneDev *__restrict__ sp,
                                              uint32_t *__restrict__ bbox,
                                              GridDev *__restrict__ grid,
                                              Counters *__restrict__ counters, uint32_t max_cells,
                                              int32_t life)
{
    __shared__ unsigned long long red[4];
    double f = 1.0;
    for (int iter = 0; iter < 24; ++iter) {
        unsigned long long local = 0;
        for (int32_t s = threadIdx.x; s < n_scenes; s += blockDim.x) {
            GridDev g;
            const float x0 = float_from_ord(bbox[4 * s + 0]);
            const float y0 = float_from_ord(bbox[4 * s + 1]);
            const float x1 = float_from_ord(bbox[4 * s + 2]);
            const float y1 = float_from_ord(bbox[4 * s + 3]);
            const double ex = (double)x1 - (double)x0, ey = (double)y1 - (double)y0;
            // cells per neighbor_dist: the 3 x 3 cells around an agent, which the
            // neighbour search reads first, should hold about 2.75 K agents at the
            // scene's mean density (fewer and the list is not full after them,
            // more and they are read for nothing): 2 for sparse crowds or large
            // K, up to 4 for dense crowds with a long neighbor_dist
            const double nd = (double)sp[s].nd;
            int32_t cpn = kMinCellsPerNd;
            if (sp[s].k > 0 && isfinite(ex) && isfinite(ey)) {
                const double area = fmax(ex * ey, nd * nd);
                const double rho = (double)(off[s + 1] - off[s]) / area;
                const double c = rint(nd * sqrt(9.0 * rho / (2.75 * (double)sp[s].k)));
                cpn = (int32_t)fmin(fmax(c, (double)kMinCellsPerNd), (double)kMaxCellsPerNd);
            }
            g.cell = nd * kCellMargin * f / (double)cpn;
            const bool ok = off[s + 1] > off[s] && isfinite(ex) && isfinite(ey) && ex >= 0.0 &&
                            ey >= 0.0 && iter < 23;
            if (ok) {
                g.x0 = x0;
                g.y0 = y0;
                const double nxd = floor(ex / g.cell) + 1.0, nyd = floor(ey / g.cell) + 1.0;
                g.nx = (int32_t)fmin(nxd, (double)(1 << 22));
                g.ny = (int32_t)fmin(nyd, (double)(1 << 22));
            } else {
                // empty, non-finite, or out of budget: one cell holds the whole scene
                g.x0 = 0.0;
                g.y0 = 0.0;
                g.cell = 1e300;
                g.nx = 1;
                g.ny = 1;
            }
            g.base = 0;
            g.pad = 0;
            grid[s] = g;
            local += (unsigned long long)g.nx * (unsigned long long)g.ny;
        }
        for (int o = 32; o > 0; o >>= 1) local += __shfl_xor(local, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = local;
        __syncthreads();
        const unsigned long long total = red[0] + red[1] + red[2] + red[3];
        __syncthreads();
        if (total <= (unsigned long long)max_cells) break;
        f *= sqrt((double)total / (double)max_cells) * 1.05;
    }
    // first cell of each scene: an exclusive scan of the scenes' cell counts,
    // a block's width of scenes at a time (each thread reads back the grids it
    // wrote itself); the total fits 32 bits, being at most max_cells
    __shared__ uint32_t wsum[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
    uint32_t carry = 0;
    for (int32_t s0 = 0; s0 < n_scenes; s0 += blockDim.x) {
        const int32_t s = s0 + threadIdx.x;
        const uint32_t c = s < n_scenes ? (uint32_t)grid[s].nx * (uint32_t)grid[s].ny : 0u;
        uint32_t inc = c;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(inc, o, 64);
            if (lane >= o) inc += y;
        }
        if (lane == 63) wsum[wave] = inc;
        __syncthreads();
        uint32_t wprefix = 0, total = 0;
        for (int w = 0; w < waves; ++w) {
            wprefix += w < wave ? wsum[w] : 0u;
            total += wsum[w];
        }
        if (s < n_scenes) grid[s].base = (int32_t)(carry + wprefix + inc - c);
        carry += total;
        __syncthreads();  // wsum is reused
    }
    if (threadIdx.x == 0) {
        counters->total_cells = carry + (life ? 1u : 0u);
        counters->n_fallback = 0;
    }
    if (threadIdx.x < kXcds) counters->tiles[threadIdx.x] = 0u;
    __syncthreads();
    for (int32_t s = threadIdx.x; s < n_scenes; s += blockDim.x) {
        bbox[4 * s + 0] = 0xffffffffu;
        bbox[4 * s + 1] = 0xffffffffu;
        bbox[4 * s + 2] = 0u;
        bbox[4 * s + 3] = 0u;
    }
}

// Cell (cx, cy) of a position in a scene's grid, clamped to the grid.  k_key
// and k_knn both take it from the agent's float32 coordinates, so they agree.
__device__ __forceinline__ void cell_of(const GridDev &g, float x, float y, int32_t &cx,
                                        int32_t &cy)
{
    double fx = floor(((double)x - g.x0) / g.cell);
    double fy = floor(((double)y - g.y0) / g.cell);
    fx = fmin(fmax(fx, 0.0), (double)(g.nx - 1));
    fy = fmin(fmax(fy, 0.0), (double)(g.ny - 1));
    cx = (int32_t)fx;
    cy = (int32_t)fy;
}

// Cell key of every agent; an absent agent (not yet spawned at the step
// counters->step, or removed) goes to the last cell, so it sorts after every
// present agent and no cell of a scene holds it.  That cell can hold most of
// the agents, so its ranks are taken with one atomic per wave.  pos4
// (resident steps, never with spawning): positions in the previous step's
// cell order; key and rank are then indexed by that order.
__global__ __launch_bounds__(256) void k_key(const float *__restrict__ pos, int32_t n,
                                             const float4 *__restrict__ pos4,
                                             const int32_t *__restrict__ agent_scene,
                                             const GridDev *__restrict__ grid,
                                             int32_t *__restrict__ key,
                                             int32_t *__restrict__ rank,
                                             int32_t *__restrict__ counts,
                                             const int32_t *__restrict__ spawn_step,
                                             const uint8_t *__restrict__ state,
                                             const Counters *__restrict__ counters)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < n;
    bool absent = false;
    if (spawn_step) {  // the same on every lane
        if (valid) absent = spawn_step[i] > counters->step || state[i] != 0;
        const uint64_t m = __ballot(absent);
        if (m) {
            const int32_t k = (int32_t)counters->total_cells - 1;
            const int leader = __ffsll((unsigned long long)m) - 1;
            int32_t base = 0;
            if ((int)(threadIdx.x & 63) == leader) base = atomicAdd(&counts[k], __popcll(m));
            base = __shfl(base, leader, 64);
            if (absent) {
                const int32_t before = (int32_t)__builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                key[i] = k;
                rank[i] = base + before;
            }
        }
    }
    if (pos4) {
        // resident step: agents come in the previous step's cell order, so
        // neighbouring lanes mostly share a cell.  Each run of lanes with
        // the same key takes its ranks with one atomic (the run's first lane
        // adds the run's length and hands the base to the others).
        int32_t k = -1;
        if (valid) {
            const GridDev g = grid[agent_scene[i]];
            const float2 q = *reinterpret_cast<const float2 *>(&pos4[i]);
            int32_t cx, cy;
            cell_of(g, q.x, q.y, cx, cy);
            k = g.base + cy * g.nx + cx;
        }
        const int lane = (int)(threadIdx.x & 63);
        const int32_t kp = __shfl_up(k, 1, 64);
        const uint64_t heads = __ballot(lane == 0 || kp != k);
        const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
        const int start = 63 - __clzll((long long)(heads & upto));
        const uint64_t above = heads & ~upto;
        const int next = above ? __ffsll((unsigned long long)above) - 1 : 64;
        int32_t base = 0;
        if (valid && lane == start) base = atomicAdd(&counts[k], next - start);
        base = __shfl(base, start, 64);
        if (valid) {
            key[i] = k;
            rank[i] = base + (lane - start);
        }
        return;
    }
    if (!valid || absent) return;
    const GridDev g = grid[agent_scene[i]];
    int32_t cx, cy;
    cell_of(g, pos[i], pos[n + i], cx, cy);
    const int32_t k = g.base + cy * g.nx + cx;
    key[i] = k;
    rank[i] = atomicAdd(&counts[k], 1);
}

__global__ __launch_bounds__(kScanBlock) void k_scan_sums(const int32_t *__restrict__ counts,
                                                          const Counters *__restrict__ counters,
                                                          uint32_t *__restrict__ partial)
{
    __shared__ uint32_t red[kScanBlock / 64];
    const uint32_t total = counters->total_cells;
    const uint32_t base = blockIdx.x * kScanTile;
    if (base >= total) {
        if (threadIdx.x == 0) partial[blockIdx.x] = 0;
        return;
    }
    uint32_t s = 0;
#pragma unroll
    for (int t = 0; t < kScanItems; ++t) {
        const uint32_t c = base + t * kScanBlock + threadIdx.x;
        if (c < total) s += (uint32_t)counts[c];
    }
    s = wave_reduce_sum_u32(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kScanBlock / 64; ++w) t += red[w];
        partial[blockIdx.x] = t;
    }
}

// cell_start[c] = sum of counts before c; cell_start[total] = n.  Counts are
// zeroed after reading so the next histogram starts from zero.  In a step
// with spawning and removal (advance), the step counter moves on here: k_key,
// its only reader, has finished.
__global__ __launch_bounds__(kScanBlock) void k_scan_apply(int32_t *__restrict__ counts,
                                                           Counters *__restrict__ counters,
                                                           const uint32_t *__restrict__ partial,
                                                           int32_t *__restrict__ cell_start,
                                                           int32_t n, int32_t advance)
{
    __shared__ uint32_t wsum[kScanBlock / 64];
    __shared__ uint32_t s_prefix;
    const uint32_t total = counters->total_cells;
    const uint32_t base = blockIdx.x * kScanTile;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        cell_start[total] = n;
        if (advance) counters->step += 1;
    }
    if (base >= total) return;
    // prefix of the earlier tiles
    uint32_t p = 0;
    for (uint32_t b = threadIdx.x; b < blockIdx.x; b += kScanBlock) p += partial[b];
    p = wave_reduce_sum_u32(p);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = p;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kScanBlock / 64; ++w) t += wsum[w];
        s_prefix = t;
    }
    __syncthreads();
    // each thread owns kScanItems consecutive cells
    const uint32_t c0 = base + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t run = 0;
#pragma unroll
    for (int t = 0; t < kScanItems; ++t) {
        const uint32_t c = c0 + t;
        v[t] = c < total ? (uint32_t)counts[c] : 0u;
        run += v[t];
    }
    // exclusive scan of the per-thread sums across the block
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = run;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    __syncthreads();
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t wprefix = 0;
    for (int w = 0; w < wave; ++w) wprefix += wsum[w];
    uint32_t acc = s_prefix + wprefix + inc - run;
#pragma unroll
    for (int t = 0; t < kScanItems; ++t) {
        const uint32_t c = c0 + t;
        if (c < total) {
            cell_start[c] = (int32_t)acc;
            counts[c] = 0;
        }
        acc += v[t];
    }
}

// Counting-sort scatter into cell order.  From the caller's arrays (agent
// order), or in a resident step from the previous step's cell order (src4,
// ids sid_prev, goals / preferred velocities sg_prev).  sg_cur (nullable)
// receives the goals or preferred velocities in the new order: from sg_prev,
// or from the caller's [2, N] array sg_src.
__global__ __launch_bounds__(256) void k_scatter(const float *__restrict__ pos,
                                                 const float *__restrict__ vel, int32_t n,
                                                 const float4 *__restrict__ src4,
                                                 const int32_t *__restrict__ sid_prev,
                                                 const float2 *__restrict__ sg_prev,
                                                 const float *__restrict__ sg_src,
                                                 float2 *__restrict__ sg_cur,
                                                 const int32_t *__restrict__ key,
                                                 const int32_t *__restrict__ rank,
                                                 const int32_t *__restrict__ cell_start,
                                                 float4 *__restrict__ sorted,
                                                 int32_t *__restrict__ sid,
                                                 int32_t *__restrict__ inv,
                                                 const float *__restrict__ radius,
                                                 float *__restrict__ srad)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t k = key[i];
    const int32_t d = cell_start[k] + rank[i];
    float4 r;
    int32_t id = i;
    if (src4) {
        r = src4[i];
        id = sid_prev[i];
        if (sg_cur) sg_cur[d] = sg_prev[i];
    } else {
        r.x = pos[i];
        r.y = pos[n + i];
        r.z = vel ? vel[i] : 0.f;
        r.w = vel ? vel[n + i] : 0.f;
        if (sg_cur) sg_cur[d] = make_float2(sg_src[i], sg_src[n + i]);
    }
    if (radius) srad[d] = radius[id];
    sorted[d] = r;
    sid[d] = id;
    inv[id] = d;
}

// Velocities into the sorted copy for a velocity pass on an existing grid;
// also starts the pass's fallback list and tile queues empty.
__global__ __launch_bounds__(256) void k_fill_vel(const float *__restrict__ vel, int32_t n,
                                                  const int32_t *__restrict__ inv,
                                                  float4 *__restrict__ sorted,
                                                  Counters *__restrict__ counters)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) counters->n_fallback = 0;
    if (i < 8) counters->tiles[i] = 0u;
    if (i >= n) return;
    float2 *dst = reinterpret_cast<float2 *>(&sorted[inv[i]]) + 1;
    *dst = make_float2(vel[i], vel[n + i]);
}

// ------------------------------------------------------------------ neighbours

// The running neighbour list of one lane: KMAX sorted 64-bit keys
// (d2 bits + kKeyBias) << 32 | id + 1.  The bias lifts the top 12 bits of
// every key to a positive normal double's exponent field (the float32 d2 bits
// stay below the infinity pattern), and positive doubles order like their bit
// patterns, so one v_min_f64 / v_max_f64 on the patterns compares two keys:
// by d2, then by id.  For K < KMAX the first KMAX - K slots hold the key 0,
// below every real key, so the K nearest always sit in the last K slots and
// the K-th is best[KMAX - 1] whatever K is.  Unfilled slots hold the pattern
// of +infinity.
constexpr uint32_t kKeyBias = 0x00100000u;
constexpr uint64_t kKeyEmpty = 0x7ff0000000000000ull;

// Offer key to the sorted list.  Each slot takes the larger of its lower
// neighbour and the smaller of itself and the key: the lower slots shift up
// past the key, the key lands in the first slot above it, the rest stay.  A
// key above the last slot changes nothing.  Each step is one v_min_f64 or
// v_max_f64 on the slot in place, written out because fmin / fmax first quiet
// every operand that the compiler cannot prove is not a signalling NaN (one
// more instruction per slot); no key is a NaN pattern, and each result is one
// operand's exact pattern.
__device__ __forceinline__ void key_min_into(uint64_t &slot, uint64_t key)
{
    asm volatile("v_min_f64 %0, %1, %0" : "+v"(slot) : "v"(key));
}
__device__ __forceinline__ void key_max_into(uint64_t &slot, uint64_t lower)
{
    asm volatile("v_max_f64 %0, %1, %0" : "+v"(slot) : "v"(lower));
}
template <int KMAX>
__device__ __forceinline__ void knn_offer(uint64_t (&best)[KMAX], uint64_t key)
{
#pragma unroll
    for (int k = KMAX - 1; k > 0; --k) {
        key_min_into(best[k], key);
        key_max_into(best[k], best[k - 1]);
    }
    key_min_into(best[0], key);
}

// Offer the candidates [i, ie) of one row run (sorted indices) to the sorted
// key list.  lim is the largest float32 bit pattern of d2, plus kKeyBias, that
// can still enter: strictly inside neighbor_dist and no farther than the
// list's K-th entry (d2 >= 0, so the bit patterns order like the values; a
// NaN's pattern exceeds every limit).  The agent itself (id myid) is skipped
// when it comes up for insertion.
template <int KMAX>
__device__ __forceinline__ void knn_run(uint64_t (&best)[KMAX], uint32_t &lim, uint32_t nd_lim,
                                        float mx, float my, uint32_t myid, int32_t i, int32_t ie,
                                        const float4 *__restrict__ sorted,
                                        const int32_t *__restrict__ sid)
{
    auto offer = [&](uint32_t hb, uint32_t id) __attribute__((always_inline)) {
        if (id == myid) return;
        knn_offer<KMAX>(best, ((uint64_t)hb << 32) | (id + 1u));
        lim = min(nd_lim, (uint32_t)(best[KMAX - 1] >> 32));
    };
    // candidates two at a time: their positions and ids are loaded together,
    // so one memory latency covers the pair (four in flight need the
    // registers of a sixth wave per SIMD, which hides latency better)
    constexpr int kBatch = 2;
    for (; i + kBatch <= ie; i += kBatch) {
        float4 o[kBatch];
        uint32_t idb[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) o[u] = sorted[i + u];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) idb[u] = (uint32_t)sid[i + u];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const uint32_t hb = __float_as_uint(dist2_f32(mx, my, o[u].x, o[u].y)) + kKeyBias;
            if (hb <= lim) offer(hb, idb[u]);
        }
    }
    for (; i < ie; ++i) {
        const float4 o = sorted[i];
        const uint32_t hb = __float_as_uint(dist2_f32(mx, my, o.x, o.y)) + kKeyBias;
        if (hb <= lim) offer(hb, (uint32_t)sid[i]);
    }
}

// Offer every candidate within reach of an agent (me, id myid, its cell's grid
// g, float32 neighbor_dist ndf) to its sorted key list, each row of cells over
// the run its chord of the disc touches (one contiguous run of sorted
// indices).  Cells are about nd/c wide (c = 2, 3 or 4, per scene), so the
// disc of radius nd reaches c rows and columns out (fewer once the grid was
// widened).  The chords are taken a little wider than the radius, so
// rounding of the cell arithmetic or of the float32 distance never drops a
// neighbour: the distance test decides.
//
// Order: first the 3 x 3 cells around the agent's own (k_grid sizes cells so
// that they hold about 2.75 K agents at the scene's mean density, enough for
// the K nearest), then the rest, with each chord cut to the list's current
// limit (the K-th distance once the list is full): the list fills with near
// candidates first and the outer cells offer few, which a wave would
// otherwise pay for with an insertion whenever any of its lanes inserts.  The
// set that can enter is the same, so the result is.
template <int KMAX>
__device__ __forceinline__ void knn_rows(uint64_t (&best)[KMAX], uint32_t &lim, uint32_t nd_lim,
                                         float4 me, uint32_t myid, const GridDev &g, float ndf,
                                         const float4 *__restrict__ sorted,
                                         const int32_t *__restrict__ sid,
                                         const int32_t *__restrict__ cell_start)
{
    int32_t cx, cy;  // the agent's cell
    cell_of(g, me.x, me.y, cx, cy);
    const double cell = g.cell, nd = (double)ndf;
    // rows and columns the disc of radius nd can reach: nd / cell rounded up
    // (cells are a little wider than nd / c, or wider still once the grid was
    // widened)
    const int32_t reach = max(1, min(kMaxCellsPerNd, (int32_t)ceil(nd / cell)));
    const double px = (double)me.x, py = (double)me.y;
    const double slack = 1e-9 * (1.0 + fabs(px) + fabs(py));
    // segments (one knn_run call site keeps the registers of one row loop):
    // 0-2 the inner three columns of rows 0, -1, +1; 3-8 the columns left and
    // right of them in the same rows, and 9-14 rows -2, +2, -3, +3, -4, +4
    // (those within reach), over chords cut to the list's current limit.
    constexpr int32_t kSegs = 9 + 2 * (kMaxCellsPerNd - 1);
    // The inner segments read columns cx - 1 .. cx + 1 whatever the chord:
    // at least the columns the chord would give (every candidate is tested
    // anyway, and the order of the offers does not change the list), and
    // with cells no wider than about nd / 2 exactly those.
    // outer chords: columns from the chord's ends times 1 / cell (a quotient
    // off by an ulp or two only where the widened chord ends within that of
    // a cell edge, which the disc itself never reaches)
    const double inv_cell = 1.0 / cell;
#pragma unroll 1
    for (int32_t q = 0; q < kSegs; ++q) {
        int32_t i, ie;
        if (q < 3) {
            const int32_t row = cy + (q == 0 ? 0 : (q == 1 ? -1 : 1));
            if (row < 0 || row >= g.ny) continue;
            const int32_t rb = g.base + row * g.nx;
            i = cell_start[rb + max(cx - 1, 0)];
            ie = cell_start[rb + min(cx + 1, g.nx - 1) + 1];
        } else {
            // row code (dy = -1, +1, -2, +2, ...) and part: 2 left, 3 right,
            // 0 the whole chord
            const int32_t qr = q < 9 ? (q - 3) >> 1 : q - 6;
            const int32_t part = q < 9 ? 2 + ((q - 3) & 1) : 0;
            const int32_t dy = (qr & 1) ? -((qr + 1) >> 1) : (qr >> 1);
            if (dy > reach || -dy > reach) continue;
            const int32_t row = cy + dy;
            if (row < 0 || row >= g.ny) continue;
            // the chord's radius: the list's current limit, at most nd
            const double r = fmin(nd, sqrt((double)__uint_as_float(lim - kKeyBias)));
            const double rx = r * (1.0 + 1e-6) + slack;
            double dyc = 0.0;  // distance from the agent to the row's band in y
            if (dy > 0) dyc = fmax(g.y0 + (double)row * cell - py, 0.0);
            if (dy < 0) dyc = fmax(py - (g.y0 + (double)(row + 1) * cell), 0.0);
            if (dyc >= rx) continue;
            const double hw = sqrt(rx * rx - dyc * dyc);
            int32_t c0 = max((int32_t)fmax(floor((px - hw - g.x0) * inv_cell), -1.0),
                             max(cx - reach, 0));
            int32_t c1 = min((int32_t)fmin(floor((px + hw - g.x0) * inv_cell), (double)g.nx),
                             min(cx + reach, g.nx - 1));
            // the agent's own column always: an agent inside the grid's extent
            // has it in its chord anyway, one outside (a scene that is one cell
            // at origin 0 because its box is not finite) still reads its cell
            c0 = min(c0, cx);
            c1 = max(c1, cx);
            if (part == 2) {
                c1 = min(c1, cx - 2);
            } else if (part == 3) {
                c0 = max(c0, cx + 2);
            }
            if (c0 > c1) continue;
            const int32_t rb = g.base + row * g.nx;
            i = cell_start[rb + c0];
            ie = cell_start[rb + c1 + 1];
        }
        knn_run<KMAX>(best, lim, nd_lim, me.x, me.y, myid, i, ie, sorted, sid);
    }
}

// The K nearest of one agent (me, id myid, in a scene with grid g, cap K and
// float32 neighbor_dist^2 nd2) among the agents of the cells within
// neighbor_dist, strictly inside it, nearest first, ties by agent id, as
// packed keys in best (see knn_offer).  Returns the number of leading slots
// that hold the key 0 (KMAX - K; KMAX when K == 0 or nd2 admits nobody).
// The candidates come from knn_rows.
template <int KMAX>
__device__ __forceinline__ int32_t knn_search(uint64_t (&best)[KMAX], float4 me, int32_t myid,
                                              const GridDev &g, int32_t K, float nd2, float ndf,
                                              const float4 *__restrict__ sorted,
                                              const int32_t *__restrict__ sid,
                                              const int32_t *__restrict__ cell_start)
{
    // d2 < nd2 as bit patterns: at most the pattern just below nd2's (an nd2
    // that underflowed to zero admits nobody)
    if (K == 0 || !(nd2 > 0.0f)) {
#pragma unroll
        for (int k = 0; k < KMAX; ++k) best[k] = 0ull;
        return KMAX;
    }
    const int32_t pad = KMAX - K;  // leading slots that hold the key 0
#pragma unroll
    for (int k = 0; k < KMAX; ++k) best[k] = k < pad ? 0ull : kKeyEmpty;
    const uint32_t nd_lim = __float_as_uint(nd2) - 1u + kKeyBias;
    uint32_t lim = nd_lim;
    knn_rows<KMAX>(best, lim, nd_lim, me, (uint32_t)myid, g, ndf, sorted, sid, cell_start);
    return pad;
}

// Neighbour-list entry of slot k of best (pad leading slots): the
// neighbour's sorted index, with bit 31 set when this agent (id myid) does
// not come first of the pair (ids order it); -1 for an empty slot.
template <int KMAX>
__device__ __forceinline__ int32_t knn_entry(const uint64_t (&best)[KMAX], int k, int32_t pad,
                                             int32_t myid, const int32_t *__restrict__ inv)
{
    if (k < pad || best[k] == kKeyEmpty) return -1;
    const uint32_t jid = (uint32_t)(best[k] & 0xffffffffu) - 1u;
    const uint32_t later = (uint32_t)myid < jid ? 0u : 0x80000000u;
    return (int32_t)((uint32_t)inv[jid] | later);
}

// K nearest of each agent (sorted order s), as knn_search finds them (the
// candidates from knn_rows).  Writes nbr[k * ld + s] (entries as knn_entry
// gives them) and ncount[s].  Held to the registers of six waves per SIMD up
// to K = 16 and eight up to K = 10 (a few bytes of spill): the search waits on
// its candidate gathers, which the extra waves cover.
#ifndef ORCA_KNN_WAVES
#define ORCA_KNN_WAVES 6
#endif
template <int KMAX>
__global__ __launch_bounds__(512)
__attribute__((amdgpu_waves_per_eu(KMAX <= 10 ? 8 : (KMAX <= 16 ? ORCA_KNN_WAVES : 1)))) void k_knn(const float4 *__restrict__ sorted,
                                             const int32_t *__restrict__ sid,
                                             const int32_t *__restrict__ inv,
                                             const int32_t *__restrict__ cell_start,
                                             const GridDev *__restrict__ grid,
                                             const int32_t *__restrict__ agent_scene,
                                             const SceneDev *__restrict__ sp, int32_t n,
                                             int32_t *__restrict__ nbr, int32_t ld,
                                             int32_t *__restrict__ ncount,
                                             Counters *__restrict__ counters, int32_t life)
{
    const int32_t s = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    // the fallback list of this velocity pass starts empty (k_lp runs after us)
    if (s == 0) counters->n_fallback = 0;
    // absent agents sit in the last cell, after every present one
    const int32_t n_present = life ? cell_start[counters->total_cells - 1] : n;
    if (s >= n_present) return;
    const float4 me = sorted[s];
    const int32_t myid = sid[s];
    // without spawning each scene holds the same index range in cell order
    // as in agent order (its cells come in scene order), so the scene is
    // read by sorted index, not gathered by id
    const int32_t sc = agent_scene[life ? myid : s];
    const GridDev g = grid[sc];
    const int32_t K = sp[sc].k;
    const float nd2 = sp[sc].nd2;
    if (K == 0 || !(nd2 > 0.0f)) {
        ncount[s] = 0;
        return;
    }
    uint64_t best[KMAX];
    const int32_t pad = knn_search<KMAX>(best, me, myid, g, K, nd2, sp[sc].nd, sorted, sid,
                                         cell_start);
    int32_t cnt = 0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int32_t e = knn_entry<KMAX>(best, k, pad, myid, inv);
        if (e != -1) {
            nbr[(int64_t)(k - pad) * ld + s] = e;
            cnt = k - pad + 1;
        }
    }
    ncount[s] = cnt;
}

}  // namespace orca

#include "orca_lp.h"

namespace orca {

static_assert(kLpStride == kLpBlock, "LP constraint stride must equal the LP block size");

// Rows of k_lp: up to 16 in registers (static indices only), more in a
// per-lane LDS column.
constexpr int kLpRegRows = 16;
template <int KMAX, bool IN_REGS = (KMAX <= kLpRegRows)>
struct LpRows;
template <int KMAX>
struct LpRows<KMAX, true> {
    double2 n[KMAX];
    double b[KMAX];
    __device__ __forceinline__ void set(int k, double2 nk, double bk)
    {
        n[k] = nk;
        b[k] = bk;
    }
    __device__ __forceinline__ double2 N(int k) const { return n[k]; }
    __device__ __forceinline__ double B(int k) const { return b[k]; }
    __device__ __forceinline__ int project(int m, double vmax, double vhx, double vhy, double &vx,
                                          double &vy, Active *act) const
    {
        return lp2_project_regs<KMAX>(n, b, m, vmax, vhx, vhy, vx, vy, act);
    }
};
template <int KMAX>
struct LpRows<KMAX, false> {
    Lane L;
    __device__ __forceinline__ void set(int k, double2 nk, double bk)
    {
        L.n[k * kLpStride] = nk;
        L.b[k * kLpStride] = bk;
    }
    __device__ __forceinline__ double2 N(int k) const { return L.N(k); }
    __device__ __forceinline__ double B(int k) const { return L.B(k); }
    __device__ __forceinline__ int project(int m, double vmax, double vhx, double vhy, double &vx,
                                          double &vy, Active *act) const
    {
        return lp2_project<true>(L, m, 0, 0.0, vmax, vhx, vhy, vx, vy, act);
    }
};

// Where build_constraints takes an agent's neighbour entries (sorted index,
// pair-order bit 31) from: the list k_knn wrote, or registers of the fused
// velocity kernel (slot k of the unrolled loops: a static index).
struct EntriesInMemory {
    const int32_t *__restrict__ nbr;
    int32_t ld, s;
    __device__ __forceinline__ int32_t operator()(int k) const { return nbr[(int64_t)k * ld + s]; }
};
template <int KMAX>
struct EntriesInRegs {
    const int32_t (&e)[KMAX];
    __device__ __forceinline__ int32_t operator()(int k) const { return e[k]; }
};

// Load the m neighbours of agent id (state me) and build their half-planes
// into `rows`.  The neighbour loads are issued G at a time, so one memory
// latency covers each group: two with the rows in registers, which keeps the
// LP kernels within the registers of three waves per SIMD, each group's
// gathers issued while the group before it is built (k_lp at 1M agents,
// K = 16: 289 to 283 us); eight with the rows in LDS, each group loaded
// before it is built.  Neighbour ids are fetched only when they are written
// out (the pair order comes with the entry).
template <int KMAX, class Rows, class Src>
__device__ __forceinline__ void build_constraints(Rows &rows, const Src &src, int m, int32_t id,
                                                  float4 me, const SceneDev &p,
                                                  const AgentProps &ag,
                                                  const float4 *__restrict__ sorted,
                                                  const int32_t *__restrict__ sid,
                                                  int32_t *__restrict__ nbr_out, int32_t krow)
{
    constexpr int G = KMAX <= kLpRegRows ? 2 : 8;
    // combined radius r_i + r_j (section 4: people of different sizes)
    const double ri = (double)(ag.radius ? ag.radius[id] : p.radius);
    const double tau = (double)p.tau, dt = (double)p.dt;
    const double inv_tau = 1.0 / tau, inv_dt = 1.0 / dt;  // shared by every row
    const double vix = (double)me.z, viy = (double)me.w;
    if constexpr (KMAX <= kLpRegRows) {
        // every entry first (independent, coalesced loads; the rows are not
        // yet live, so their registers are free), then the neighbours G at a
        // time with the next group's gathers issued before this group's
        // half-planes are built
        int32_t e[KMAX];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) e[k] = k < m ? src(k) : 0;
        auto gather = [&](int k) __attribute__((always_inline)) -> float4 {
            return k < m ? sorted[e[k] & 0x7fffffff] : make_float4(0.f, 0.f, 0.f, 0.f);
        };
        float4 cur[G];
#pragma unroll
        for (int u = 0; u < G; ++u) cur[u] = gather(u);
#pragma unroll
        for (int k0 = 0; k0 < KMAX; k0 += G) {
            float4 nxt[G];
#pragma unroll
            for (int u = 0; u < G; ++u)
                nxt[u] = k0 + G + u < KMAX ? gather(k0 + G + u) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const int k = k0 + u;
                if (k >= KMAX) continue;
                const float rj = ag.radius && k < m ? ag.srad[e[k] & 0x7fffffff] : p.radius;
                double2 nk = make_double2(0.0, 0.0);
                double bk = 0.0;
                if (k < m) {
                    const double Px = (double)cur[u].x - (double)me.x;
                    const double Py = (double)cur[u].y - (double)me.y;
                    const double Vx = vix - (double)cur[u].z, Vy = viy - (double)cur[u].w;
                    double ux, uy, nx, ny;
                    obstacle_exit(Px, Py, Vx, Vy, ri + (double)rj, tau, dt, inv_tau, inv_dt,
                                  e[k] >= 0, ux, uy, nx, ny);
                    const double qx = vix + 0.5 * ux, qy = viy + 0.5 * uy;
                    nk = make_double2(nx, ny);
                    bk = nx * qx + ny * qy;
                }
                rows.set(k, nk, bk);
                if (nbr_out && k < krow)
                    nbr_out[(int64_t)id * krow + k] = k < m ? sid[e[k] & 0x7fffffff] : -1;
            }
#pragma unroll
            for (int u = 0; u < G; ++u) cur[u] = nxt[u];
        }
        return;
    }
#pragma unroll
    for (int k0 = 0; k0 < KMAX; k0 += G) {
        int32_t e[G];
        float4 o[G];
        float rj[G];
#pragma unroll
        for (int u = 0; u < G; ++u) e[u] = k0 + u < KMAX && k0 + u < m ? src(k0 + u) : 0;
#pragma unroll
        for (int u = 0; u < G; ++u)
            o[u] = k0 + u < KMAX && k0 + u < m ? sorted[e[u] & 0x7fffffff]
                                               : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int u = 0; u < G; ++u)
            rj[u] = ag.radius && k0 + u < KMAX && k0 + u < m ? ag.srad[e[u] & 0x7fffffff] : p.radius;
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int k = k0 + u;
            if (k >= KMAX) continue;
            double2 nk = make_double2(0.0, 0.0);
            double bk = 0.0;
            if (k < m) {
                const double Px = (double)o[u].x - (double)me.x, Py = (double)o[u].y - (double)me.y;
                const double Vx = vix - (double)o[u].z, Vy = viy - (double)o[u].w;
                double ux, uy, nx, ny;
                obstacle_exit(Px, Py, Vx, Vy, ri + (double)rj[u], tau, dt, inv_tau, inv_dt,
                              e[u] >= 0, ux, uy, nx, ny);
                const double qx = vix + 0.5 * ux, qy = viy + 0.5 * uy;
                nk = make_double2(nx, ny);
                bk = nx * qx + ny * qy;
            }
            rows.set(k, nk, bk);
            if (nbr_out && k < krow)
                nbr_out[(int64_t)id * krow + k] = k < m ? sid[e[u] & 0x7fffffff] : -1;
        }
    }
}

// sg (resident steps): the goal or preferred velocity by sorted index s.
__device__ __forceinline__ void preferred_velocity(const SceneDev &p, const AgentProps &ag,
                                                   float4 me, int32_t id, int32_t n,
                                                   const float *__restrict__ pref,
                                                   const float *__restrict__ goals,
                                                   const float2 *__restrict__ sg, int32_t s,
                                                   double &vhx, double &vhy)
{
#pragma clang fp contract(off)
    float2 g = make_float2(0.f, 0.f);
    if (sg) g = sg[s];
    else if (goals) g = make_float2(goals[id], goals[n + id]);
    else g = make_float2(pref[id], pref[n + id]);
    if (goals) {
        // walking speed toward the goal; the last step lands on it
        const double ex = (double)g.x - (double)me.x;
        const double ey = (double)g.y - (double)me.y;
        const double el = sqrt(ex * ex + ey * ey);
        const double s = (double)(ag.pref_speed ? ag.pref_speed[id] : p.pref_speed);
        const double dt = (double)p.dt;
        if (el > s * dt) {
            vhx = s * ex / el;
            vhy = s * ey / el;
        } else {
            vhx = ex / dt;
            vhy = ey / dt;
        }
    } else {
        vhx = (double)g.x;
        vhy = (double)g.y;
    }
}

// Kernel variants: plain, recording a tape for the adjoint, or with spawning
// and removal (which never records).
constexpr int kModePlain = 0, kModeRec = 1, kModeLife = 2;

template <bool LIFE>
__device__ __forceinline__ void write_result(const OutArgs &o, float mex, float mey, float dtf,
                                             int32_t id, int32_t s, int32_t n, double vx,
                                             double vy, double vhx, double vhy, uint8_t status)
{
#pragma clang fp contract(off)
    if (o.nxt) {
        // resident step: the new state stays in this step's cell order
        const double dt = (double)dtf;
        o.nxt[s] = make_float4((float)((double)mex + dt * vx), (float)((double)mey + dt * vy),
                               (float)vx, (float)vy);
        return;
    }
    if (o.new_vel) {
        o.new_vel[id] = (float)vx;
        o.new_vel[n + id] = (float)vy;
    }
    if (o.pos) {
        const double dt = (double)dtf;
        const float px = (float)((double)mex + dt * vx);
        const float py = (float)((double)mey + dt * vy);
        o.pos[id] = px;
        o.pos[n + id] = py;
        o.vel[id] = (float)vx;
        o.vel[n + id] = (float)vy;
        if (o.goals) {
            o.pref[id] = (float)vhx;
            o.pref[n + id] = (float)vhy;
        }
        if (LIFE) {
            // removed once the goal lies within the agent's own radius of its
            // new position (float64 on the float32 coordinates)
            const double ex = (double)o.goals[id] - (double)px;
            const double ey = (double)o.goals[n + id] - (double)py;
            const double sx = ex * ex;
            const double sy = ey * ey;
            const double r = (double)(o.ag.radius ? o.ag.radius[id]
                                                  : o.life.sp[o.life.agent_scene[id]].radius);
            if (sx + sy <= r * r) o.life.state[id] = 1;
        }
    }
    if (o.status) o.status[id] = status;
}

// Velocity of agent s (sorted order; state me, id id, its m neighbour
// entries from src): preferred velocity, half-planes, 2D LP.  A feasible
// agent gets its result written (and its choice recorded with REC) and false
// is returned; an agent whose projection is empty gets its fallback record in
// `it` and true is returned (its rows stay in `rows`).
template <int KMAX, int MODE, class Src>
__device__ __forceinline__ bool lp_agent(LpRows<KMAX> &rows, FallbackItem &it, const Src &src,
                                         int m, int32_t s, float4 me, int32_t id,
                                         const SceneDev &p, const OutArgs &out, int32_t n,
                                         const float4 *__restrict__ sorted,
                                         const int32_t *__restrict__ sid)
{
    constexpr bool REC = MODE == kModeRec, LIFE = MODE == kModeLife;
    double vhx, vhy;
    preferred_velocity(p, out.ag, me, id, n, out.pref, out.goals, out.sg, s, vhx, vhy);
    const float vmaxf = out.ag.max_speed ? out.ag.max_speed[id] : p.vmax;
    const double vmax = (double)vmaxf;
    double vx, vy;
    disc_clip(vmax, vhx, vhy, vx, vy);
    build_constraints<KMAX>(rows, src, m, id, me, p, out.ag, sorted, sid, out.nbr_out, out.krow);
    Active act;
    const int fail = rows.project(m, vmax, vhx, vhy, vx, vy, &act);
    if (REC) out.tape_state[s] = me;
    if (fail < 0) {
        write_result<LIFE>(out, me.x, me.y, p.dt, id, s, n, vx, vy, vhx, vhy, 0);
        if (REC) {
            TapeCode tc{};
            tc.status = 0;
            tc.p_line = (int8_t)act.line;
            tc.p_src = (int8_t)act.src;
            tc.d_plane = -1;
            tc.d_line = (int8_t)kLineNone;
            tc.d_src = (int8_t)kSrcDisc;
            out.tape_codes[s] = tc;
        }
        return false;
    }
    it.s = s;
    it.id = id;
    it.m = (int8_t)m;
    it.fail = (int8_t)fail;
    it.line = (int8_t)act.line;
    it.src = (int8_t)act.src;
    // the most violated row from the failed one on, at the last optimum
    it.worst = (int8_t)worst_row<KMAX>(rows, fail, m, vx, vy);
    it.vx = vx;
    it.vy = vy;
    it.vhx = vhx;
    it.vhy = vhy;
    it.vmax = vmaxf;
    it.dt = p.dt;
    it.mex = me.x;
    it.mey = me.y;
    return true;
}

// Hand the wave's infeasible agents to the fallback list (one atomic per
// wave): each one's record, its sort key (the failed row) and its half-planes
// in its stash slot, in stash_position order.  Every lane of the wave calls it.
template <int KMAX>
__device__ __forceinline__ void append_fallback(bool need_fb, const FallbackItem &it,
                                                const LpRows<KMAX> &rows,
                                                FallbackItem *__restrict__ fb_list,
                                                uint8_t *__restrict__ fb_key, int32_t kcap,
                                                double2 *__restrict__ stash_n,
                                                double *__restrict__ stash_b,
                                                Counters *__restrict__ counters)
{
    const uint64_t mask = __ballot(need_fb);
    if (!mask) return;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t before = __builtin_amdgcn_mbcnt_hi(
        (uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    uint32_t slot0 = 0;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    if ((int)lane == leader) slot0 = atomicAdd(&counters->n_fallback, (uint32_t)__popcll(mask));
    slot0 = __shfl(slot0, leader, 64);
    if (need_fb) {
        const uint32_t slot = slot0 + before;
        fb_list[slot] = it;
        fb_key[slot] = (uint8_t)it.fail;
        double2 *gn = stash_n + (int64_t)slot * kcap;
        double *gb = stash_b + (int64_t)slot * kcap;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            if (k < it.m) {
                const int q = stash_position(k, it);
                gn[q] = rows.N(k);
                gb[q] = rows.B(k);
            }
        }
    }
}

// One lane per agent in cell order, half-planes in registers (LDS above 16
// rows).  With the rows in registers the kernel is held to the registers of
// three waves per SIMD, four up to 10 rows: it is bound by the latency of its
// float64 chains and gathers, which another wave covers better than the
// unconstrained count (a few bytes of spill).  Feasible agents finish here;
// the others go to the fallback list.
template <int KMAX, int MODE>
__global__ __launch_bounds__(kLpBlock)
__attribute__((amdgpu_waves_per_eu(KMAX <= 10 ? 4 : (KMAX <= kLpRegRows ? 3 : 1)))) void k_lp(
    const float4 *__restrict__ sorted, const int32_t *__restrict__ sid,
    const int32_t *__restrict__ agent_scene, const SceneDev *__restrict__ sp, int32_t n,
    const int32_t *__restrict__ nbr, int32_t ld, const int32_t *__restrict__ ncount, OutArgs out,
    FallbackItem *__restrict__ fb_list, uint8_t *__restrict__ fb_key, int32_t kcap,
    double2 *__restrict__ stash_n, double *__restrict__ stash_b, Counters *__restrict__ counters,
    const int32_t *__restrict__ cell_start)
{
    constexpr bool LIFE = MODE == kModeLife;
    constexpr bool kRegs = KMAX <= kLpRegRows;
    __shared__ double2 s_n[kRegs ? 1 : KMAX * kLpBlock];
    __shared__ double s_b[kRegs ? 1 : KMAX * kLpBlock];
    const int32_t s = xcd_tile(blockIdx.x, gridDim.x) * kLpBlock + threadIdx.x;
    LpRows<KMAX> rows;
    if constexpr (!kRegs) rows.L = Lane{s_n + threadIdx.x, s_b + threadIdx.x};
    bool need_fb = false;
    FallbackItem it{};
    // absent agents (spawning and removal) sit after every present one
    const int32_t n_present = LIFE ? cell_start[counters->total_cells - 1] : n;
    if (LIFE && s >= n_present && s < n) {
        // not in the simulation this step: status 2, zero velocity, no neighbours;
        // a step leaves its position and velocity as they are
        const int32_t id = sid[s];
        if (out.new_vel) {
            out.new_vel[id] = 0.f;
            out.new_vel[n + id] = 0.f;
        }
        if (out.status) out.status[id] = 2;
        if (out.nbr_out)
            for (int k = 0; k < out.krow; ++k) out.nbr_out[(int64_t)id * out.krow + k] = -1;
    }
    if (s < n_present) {
        const float4 me = sorted[s];
        const int32_t id = sid[s];
        const SceneDev p = sp[agent_scene[LIFE ? id : s]];  // as in k_knn
        need_fb = lp_agent<KMAX, MODE>(rows, it, EntriesInMemory{nbr, ld, s}, ncount[s], s, me,
                                       id, p, out, n, sorted, sid);
    }
    append_fallback<KMAX>(need_fb, it, rows, fb_list, fb_key, kcap, stash_n, stash_b, counters);
}

// Persistent velocity kernel: the neighbour search, half-planes and 2D LP of
// each agent in one pass, so its neighbour list never leaves registers (no
// list written and read back, one launch instead of two).  One-wave blocks
// take tiles of kLpBlock * APL agents in cell order (each lane APL agents, a
// wave apart) from queues of tiles, one queue per XCD over one contiguous
// eighth of the tiles: a block takes from the queue of its own XCD (blocks
// go to XCDs round robin), so neighbouring tiles share that XCD's L2, and
// when that queue is empty it takes from the others in turn.  A queue's
// counter is only ever incremented, and a block leaves once every queue is
// past its end, so every block exits.  Plain steps only (no recording, no
// spawning and removal); results equal those of k_knn + k_lp bit for bit.
template <int KMAX, int APL>
__global__ __launch_bounds__(kLpBlock)
__attribute__((amdgpu_waves_per_eu(KMAX <= kLpRegRows ? 3 : 1))) void k_velocity(
    const float4 *__restrict__ sorted, const int32_t *__restrict__ sid,
    const int32_t *__restrict__ inv, const int32_t *__restrict__ cell_start,
    const GridDev *__restrict__ grid, const int32_t *__restrict__ agent_scene,
    const SceneDev *__restrict__ sp, int32_t n, OutArgs out, FallbackItem *__restrict__ fb_list,
    uint8_t *__restrict__ fb_key, int32_t kcap, double2 *__restrict__ stash_n,
    double *__restrict__ stash_b, Counters *__restrict__ counters)
{
    constexpr bool kRegs = KMAX <= kLpRegRows;
    __shared__ double2 s_n[kRegs ? 1 : KMAX * kLpBlock];
    __shared__ double s_b[kRegs ? 1 : KMAX * kLpBlock];
    LpRows<KMAX> rows;
    if constexpr (!kRegs) rows.L = Lane{s_n + threadIdx.x, s_b + threadIdx.x};
    constexpr int32_t kTile = kLpBlock * APL;
    const int32_t n_tiles = (n + kTile - 1) / kTile;
    const int32_t q = n_tiles / kXcds, r = n_tiles % kXcds;
    const int32_t home = (int32_t)(blockIdx.x % kXcds);
    for (int32_t v = 0; v < kXcds; ++v) {
        const int32_t x = (home + v) % kXcds;
        const int32_t t0 = x * q + min(x, r);
        const int32_t len = q + (x < r ? 1 : 0);
        for (;;) {
            uint32_t t = 0;
            if (threadIdx.x == 0) t = atomicAdd(&counters->tiles[x], 1u);
            t = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)t);
            if (t >= (uint32_t)len) break;
            const int32_t base = (t0 + (int32_t)t) * kTile;
#pragma unroll 1
            for (int32_t a = 0; a < APL; ++a) {
                const int32_t s = base + a * kLpBlock + (int32_t)threadIdx.x;
                bool need_fb = false;
                FallbackItem it{};
                if (s < n) {
                    const float4 me = sorted[s];
                    const int32_t id = sid[s];
                    const int32_t sc = agent_scene[s];  // as in k_knn
                    const SceneDev p = sp[sc];
                    int32_t e[KMAX];
                    int m = 0;
                    {
                        uint64_t best[KMAX];
                        const int32_t pad = knn_search<KMAX>(best, me, id, grid[sc], p.k, p.nd2,
                                                             p.nd, sorted, sid, cell_start);
#pragma unroll
                        for (int k = 0; k < KMAX; ++k) {
                            e[k] = knn_entry<KMAX>(best, k, pad, id, inv);
                            m += e[k] != -1 ? 1 : 0;
                        }
                        // the K nearest sit in the last K slots: move them to
                        // the front (a shifter over static indices, by pad)
#pragma unroll
                        for (int b = 1; b < KMAX; b <<= 1) {
                            const bool sh = (pad & b) != 0;
#pragma unroll
                            for (int k = 0; k < KMAX; ++k)
                                e[k] = sh ? (k + b < KMAX ? e[k + b] : -1) : e[k];
                        }
                    }
                    need_fb = lp_agent<KMAX, kModePlain>(rows, it, EntriesInRegs<KMAX>{e}, m, s,
                                                         me, id, p, out, n, sorted, sid);
                }
                append_fallback<KMAX>(need_fb, it, rows, fb_list, fb_key, kcap, stash_n, stash_b,
                                      counters);
            }
        }
    }
}

// Counting sort of each chunk of kFbSortChunk fallback slots by the row at
// which their projection failed, so that a wave of k_fallback takes agents
// whose programs start at the same row and follow similar paths.  Order
// within a key is whatever the LDS atomics give; results do not depend on it.
// fb_total (profiling, nullable): the pass's fallback count is added to it.
__global__ __launch_bounds__(kFbSortBlock) void k_fb_sort(const uint8_t *__restrict__ key,
                                                          int32_t *__restrict__ order,
                                                          const Counters *__restrict__ counters,
                                                          unsigned long long *__restrict__ fb_total)
{
    constexpr int kPer = kFbSortChunk / kFbSortBlock;
    __shared__ uint32_t hist[64];
    const uint32_t count = counters->n_fallback;
    if (fb_total && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(fb_total, (unsigned long long)count);
    const uint32_t c0 = blockIdx.x * (uint32_t)kFbSortChunk;
    if (c0 >= count) return;  // uniform over the block
    const uint32_t c1 = min(c0 + (uint32_t)kFbSortChunk, count);
    if (threadIdx.x < 64) hist[threadIdx.x] = 0u;
    __syncthreads();
    uint32_t rk[kPer];
    uint32_t kv[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const uint32_t i = c0 + q * kFbSortBlock + threadIdx.x;
        kv[q] = 0u;
        rk[q] = 0u;
        if (i < c1) {
            kv[q] = key[i] & 63u;
            rk[q] = atomicAdd(&hist[kv[q]], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const uint32_t v = hist[threadIdx.x];
        uint32_t inc = v;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(inc, o, 64);
            if ((int)threadIdx.x >= o) inc += u;
        }
        hist[threadIdx.x] = inc - v;  // exclusive
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const uint32_t i = c0 + q * kFbSortBlock + threadIdx.x;
        if (i < c1) order[c0 + hist[kv[q]] + rk[q]] = (int32_t)i;
    }
}

// Rows of k_fallback: up to 16 in registers, read there with wave-uniform
// indices (every loop of the programs runs over fixed bounds) and from the
// agent's stash slot with a lane's own index; more in a per-lane LDS column.
template <int KMAX, bool IN_REGS = (KMAX <= kLpRegRows)>
struct FbRows;
template <int KMAX>
struct FbRows<KMAX, true> {
    // references to three local arrays of doubles of the kernel: arrays of
    // their own (not members of a struct, not double2) are kept in registers
    double (&nx)[KMAX];
    double (&ny)[KMAX];
    double (&b)[KMAX];
    const double2 *gn;  // the same rows in the stash slot
    const double *gb;
    __device__ __forceinline__ double2 N(int k) const { return make_double2(nx[k], ny[k]); }
    __device__ __forceinline__ double B(int k) const { return b[k]; }
    __device__ __forceinline__ double2 NL(int k) const { return gn[k]; }
    __device__ __forceinline__ double BL(int k) const { return gb[k]; }
    __device__ __forceinline__ void slot(const double2 *n_, const double *b_)
    {
        gn = n_;
        gb = b_;
    }
    __device__ __forceinline__ void set(int k, double2 nk, double bk)
    {
        nx[k] = nk.x;
        ny[k] = nk.y;
        b[k] = bk;
    }
};
template <int KMAX>
struct FbRows<KMAX, false> {
    Lane L;
    __device__ __forceinline__ double2 N(int k) const { return L.N(k); }
    __device__ __forceinline__ double B(int k) const { return L.B(k); }
    __device__ __forceinline__ double2 NL(int k) const { return L.N(k); }
    __device__ __forceinline__ double BL(int k) const { return L.B(k); }
    __device__ __forceinline__ void slot(const double2 *, const double *) {}
    __device__ __forceinline__ void set(int k, double2 nk, double bk)
    {
        L.n[k * kLpStride] = nk;
        L.b[k * kLpStride] = bk;
    }
};

// ------------------------------------------------------------------ work units
//
// Work units (section 3): the recompute of a new velocity is cut into pieces
// of equal size that lanes with nothing to recompute take over.  In the
// fallback the recompute that runs longest is the 1D program on a violated
// line of a plane subproblem: it visits every earlier row of the lane's own
// store, so a wave pays for its longest such program while the lanes that
// have none (or have finished their agent) wait.  With work units, the lanes
// whose line i is violated (at most kLpBlock / kWuGroup of them) publish the
// line in LDS; kWuGroup lanes per line each fold an equal, contiguous share
// of its i + 1 earlier rows (read from the owner's rows in LDS) into a
// partial interval; the group combines its partials in row order across
// lanes (the later partial's ends are offered to the earlier one, with the
// same strict tests as adding a row, so the earliest of equal bounds wins as
// in the one-lane program); the owner takes the result.  Lines with fewer
// than kWuFrom earlier rows, or steps where too many lanes recompute at once,
// run the one-lane program.  Each partial starts from the disc's interval,
// which is part of every line's program.

// Lanes of one wave hand values to each other through LDS: the wave's LDS
// accesses complete in issue order, so it takes only that neither the
// compiler moves an access across this point (a wavefront-scope fence, which
// emits no instruction) nor the lanes part (the wave barrier).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kWuGroup = 4;  // lanes per published line
constexpr int kWuFrom = 6;   // fewest earlier rows (i + 1) worth splitting
constexpr int kWuLines = kLpBlock / kWuGroup;

// LDS of one fallback wave (one-wave blocks): each lane's rows in stash
// order, and the lines of one step with their combined intervals.
template <int KB>
struct WuShared {
    double nx[KB][kLpBlock], ny[KB][kLpBlock], b[KB][kLpBlock];
    double line[kWuLines][8];  // mx, my, ci, mm, root, nk.x, nk.y, bk of the owner's line
    int32_t owner[kWuLines];
    double res[kWuLines][4];   // lo_n, lo_d, hi_n, hi_d
    int32_t rsrc[kWuLines][2];
};

__device__ __forceinline__ void shfl_xor_interval(const Interval &a, Interval &o, int d)
{
    o.lo_n = __shfl_xor(a.lo_n, d, 64);
    o.lo_d = __shfl_xor(a.lo_d, d, 64);
    o.hi_n = __shfl_xor(a.hi_n, d, 64);
    o.hi_d = __shfl_xor(a.hi_d, d, 64);
    o.lo_src = __shfl_xor(a.lo_src, d, 64);
    o.hi_src = __shfl_xor(a.hi_src, d, 64);
}

// lp2_plane for a whole wave with work units.  Every lane of the wave calls
// it (active: the lane has a plane k to solve; the others only help).
template <int KB, class RS>
__device__ __forceinline__ bool lp2_plane_wu(const RS &L, WuShared<KB> &W, bool active, int k,
                                             double2 nk, double bk, double vmax, double &vx,
                                             double &vy, Active *act)
{
    const int lane = (int)(threadIdx.x & 63);
    const double vm2 = vmax * vmax;
    vx = vmax * nk.x;
    vy = vmax * nk.y;
    act->line = kLineNone;
    act->src = kSrcDisc;
    bool ok = active;
#pragma unroll
    for (int i = -1; i < KB - 1; ++i) {
        // this lane's step i of the plane program: is line i violated, and
        // does its 1D program run?
        bool run = false;
        double mx = 0.0, my = 0.0, ci = 0.0, mm = 0.0, root = 0.0;
        if (ok && i < k) {
            plane_row(L, i, nk, bk, mx, my, ci);
            if (!(mx * vx + my * vy >= ci)) {
                mm = mx * mx + my * my;
                if (mm == 0.0) {
                    ok = !(ci > 0.0);
                } else {
                    const double disc = vm2 * mm - ci * ci;
                    if (disc < 0.0) {
                        ok = false;
                    } else {
                        root = sqrt(disc);
                        run = true;
                    }
                }
            }
        }
        const uint64_t mask = __ballot(run);
        if (mask == 0) continue;
        Interval iv;
        const int nrun = __popcll(mask);
        if (i + 1 >= kWuFrom && nrun <= kWuLines) {
            const int rank = (int)__builtin_amdgcn_mbcnt_hi(
                (uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
            if (run) {
                W.owner[rank] = lane;
                W.line[rank][0] = mx;
                W.line[rank][1] = my;
                W.line[rank][2] = ci;
                W.line[rank][3] = mm;
                W.line[rank][4] = root;
                W.line[rank][5] = nk.x;
                W.line[rank][6] = nk.y;
                W.line[rank][7] = bk;
            }
            // one wave per block: its LDS accesses complete in issue order
            wave_lds_sync();
            const int g = lane / kWuGroup, r = lane % kWuGroup;
            const int per = (i + 1 + kWuGroup - 1) / kWuGroup;  // rows per share
            Interval part;
            part.init(1.0, 1.0);
            if (g < nrun) {
                const int p = W.owner[g];
                const double pmx = W.line[g][0], pmy = W.line[g][1], pci = W.line[g][2];
                const double pmm = W.line[g][3];
                const double pkx = W.line[g][5], pky = W.line[g][6], pbk = W.line[g][7];
                part.init(W.line[g][4], pmm);
#pragma unroll
                for (int u = 0; u < per; ++u) {
                    const int j = -1 + r * per + u;
                    if (j < i) {
                        double ax, ay, cj;
                        if (j < 0) {
                            ax = -pkx;
                            ay = -pky;
                            cj = -pbk;
                        } else {
                            ax = W.nx[j][p] - pkx;
                            ay = W.ny[j][p] - pky;
                            cj = W.b[j][p] - pbk;
                        }
                        double den, num;
                        plane_term(ax, ay, cj, pmx, pmy, pci, pmm, den, num);
                        part.add(den, num, j);
                    }
                }
            }
            // combine the group's partials, earlier rows first
#pragma unroll
            for (int d = 1; d < kWuGroup; d <<= 1) {
                Interval o;
                shfl_xor_interval(part, o, d);
                if (lane & d) {
                    o.add(part.lo_d, part.lo_n, part.lo_src);
                    o.add(part.hi_d, part.hi_n, part.hi_src);
                    part = o;
                } else {
                    part.add(o.lo_d, o.lo_n, o.lo_src);
                    part.add(o.hi_d, o.hi_n, o.hi_src);
                }
            }
            if (g < nrun && r == 0) {
                W.res[g][0] = part.lo_n;
                W.res[g][1] = part.lo_d;
                W.res[g][2] = part.hi_n;
                W.res[g][3] = part.hi_d;
                W.rsrc[g][0] = part.lo_src;
                W.rsrc[g][1] = part.hi_src;
            }
            wave_lds_sync();
            if (run) {
                iv.lo_n = W.res[rank][0];
                iv.lo_d = W.res[rank][1];
                iv.hi_n = W.res[rank][2];
                iv.hi_d = W.res[rank][3];
                iv.lo_src = W.rsrc[rank][0];
                iv.hi_src = W.rsrc[rank][1];
            }
            // the next step's writes must not pass this step's reads
            wave_lds_sync();
        } else if (run) {
            iv.init(root, mm);
            for (int j = -1; j < i; ++j) {
                double ax, ay, cj;
                plane_row(L, j, nk, bk, ax, ay, cj);
                double den, num;
                plane_term(ax, ay, cj, mx, my, ci, mm, den, num);
                iv.add(den, num, j);
            }
        }
        if (run) {
            if (iv.empty()) {
                ok = false;
                continue;
            }
            plane_point(iv, nk, mx, my, ci, mm, vx, vy, act);
            act->line = i;
        }
    }
    return ok;
}

// lp3_least_penetration with every lane staying in the pass loop while any
// lane still has a plane to take, so the lanes that are done help the others
// (lp2_plane_wu).  The same passes, planes and arithmetic otherwise.
template <int KB, class RS>
__device__ __forceinline__ double lp3_least_penetration_wu(const RS &L, WuShared<KB> &W, int m,
                                                           int start, double vmax, double &vx,
                                                           double &vy, int *plane, Active *act)
{
    double t = 0.0;
    *plane = -1;
    act->line = kLineNone;
    act->src = kSrcDisc;
    uint32_t left = rows_below(m) & ~rows_below(start);
#pragma unroll 1
    for (int pass = 0; pass < KB; ++pass) {
        int k = KB;
        for (int u = KB - 1; u >= 0; --u) {
            const double2 nu = L.N(u);
            const bool hit = ((left >> u) & 1u) != 0u && !(nu.x * vx + nu.y * vy + t >= L.B(u));
            k = hit ? u : k;
        }
        const bool active = k < KB;
        if (__ballot(active) == 0) break;
        if (active) left &= ~rows_below(k + 1);
        const int kk = active ? k : 0;
        const double2 nk = L.NL(kk);
        const double bk = L.BL(kk);
        double wx, wy;
        Active pa;
        const bool okp = lp2_plane_wu<KB>(L, W, active, k, nk, bk, vmax, wx, wy, &pa);
        if (active && okp) {
            vx = wx;
            vy = wy;
            t = fmax(bk - (nk.x * vx + nk.y * vy), 0.0);
            *plane = k;
            *act = pa;
        }
    }
    return t;
}

template <int KB>
struct Lp3WorkUnits {
    WuShared<KB> *W;
    template <int KB2, class RS>
    __device__ __forceinline__ double run(const RS &L, int m, int start, double vmax, double &vx,
                                          double &vy, int *plane, Active *act) const
    {
        return lp3_least_penetration_wu<KB2>(L, *W, m, start, vmax, vx, vy, plane, act);
    }
};

// The persistent loop of k_fallback over its share of the sorted list.  With
// work units (WU) the loop runs in whole-wave rounds (a lane past the end of
// the list has no agent but stays to help) and each lane's rows also go to
// LDS for its helpers.
template <int KMAX, int MODE, bool WU, class RS>
__device__ __forceinline__ void fallback_items(RS &rows, WuShared<KMAX> *W, const OutArgs &out,
                                               int32_t n, int32_t kcap,
                                               const FallbackItem *__restrict__ fb_list,
                                               const int32_t *__restrict__ fb_order,
                                               const double2 *__restrict__ stash_n,
                                               const double *__restrict__ stash_b, uint32_t count)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t stride = gridDim.x * kLpBlock;
    for (uint32_t base = blockIdx.x * kLpBlock; WU ? base < count : base + lane < count;
         base += stride) {
        const uint32_t q = base + lane;
        const bool have = q < count;
        const int32_t slot = have ? fb_order[q] : 0;
        FallbackItem it{};
        if (have) it = fb_list[slot];
        const int m = have ? it.m : 0, fail = have ? it.fail : 0;
        const double2 *gn = stash_n + (int64_t)slot * kcap;
        const double *gb = stash_b + (int64_t)slot * kcap;
        rows.slot(gn, gb);
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            if (k < m) rows.set(k, gn[k], gb[k]);
            else rows.set(k, make_double2(0.0, 0.0), 0.0);
        }
        double vx = it.vx, vy = it.vy;
        int plane = -1;
        Active dact, ract;
        bool ok;
        double d;
        if constexpr (WU) {
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                const double2 nk = rows.N(k);
                W->nx[k][lane] = nk.x;
                W->ny[k][lane] = nk.y;
                W->b[k][lane] = rows.B(k);
            }
            wave_lds_sync();
            d = fallback_velocity<KMAX>(rows, m, fail, (double)it.vmax, it.vhx, it.vhy, vx, vy,
                                        &plane, &dact, &ract, &ok, Lp3WorkUnits<KMAX>{W});
            wave_lds_sync();
        } else {
            d = fallback_velocity<KMAX>(rows, m, fail, (double)it.vmax, it.vhx, it.vhy, vx, vy,
                                        &plane, &dact, &ract, &ok);
        }
        if (!have) continue;
        if (MODE == kModeRec) {
            TapeCode tc{};
            tc.status = 1;
            tc.p_line = (int8_t)stash_row(ract.line, it);
            tc.p_src = (int8_t)stash_row(ract.src, it);
            tc.d_plane = (int8_t)stash_row(plane, it);
            tc.d_line = (int8_t)stash_row(dact.line, it);
            tc.d_src = (int8_t)stash_row(dact.src, it);
            tc.relaxed_empty = ok ? 0 : 1;
            tc.dstar = d;
            out.tape_codes[it.s] = tc;
        }
        write_result<MODE == kModeLife>(out, it.mex, it.mey, it.dt, it.id, it.s, n, vx, vy,
                                        it.vhx, it.vhy, 1);
    }
}

// Persistent over the fallback list in sorted order.  The rows come in stash
// order (stash_position): d* from the projection's last optimum (the rows
// before the failed one hold there with t = 0), then the point closest to
// vhat among those within d* + delta of every half-plane, with the rows that
// fix d* taken first: the relaxed projection's optimum lies where they cross,
// so the other rows are rarely violated.  WU: the least-penetration program
// with work units (rows in registers only, K <= 16).
template <int KMAX, int MODE, bool WU>
__global__ __launch_bounds__(kLpBlock) void k_fallback(OutArgs out, int32_t n, int32_t kcap,
                                                       const FallbackItem *__restrict__ fb_list,
                                                       const int32_t *__restrict__ fb_order,
                                                       const double2 *__restrict__ stash_n,
                                                       const double *__restrict__ stash_b,
                                                       const Counters *__restrict__ counters)
{
    constexpr bool kRegs = KMAX <= kLpRegRows;
    static_assert(!WU || kRegs, "work units serve the register-row fallback");
    __shared__ double2 s_n[kRegs ? 1 : KMAX * kLpBlock];
    __shared__ double s_b[kRegs ? 1 : KMAX * kLpBlock];
    __shared__ WuShared<WU ? KMAX : 1> s_wu;
    const uint32_t count = counters->n_fallback;
    double rnx[kRegs ? KMAX : 1], rny[kRegs ? KMAX : 1], rb[kRegs ? KMAX : 1];
    if constexpr (kRegs) {
        FbRows<KMAX> rows{rnx, rny, rb, nullptr, nullptr};
        fallback_items<KMAX, MODE, WU>(rows, (WuShared<KMAX> *)&s_wu, out, n, kcap, fb_list,
                                       fb_order, stash_n, stash_b, count);
    } else {
        FbRows<KMAX> rows{Lane{s_n + threadIdx.x, s_b + threadIdx.x}};
        fallback_items<KMAX, MODE, false>(rows, (WuShared<KMAX> *)nullptr, out, n, kcap, fb_list,
                                          fb_order, stash_n, stash_b, count);
    }
}

// Number of removed agents (state 1) into counters->removed: one block.
__global__ __launch_bounds__(256) void k_count_removed(const uint8_t *__restrict__ state,
                                                       int32_t n, Counters *__restrict__ counters)
{
    __shared__ uint32_t red[4];
    uint32_t c = 0;
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) c += state[i] == 1 ? 1u : 0u;
    c = wave_reduce_sum_u32(c);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) counters->removed = red[0] + red[1] + red[2] + red[3];
}

// ------------------------------------------------------------------ launchers

// Recording (for the adjoint) and spawning / removal are separate
// instantiations: the plain one carries none of their bookkeeping.
inline int plan_mode(const Plan &pl)
{
    return pl.out.tape_codes ? kModeRec : (pl.out.life.spawn_step ? kModeLife : kModePlain);
}

// The fused velocity kernel serves plain passes when it is selected.
inline bool plan_fused(const Plan &pl) { return pl.vel_apl > 0 && plan_mode(pl) == kModePlain; }

template <int KMAX>
hipError_t launch_knn_k(const Plan &pl, hipStream_t st)
{
    if (plan_fused(pl)) return hipSuccess;  // k_velocity searches the neighbours itself
    const int32_t n = pl.n;
    const int32_t bs = pl.knn_block;
    hipLaunchKernelGGL(k_knn<KMAX>, dim3((n + bs - 1) / bs), dim3(bs), 0, st, pl.sorted, pl.sid,
                       pl.inv, pl.cell_start, pl.grid, pl.agent_scene, pl.sp, n, pl.nbr, pl.ld,
                       pl.ncount, pl.counters, pl.out.life.spawn_step ? 1 : 0);
    return hipGetLastError();
}

template <int KMAX, int MODE>
hipError_t launch_lp_mode(const Plan &pl, hipStream_t st)
{
    const int32_t n = pl.n;
    const int32_t gl = (n + kLpBlock - 1) / kLpBlock;
    hipLaunchKernelGGL((k_lp<KMAX, MODE>), dim3(gl), dim3(kLpBlock), 0, st, pl.sorted, pl.sid,
                       pl.agent_scene, pl.sp, n, pl.nbr, pl.ld, pl.ncount, pl.out, pl.fb_list,
                       pl.fb_key, pl.kcap, pl.stash_n, pl.stash_b, pl.counters, pl.cell_start);
    return hipGetLastError();
}

template <int KMAX, int MODE>
hipError_t launch_fallback_mode(const Plan &pl, hipStream_t st)
{
    // persistent: fb_waves_per_cu one-wave blocks per CU loop over the device-side list
    const int32_t gs = (pl.n + kFbSortChunk - 1) / kFbSortChunk;
    hipLaunchKernelGGL(k_fb_sort, dim3(gs), dim3(kFbSortBlock), 0, st, pl.fb_key, pl.fb_order,
                       pl.counters, pl.fb_total);
    const int32_t gf = max(1, min((pl.n + kLpBlock - 1) / kLpBlock, pl.fb_waves_per_cu * pl.cus));
    if (pl.fb_work_units && KMAX <= kLpRegRows)
        hipLaunchKernelGGL((k_fallback<KMAX, MODE, KMAX <= kLpRegRows>), dim3(gf), dim3(kLpBlock),
                           0, st, pl.out, pl.n, pl.kcap, pl.fb_list, pl.fb_order, pl.stash_n,
                           pl.stash_b, pl.counters);
    else
        hipLaunchKernelGGL((k_fallback<KMAX, MODE, false>), dim3(gf), dim3(kLpBlock), 0, st,
                           pl.out, pl.n, pl.kcap, pl.fb_list, pl.fb_order, pl.stash_n, pl.stash_b,
                           pl.counters);
    return hipGetLastError();
}

template <int KMAX, int APL>
hipError_t launch_velocity_apl(const Plan &pl, hipStream_t st)
{
    // persistent: vel_waves_per_cu one-wave blocks per CU, a multiple of the
    // XCD count so every XCD's queue has its share of blocks
    constexpr int32_t kTile = kLpBlock * APL;
    const int32_t tiles = (pl.n + kTile - 1) / kTile;
    int32_t g = min(pl.vel_waves_per_cu * pl.cus, tiles);
    g = max(kXcds, (g + kXcds - 1) / kXcds * kXcds);
    hipLaunchKernelGGL((k_velocity<KMAX, APL>), dim3(g), dim3(kLpBlock), 0, st, pl.sorted, pl.sid,
                       pl.inv, pl.cell_start, pl.grid, pl.agent_scene, pl.sp, pl.n, pl.out,
                       pl.fb_list, pl.fb_key, pl.kcap, pl.stash_n, pl.stash_b, pl.counters);
    return hipGetLastError();
}

template <int KMAX>
hipError_t launch_lp_k(const Plan &pl, hipStream_t st)
{
    if (plan_fused(pl)) {
        switch (pl.vel_apl) {
        case 1: return launch_velocity_apl<KMAX, 1>(pl, st);
        case 2: return launch_velocity_apl<KMAX, 2>(pl, st);
        default: return launch_velocity_apl<KMAX, 4>(pl, st);
        }
    }
    switch (plan_mode(pl)) {
    case kModeRec: return launch_lp_mode<KMAX, kModeRec>(pl, st);
    case kModeLife: return launch_lp_mode<KMAX, kModeLife>(pl, st);
    default: return launch_lp_mode<KMAX, kModePlain>(pl, st);
    }
}

template <int KMAX>
hipError_t launch_fallback_k(const Plan &pl, hipStream_t st)
{
    switch (plan_mode(pl)) {
    case kModeRec: return launch_fallback_mode<KMAX, kModeRec>(pl, st);
    case kModeLife: return launch_fallback_mode<KMAX, kModeLife>(pl, st);
    default: return launch_fallback_mode<KMAX, kModePlain>(pl, st);
    }
}

// The neighbour-list length picks the register / LDS footprint.
#define ORCA_DISPATCH_K(fn)                                  \
    if (pl.n == 0) return hipSuccess;                        \
    if (kmax <= 10) return fn<10>(pl, st);                   \
    if (kmax <= 16) return fn<16>(pl, st);                   \
    return fn<32>(pl, st);

hipError_t launch_knn(const Plan &pl, int kmax, hipStream_t st) { ORCA_DISPATCH_K(launch_knn_k) }
hipError_t launch_lp(const Plan &pl, int kmax, hipStream_t st) { ORCA_DISPATCH_K(launch_lp_k) }
hipError_t launch_fallback(const Plan &pl, int kmax, hipStream_t st)
{
    ORCA_DISPATCH_K(launch_fallback_k)
}

hipError_t launch_scene_map(const int32_t *off, int32_t n_scenes, int32_t *agent_scene, int32_t n,
                            uint32_t *bbox, hipStream_t st)
{
    if (n > 0)
        hipLaunchKernelGGL(k_scene_of_agent, dim3((n + 255) / 256), dim3(256), 0, st, off,
                           n_scenes, agent_scene, n);
    hipLaunchKernelGGL(k_reset_bbox, dim3((n_scenes + 255) / 256), dim3(256), 0, st, bbox,
                       n_scenes);
    return hipGetLastError();
}

hipError_t launch_grid(const Plan &pl, const float *pos, const float *vel, bool advance,
                       hipStream_t st)
{
    const int32_t n = pl.n;
    const LifeArgs &life = pl.out.life;
    if (n > 0)
        hipLaunchKernelGGL(k_bbox, dim3(pl.n_chunks), dim3(kBboxBlock), 0, st, pos, n, pl.res_src,
                           pl.chunks, pl.off, pl.bbox);
    hipLaunchKernelGGL(k_grid, dim3(1), dim3(256), 0, st, pl.n_scenes, pl.off, pl.sp, pl.bbox,
                       pl.grid, pl.counters, pl.max_cells, life.spawn_step ? 1 : 0);
    if (n > 0)
        hipLaunchKernelGGL(k_key, dim3((n + 255) / 256), dim3(256), 0, st, pos, n, pl.res_src,
                           pl.agent_scene, pl.grid, pl.key, pl.rank, pl.counts, life.spawn_step,
                           life.state, pl.counters);
    // the scan covers the scenes' cells and the cell of absent agents
    const int32_t tiles = (int32_t)((pl.max_cells + 1 + kScanTile - 1) / kScanTile);
    hipLaunchKernelGGL(k_scan_sums, dim3(tiles), dim3(kScanBlock), 0, st, pl.counts, pl.counters,
                       pl.partial);
    hipLaunchKernelGGL(k_scan_apply, dim3(tiles), dim3(kScanBlock), 0, st, pl.counts,
                       pl.counters, pl.partial, pl.cell_start, n,
                       advance && life.spawn_step ? 1 : 0);
    if (n == 0) return hipGetLastError();
    hipLaunchKernelGGL(k_scatter, dim3((n + 255) / 256), dim3(256), 0, st, pos, vel, n,
                       pl.res_src, pl.sid_prev, pl.sg_prev, pl.sg_src, pl.sg_cur, pl.key, pl.rank,
                       pl.cell_start, pl.sorted, pl.sid, pl.inv, pl.out.ag.radius, pl.out.ag.srad);
    return hipGetLastError();
}

hipError_t launch_count_removed(const uint8_t *state, int32_t n, Counters *counters,
                                hipStream_t st)
{
    hipLaunchKernelGGL(k_count_removed, dim3(1), dim3(256), 0, st, state, n, counters);
    return hipGetLastError();
}

hipError_t launch_fill_vel(const Plan &pl, const float *vel, hipStream_t st)
{
    if (pl.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_vel, dim3((pl.n + 255) / 256), dim3(256), 0, st, vel, pl.n, pl.inv,
                       pl.sorted, pl.counters);
    return hipGetLastError();
}

}  // namespace orca
