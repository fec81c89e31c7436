// orca_internal.h -- types shared by the kernels and the host side of liborca.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "orca_adjoint.h"

namespace orca {

constexpr int kScanItems = 4;                       // cells per thread of a scan block
constexpr int kScanBlock = 1024;                    // 1024 threads: more loads in flight than 256
constexpr int kScanTile = kScanItems * kScanBlock;  // cells per scan tile
constexpr int kLpBlock = 64;                        // one wave per LP block
constexpr int kBboxChunk = 8192;                    // agents per bounding-box block
constexpr int kBboxBlock = 1024;                    // threads per bounding-box block
constexpr double kCellMargin = 1.0 + 1.0 / 1024.0;  // cell side / (neighbor_dist / cells per nd)
constexpr int kMinCellsPerNd = 2;                   // grid cells across one neighbor_dist: 2 ..
constexpr int kMaxCellsPerNd = 4;                   // .. 4, per scene (k_grid)
constexpr int kFbSortChunk = 4096;                  // fallback slots sorted together
constexpr int kFbSortBlock = 1024;                  // threads per fallback-sort block (4 slots each)

// Tile of block b of nb.  Workgroups are handed to the 8 XCDs round robin
// (block b to XCD b mod 8), and each XCD has its own L2; this mapping gives
// each XCD one contiguous range of tiles, so agents that share neighbours (cell
// order) meet in the same L2.  A bijection of [0, nb) for any nb.
constexpr int32_t kXcds = 8;
__device__ __forceinline__ int32_t xcd_tile(int32_t b, int32_t nb)
{
    const int32_t q = nb / kXcds, r = nb % kXcds, x = b % kXcds, i = b / kXcds;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Per-scene parameters as the kernels read them.
struct SceneDev {
    float radius, vmax, nd, tau, dt, pref_speed;
    float nd2;  // float32 neighbor_dist^2 (the same rounding as every distance test)
    int32_t k;
};

// Per-scene grid: cell c = (cx, cy) has key base + cy * nx + cx.
struct GridDev {
    double x0, y0, cell;
    int32_t nx, ny, base, pad;
};

// Device-side counters of the context.  total_cells counts the grid cells of
// every scene plus, with spawning and removal on, one last cell that holds the
// absent agents (so cell_start of that cell is the number of present agents).
// step is the step index the next binning evaluates presence at; removed is
// written on request (the agents whose state is 1).  tiles are the per-XCD
// tile queues of the fused velocity kernel (cleared before every pass).
struct Counters {
    uint32_t total_cells;
    uint32_t n_fallback;
    int32_t step;
    uint32_t removed;
    uint32_t tiles[8];
};

// FallbackItem (the record of an agent whose projection was empty) and the
// stash order of its rows (stash_position / stash_row) are in orca_lp.h.

// Optional per-agent properties, indexed by agent (nullptr: the scene's
// value).  srad holds the radii in cell order when radius is given.
struct AgentProps {
    const float *radius;
    const float *max_speed;
    const float *pref_speed;
    float *srad;
};

// Spawning and removal (caller's device arrays): agent i takes part in the
// step at index t when spawn_step[i] <= t and state[i] == 0; a step that ends
// with the agent's goal within its own radius sets state[i] = 1.
struct LifeArgs {
    const int32_t *spawn_step;  // [N] or nullptr (off)
    uint8_t *state;             // [N]
    const SceneDev *sp;         // scene radius, when no per-agent radius is given
    const int32_t *agent_scene;
    Counters *counters;
};

// Where the velocity kernels put their results.  Step mode has pos != nullptr.
struct OutArgs {
    float *new_vel;      // [2, N] or nullptr
    float *pos;          // [2, N] updated in place (step mode) or nullptr
    float *vel;          // [2, N] (step mode)
    float *pref;         // [2, N]: read when goals == nullptr, written in step mode with goals
    const float *goals;  // [2, N] or nullptr
    uint8_t *status;     // [N] or nullptr
    int32_t *nbr_out;    // [N, krow] or nullptr
    int32_t krow;
    float4 *tape_state;  // recorded step: state (x, y, vx, vy) at the step's start by sorted
                         // index, or nullptr
    TapeCode *tape_codes;  // recorded step: how each velocity was chosen, by sorted index
    AgentProps ag;         // per-agent properties of this pass
    LifeArgs life;         // spawning and removal (life.spawn_step == nullptr: off)
    // Resident steps (the inner steps of a multi-step call): the new state
    // goes to nxt by sorted index instead of the caller's arrays, and the
    // goal (goals given) or preferred velocity is read from sg by sorted index.
    float4 *nxt;           // [ld] (x', y', vx', vy') or nullptr
    const float2 *sg;      // [ld] or nullptr
};

// Device buffers and sizes of one launch sequence.
struct Plan {
    int32_t n, n_scenes, ld, cus, n_chunks;
    int32_t knn_block;        // threads per k_knn block (64..512)
    int32_t fb_waves_per_cu;  // persistent k_fallback waves per CU
    int32_t vel_apl;          // 0: k_knn + k_lp; 1, 2, 4: the fused k_velocity, agents per lane
    int32_t vel_waves_per_cu; // persistent k_velocity waves per CU
    int32_t fb_work_units;    // 1: k_fallback with work units (K <= 16)
    uint32_t max_cells;
    const int32_t *off;
    const SceneDev *sp;
    int32_t *agent_scene;
    uint32_t *bbox;
    const int2 *chunks;  // (scene, first agent) of each bounding-box block
    GridDev *grid;
    Counters *counters;
    int32_t *key, *rank, *counts, *cell_start;
    uint32_t *partial;
    float4 *sorted;
    int32_t *sid, *inv;
    int32_t *nbr, *ncount;
    int32_t kcap;      // rows per stash slot (the context's k_max)
    FallbackItem *fb_list;
    uint8_t *fb_key;   // [ld] failed row of each fallback slot (the sort key)
    int32_t *fb_order; // [ld] fallback slots, sorted by fb_key within chunks of kFbSortChunk
    double2 *stash_n;  // [ld, kcap] half-plane normals of fallback slots, one slot contiguous
    double *stash_b;   // [ld, kcap] half-plane offsets
    // Binning of a resident step reads the state the previous step left in
    // cell order (res_src by that step's sorted index, ids in sid_prev, goals
    // or preferred velocities in sg_prev) instead of the caller's arrays;
    // otherwise sg_src (the caller's goals or preferred velocities, [2, N]),
    // when given, is copied into cell order.  The copy goes to sg_cur.
    const float4 *res_src;
    const int32_t *sid_prev;
    const float2 *sg_prev;
    const float *sg_src;
    float2 *sg_cur;
    unsigned long long *fb_total;  // profiling: the pass's fallback count is added here
    OutArgs out;
};

hipError_t launch_scene_map(const int32_t *off, int32_t n_scenes, int32_t *agent_scene, int32_t n,
                            uint32_t *bbox, hipStream_t st);
// advance: move the step counter on (a step with spawning and removal)
hipError_t launch_grid(const Plan &pl, const float *pos, const float *vel, bool advance,
                       hipStream_t st);
// also clears the fallback count and the tile queues for the velocity pass
hipError_t launch_fill_vel(const Plan &pl, const float *vel, hipStream_t st);
hipError_t launch_count_removed(const uint8_t *state, int32_t n, Counters *counters,
                                hipStream_t st);
hipError_t launch_knn(const Plan &pl, int kmax, hipStream_t st);
hipError_t launch_lp(const Plan &pl, int kmax, hipStream_t st);
hipError_t launch_fallback(const Plan &pl, int kmax, hipStream_t st);

// Adjoint of one recorded step (orca_adjoint.hip).
// The tape of a step is in that step's cell order (sorted index s).
struct BackArgs {
    int32_t n, n_scenes, ld;
    const int32_t *agent_scene;
    const SceneDev *sp;
    const float4 *state;      // tape: state at the step's start [s]
    const int32_t *nbr;       // tape: neighbour lists [k * ld + s] as k_knn wrote them
    const TapeCode *codes;    // tape: choices [s]
    const int32_t *sid;       // tape: agent id of each sorted index [s]
    const float *pref;        // fixed preferred velocities [2, n]
    const float *g_pos_next, *g_vel_next;
    float *g_pos, *g_vel, *g_pref, *g_max_speed, *g_time_horizon;
    const float *radius;      // per-agent radii of the recorded step, or nullptr
    const float *max_speed;   // per-agent max speeds of the recorded step, or nullptr
    double *acc;              // [4, n] float64 accumulators by sorted index (kept zero)
    double *own;              // [4, n] each agent's own share by sorted index
    // several steps in a row (orca_backward_steps): the gradients between
    // steps as one float4 (dL/dx, dL/dv) per agent id, the preferred
    // velocities and their gradient as float2 per agent id (one line per
    // agent instead of one per component); nullptr: the [2, n] arrays above
    const float4 *g_in4;      // dL/dx', dL/dv_next by id
    float4 *g_out4;           // dL/dx, dL/dv by id (may be g_in4: read then written per id)
    const float2 *pref2;
    float2 *g_pref2;          // accumulated
    double *acc_scene;        // [2, n_scenes]
};
hipError_t launch_backward(const BackArgs &a, hipStream_t st);
// pref [2, n] -> pref2, g_pref2 cleared (before a run of steps); g_pref [2, n] += g_pref2 (after)
hipError_t launch_backward_prep(const float *pref, float2 *pref2, float2 *g_pref2, int32_t n,
                                hipStream_t st);
hipError_t launch_backward_post(const float2 *g_pref2, float *g_pref, int32_t n, hipStream_t st);

}  // namespace orca
