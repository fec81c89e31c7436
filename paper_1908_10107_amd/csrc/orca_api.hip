// orca_api.hip -- host side of the C ABI declared in include/orca.h.
//
// Validation happens on the host before anything is enqueued, so bad
// arguments never reach a kernel.  All device memory is allocated in
// orca_create; the per-step calls only enqueue kernels on the context stream.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <algorithm>
#include <vector>

#include "orca.h"
#include "orca_internal.h"

using orca::Counters;
using orca::GridDev;
using orca::SceneDev;

struct orca_ctx {
    int64_t max_agents = 0;
    int32_t max_scenes = 0, k_max = 0, tape_steps = 0;
    hipStream_t stream = nullptr;
    uint32_t max_cells = 0;
    int32_t n_tiles = 0, cus = 0;

    // device scratch
    int32_t *off = nullptr;
    SceneDev *sp = nullptr;
    int32_t *agent_scene = nullptr;
    uint32_t *bbox = nullptr;
    int2 *chunks = nullptr;
    int64_t max_chunks = 0;
    GridDev *grid = nullptr;
    Counters *counters = nullptr;
    int32_t *key = nullptr, *rank = nullptr, *counts = nullptr, *cell_start = nullptr;
    uint32_t *partial = nullptr;
    float4 *sorted = nullptr;
    int32_t *sid = nullptr, *inv = nullptr;
    int32_t *nbr = nullptr, *ncount = nullptr;
    orca::FallbackItem *fb_list = nullptr;
    uint8_t *fb_key = nullptr;
    int32_t *fb_order = nullptr;
    double2 *stash_n = nullptr;
    double *stash_b = nullptr;
    float *srad = nullptr;  // per-agent radii in cell order
    // resident steps (the inner steps of one orca_step call): the state in
    // cell order, a second id buffer and two buffers of goals or preferred
    // velocities in cell order (each step reads one, writes the other)
    float4 *nxt = nullptr;
    int32_t *sid2 = nullptr;
    float2 *sg[2] = {nullptr, nullptr};
    std::vector<void *> allocs;

    // optional per-agent properties (caller's device arrays), see orca_set_agents
    const float *a_radius = nullptr, *a_vmax = nullptr, *a_speed = nullptr;

    // spawning and removal (caller's device arrays), see orca_set_lifecycle
    const int32_t *l_spawn = nullptr;
    uint8_t *l_state = nullptr;
    int32_t h_life = 0;          // staging of the step index for the counter upload
    bool life_binned = false;    // a binning with spawning and removal has been enqueued

    // scene set currently on the device
    int32_t n_scenes = 0;
    int64_t n = 0;
    int32_t kmax_cur = 0;
    std::vector<int64_t> h_off;
    std::vector<orca_params> h_par;
    std::vector<int32_t> h_off32;
    std::vector<SceneDev> h_sp;
    std::vector<int2> h_chunks;
    bool uploaded = false;

    // grid state
    bool grid_valid = false;
    const float *grid_pos = nullptr;
    const float *grid_radius = nullptr;  // per-agent radii the grid's sorted copy came from

    // per-stage timing (diagnostics): events on the context stream between stages
    bool profiling = false;
    // mode 2: events of every pass recorded without waiting (read at the end);
    // the fallback agents of those passes are summed on the device
    int32_t prof_mode = 0;
    std::vector<hipEvent_t> pev;
    unsigned long long *fb_total = nullptr;
    hipEvent_t ev[ORCA_PROF_STAGES + 1] = {};
    double stage_ms[ORCA_PROF_STAGES] = {0};
    int64_t prof_steps = 0, prof_fallback = 0;

    // tape of recorded steps for orca_backward
    // each recorded step in its own cell order (sorted index s): the state,
    // the neighbour lists as the neighbour kernel wrote them ([k_max, A]) and
    // the id of each s (the counting sort writes these two in place)
    float4 *tape_state = nullptr;           // [tape_steps, A]
    int32_t *tape_nbr = nullptr;            // [tape_steps, k_max, A]
    orca::TapeCode *tape_codes = nullptr;   // [tape_steps, A]
    int32_t *tape_sid = nullptr;            // [tape_steps, A]
    double *acc = nullptr;                  // [4, A]
    double *own = nullptr;                  // [4, A]
    float4 *g4 = nullptr;                   // [A] gradients between steps (orca_backward_steps)
    float2 *pref2 = nullptr, *g_pref2 = nullptr;  // [A] each
    double *acc_scene = nullptr;            // [2, S]
    int32_t tape_len = 0;                   // steps held by the last recording
    uint64_t tape_scene_version = 0;
    const float *tape_pref = nullptr;
    const float *tape_radius = nullptr, *tape_vmax = nullptr;

    // launch shapes (orca_autotune picks them)
    int32_t knn_block = 256, fb_waves_per_cu = 16;
    int32_t vel_apl = 0, vel_waves_per_cu = 12;  // velocity kernels (orca_set_kernels)
    int32_t fb_work_units = 0;                   // fallback with work units (orca_set_kernels)

    // step graphs replayed by orca_step_graph: one step, and a block of
    // kGraphBlock resident steps (plain steps only)
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t gblock = nullptr;
    hipGraphExec_t gblock_exec = nullptr;
    const void *graph_key[9] = {};
    uint64_t graph_scene_version = 0, scene_version = 0;
    int32_t graph_knn_block = 0, graph_fb = 0, graph_apl = -1, graph_vw = 0, graph_wu = -1;

    char err[512] = {0};
};

namespace {

int fail(orca_ctx *c, int code, const char *fmt, ...)
{
    if (c) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(c->err, sizeof(c->err), fmt, ap);
        va_end(ap);
    }
    return code;
}

int hip_fail(orca_ctx *c, hipError_t e, const char *where)
{
    return fail(c, ORCA_EHIP, "%s: %s", where, hipGetErrorString(e));
}

#define HIP_OK(call)                                             \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #call);   \
    } while (0)

bool finite_pos(float v) { return isfinite(v) && v > 0.0f; }
bool finite_nonneg(float v) { return isfinite(v) && v >= 0.0f; }

// Host-only checks of a scene set; no HIP call.
int check_scenes(orca_ctx *ctx, int32_t n_scenes, const int64_t *off, const orca_params *par)
{
    if (n_scenes < 1) return fail(ctx, ORCA_EINVAL, "n_scenes must be >= 1 (got %d)", n_scenes);
    if (n_scenes > ctx->max_scenes)
        return fail(ctx, ORCA_ECAPACITY, "n_scenes %d exceeds the context's %d", n_scenes,
                    ctx->max_scenes);
    if (!off || !par) return fail(ctx, ORCA_EINVAL, "scene_offsets and params must be non-NULL");
    if (off[0] != 0) return fail(ctx, ORCA_EINVAL, "scene_offsets[0] must be 0");
    for (int32_t s = 0; s < n_scenes; ++s)
        if (off[s + 1] < off[s])
            return fail(ctx, ORCA_EINVAL, "scene_offsets must be non-decreasing (scene %d)", s);
    if (off[n_scenes] > ctx->max_agents)
        return fail(ctx, ORCA_ECAPACITY, "%lld agents exceed the context's %lld",
                    (long long)off[n_scenes], (long long)ctx->max_agents);
    for (int32_t s = 0; s < n_scenes; ++s) {
        const orca_params &p = par[s];
        if (!finite_nonneg(p.radius) || !finite_pos(p.max_speed) ||
            !finite_pos(p.neighbor_dist) || !finite_pos(p.time_horizon) || !finite_pos(p.dt) ||
            !finite_nonneg(p.pref_speed) || p.reserved != 0)
            return fail(ctx, ORCA_EINVAL,
                        "scene %d: radius, pref_speed must be finite and >= 0; max_speed, "
                        "neighbor_dist, time_horizon, dt finite and > 0; reserved 0", s);
        if (p.max_neighbors < 0)
            return fail(ctx, ORCA_EINVAL, "scene %d: max_neighbors must be >= 0", s);
        if (p.max_neighbors > ctx->k_max)
            return fail(ctx, ORCA_ECAPACITY, "scene %d: max_neighbors %d exceeds k_max %d", s,
                        p.max_neighbors, ctx->k_max);
    }
    return ORCA_OK;
}

bool same_scenes(const orca_ctx *ctx, int32_t n_scenes, const int64_t *off, const orca_params *par)
{
    if (!ctx->uploaded || ctx->n_scenes != n_scenes) return false;
    if (memcmp(ctx->h_off.data(), off, sizeof(int64_t) * (size_t)(n_scenes + 1)) != 0) return false;
    return memcmp(ctx->h_par.data(), par, sizeof(orca_params) * (size_t)n_scenes) == 0;
}

// Validate and, if the scene set changed, upload it and rebuild the agent->scene map.
int use_scenes(orca_ctx *ctx, int32_t n_scenes, const int64_t *off, const orca_params *par)
{
    int rc = check_scenes(ctx, n_scenes, off, par);
    if (rc != ORCA_OK) return rc;
    if (same_scenes(ctx, n_scenes, off, par)) return ORCA_OK;
    // the staging vectors may still feed an earlier copy: let the stream drain first
    if (ctx->uploaded) HIP_OK(hipStreamSynchronize(ctx->stream));
    ctx->n_scenes = n_scenes;
    ctx->n = off[n_scenes];
    ctx->h_off.assign(off, off + n_scenes + 1);
    ctx->h_par.assign(par, par + n_scenes);
    ctx->h_off32.resize((size_t)n_scenes + 1);
    ctx->h_sp.resize((size_t)n_scenes);
    ctx->kmax_cur = 0;
    for (int32_t s = 0; s <= n_scenes; ++s) ctx->h_off32[s] = (int32_t)off[s];
    ctx->h_chunks.clear();
    for (int32_t s = 0; s < n_scenes; ++s)
        for (int64_t a = off[s]; a < off[s + 1]; a += orca::kBboxChunk)
            ctx->h_chunks.push_back(make_int2(s, (int32_t)a));
    for (int32_t s = 0; s < n_scenes; ++s) {
        SceneDev d;
        d.radius = par[s].radius;
        d.vmax = par[s].max_speed;
        d.nd = par[s].neighbor_dist;
        d.tau = par[s].time_horizon;
        d.dt = par[s].dt;
        d.pref_speed = par[s].pref_speed;
        volatile float nd = par[s].neighbor_dist;
        d.nd2 = nd * nd;  // float32 product, as every distance test rounds it
        d.k = par[s].max_neighbors;
        ctx->h_sp[s] = d;
        if (d.k > ctx->kmax_cur) ctx->kmax_cur = d.k;
    }
    HIP_OK(hipMemcpyAsync(ctx->off, ctx->h_off32.data(), sizeof(int32_t) * (size_t)(n_scenes + 1),
                          hipMemcpyHostToDevice, ctx->stream));
    HIP_OK(hipMemcpyAsync(ctx->sp, ctx->h_sp.data(), sizeof(SceneDev) * (size_t)n_scenes,
                          hipMemcpyHostToDevice, ctx->stream));
    if (!ctx->h_chunks.empty())
        HIP_OK(hipMemcpyAsync(ctx->chunks, ctx->h_chunks.data(),
                              sizeof(int2) * ctx->h_chunks.size(), hipMemcpyHostToDevice,
                              ctx->stream));
    HIP_OK(orca::launch_scene_map(ctx->off, n_scenes, ctx->agent_scene, (int32_t)ctx->n, ctx->bbox,
                                  ctx->stream));
    ctx->uploaded = true;
    ctx->grid_valid = false;
    ++ctx->scene_version;
    return ORCA_OK;
}

orca::Plan make_plan(const orca_ctx *ctx)
{
    orca::Plan p{};
    p.n = (int32_t)ctx->n;
    p.n_scenes = ctx->n_scenes;
    p.ld = (int32_t)ctx->max_agents;
    p.cus = ctx->cus;
    p.knn_block = ctx->knn_block;
    p.fb_waves_per_cu = ctx->fb_waves_per_cu;
    p.vel_apl = ctx->vel_apl;
    p.vel_waves_per_cu = ctx->vel_waves_per_cu;
    p.fb_work_units = ctx->fb_work_units;
    p.max_cells = ctx->max_cells;
    p.off = ctx->off;
    p.sp = ctx->sp;
    p.agent_scene = ctx->agent_scene;
    p.bbox = ctx->bbox;
    p.chunks = ctx->chunks;
    p.n_chunks = (int32_t)ctx->h_chunks.size();
    p.grid = ctx->grid;
    p.counters = ctx->counters;
    p.key = ctx->key;
    p.rank = ctx->rank;
    p.counts = ctx->counts;
    p.cell_start = ctx->cell_start;
    p.partial = ctx->partial;
    p.sorted = ctx->sorted;
    p.sid = ctx->sid;
    p.inv = ctx->inv;
    p.nbr = ctx->nbr;
    p.ncount = ctx->ncount;
    p.kcap = ctx->k_max;
    p.fb_list = ctx->fb_list;
    p.fb_key = ctx->fb_key;
    p.fb_order = ctx->fb_order;
    p.stash_n = ctx->stash_n;
    p.stash_b = ctx->stash_b;
    p.out.ag.radius = ctx->a_radius;
    p.out.ag.max_speed = ctx->a_vmax;
    p.out.ag.pref_speed = ctx->a_speed;
    p.out.ag.srad = ctx->srad;
    p.out.life.spawn_step = ctx->l_spawn;
    p.out.life.state = ctx->l_state;
    p.out.life.sp = ctx->sp;
    p.out.life.agent_scene = ctx->agent_scene;
    p.out.life.counters = ctx->counters;
    return p;
}

constexpr int64_t kProfPasses = 1024;  // passes a no-wait profile records

#define STAGE_MARK(i)                                                                     \
    do {                                                                                  \
        if (ctx->profiling && ctx->prof_mode == 1)                                        \
            HIP_OK(hipEventRecord(ctx->ev[(i)], ctx->stream));                            \
        if (ctx->profiling && ctx->prof_mode == 2 && ctx->prof_steps < kProfPasses)       \
            HIP_OK(hipEventRecord(ctx->pev[ctx->prof_steps * (ORCA_PROF_STAGES + 1) + (i)], \
                                  ctx->stream));                                          \
    } while (0)

// Enqueue one pass: optional grid build, then neighbours, 2D LP, fallback.
// With profiling on, the stream is drained after the pass and the time
// between the stage events is accumulated.
int run_pass(orca_ctx *ctx, const orca::Plan &pl_in, const float *grid_pos, const float *grid_vel)
{
    orca::Plan pl = pl_in;
    if (ctx->profiling && ctx->prof_mode == 2 && ctx->prof_steps < kProfPasses)
        pl.fb_total = ctx->fb_total;
    STAGE_MARK(0);
    if (grid_pos) {
        HIP_OK(orca::launch_grid(pl, grid_pos, grid_vel, true, ctx->stream));
        if (ctx->l_spawn) ctx->life_binned = true;
    }
    STAGE_MARK(1);
    HIP_OK(orca::launch_knn(pl, ctx->kmax_cur, ctx->stream));
    STAGE_MARK(2);
    HIP_OK(orca::launch_lp(pl, ctx->kmax_cur, ctx->stream));
    STAGE_MARK(3);
    HIP_OK(orca::launch_fallback(pl, ctx->kmax_cur, ctx->stream));
    STAGE_MARK(4);
    if (ctx->profiling && ctx->prof_mode == 2) {
        if (ctx->prof_steps < kProfPasses) ctx->prof_steps += 1;
        return ORCA_OK;
    }
    if (ctx->profiling) {
        HIP_OK(hipEventSynchronize(ctx->ev[ORCA_PROF_STAGES]));
        for (int i = 0; i < ORCA_PROF_STAGES; ++i) {
            float ms = 0.f;
            HIP_OK(hipEventElapsedTime(&ms, ctx->ev[i], ctx->ev[i + 1]));
            ctx->stage_ms[i] += ms;
        }
        Counters c;
        HIP_OK(hipMemcpy(&c, ctx->counters, sizeof(c), hipMemcpyDeviceToHost));
        ctx->prof_fallback += c.n_fallback;
        ctx->prof_steps += 1;
    }
    return ORCA_OK;
}

// Buffers of step t of a resident run of n plain steps: the state stays in
// cell order between steps, so only the first step reads and only the last
// writes the caller's arrays in agent order.  Results equal those of one-step
// calls bit for bit (nothing depends on the order within a cell).  The id and
// goal buffers alternate so that the last step's ids are in ctx->sid.
void resident_step(const orca_ctx *ctx, orca::Plan &pl, int32_t t, int32_t n, const float *src)
{
    const int cur = (n - 1 - t) & 1;
    const bool in = t > 0, out = t < n - 1;
    pl.sid = cur == 0 ? ctx->sid : ctx->sid2;
    pl.sid_prev = in ? (cur == 0 ? ctx->sid2 : ctx->sid) : nullptr;
    pl.res_src = in ? ctx->nxt : nullptr;
    pl.sg_cur = ctx->sg[cur];
    pl.sg_prev = in ? ctx->sg[cur ^ 1] : nullptr;
    pl.sg_src = in ? nullptr : src;
    pl.out.sg = ctx->sg[cur];
    pl.out.nxt = out ? ctx->nxt : nullptr;
}

void drop_graph(orca_ctx *c)
{
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->gblock_exec) (void)hipGraphExecDestroy(c->gblock_exec);
    if (c->gblock) (void)hipGraphDestroy(c->gblock);
    c->graph_exec = nullptr;
    c->graph = nullptr;
    c->gblock_exec = nullptr;
    c->gblock = nullptr;
}

// Resident steps a block graph of orca_step_graph holds.
constexpr int32_t kGraphBlock = 10;

void free_all(orca_ctx *c)
{
    drop_graph(c);
    if (c->cap_stream) {
        (void)hipStreamDestroy(c->cap_stream);
        c->cap_stream = nullptr;
    }
    for (int i = 0; i <= ORCA_PROF_STAGES; ++i)
        if (c->ev[i]) {
            (void)hipEventDestroy(c->ev[i]);
            c->ev[i] = nullptr;
        }
    for (hipEvent_t &e : c->pev)
        if (e) (void)hipEventDestroy(e);
    c->pev.clear();
    for (void *p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
}

}  // namespace

extern "C" {

const char *orca_last_error(const orca_ctx *ctx)
{
    return ctx ? ctx->err : "no context";
}

int orca_create(orca_ctx **out, int64_t max_agents, int32_t max_scenes, int32_t k_max,
                int32_t tape_steps, void *hip_stream)
{
    if (!out) return ORCA_EINVAL;
    *out = nullptr;
    if (max_agents < 1 || max_agents > (int64_t)INT32_MAX / 2 || max_scenes < 1 ||
        max_scenes > (1 << 24) || k_max < 1 || tape_steps < 0)
        return ORCA_EINVAL;
    if (k_max > ORCA_K_LIMIT) return ORCA_ECAPACITY;
    orca_ctx *ctx = new (std::nothrow) orca_ctx;
    if (!ctx) return ORCA_ENOMEM;
    ctx->max_agents = max_agents;
    ctx->max_scenes = max_scenes;
    ctx->k_max = k_max;
    ctx->tape_steps = tape_steps;
    ctx->stream = (hipStream_t)hip_stream;
    // cell budget: room for 4 cells per agent plus a margin per scene
    const int64_t cells = 4 * max_agents + 64 * (int64_t)max_scenes + 4096;
    ctx->max_cells = (uint32_t)(cells < (int64_t)INT32_MAX - 2 ? cells : (int64_t)INT32_MAX - 2);
    // the scan also covers the cell of absent agents (spawning and removal)
    ctx->n_tiles = (int32_t)((ctx->max_cells + 1 + orca::kScanTile - 1) / orca::kScanTile);
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
            cus = prop.multiProcessorCount;
    }
    ctx->cus = cus;
    // each scene's agents split into chunks of kBboxChunk: at most A / chunk + S chunks
    ctx->max_chunks = max_agents / orca::kBboxChunk + max_scenes + 1;

    auto alloc = [&](void **p, size_t bytes) -> bool {
        if (hipMalloc(p, bytes < 256 ? 256 : bytes) != hipSuccess) {
            *p = nullptr;
            return false;
        }
        ctx->allocs.push_back(*p);
        return true;
    };
    const size_t A = (size_t)max_agents, S = (size_t)max_scenes, C = (size_t)ctx->max_cells;
    bool ok = alloc((void **)&ctx->off, sizeof(int32_t) * (S + 1)) &&
              alloc((void **)&ctx->sp, sizeof(SceneDev) * S) &&
              alloc((void **)&ctx->agent_scene, sizeof(int32_t) * A) &&
              alloc((void **)&ctx->bbox, sizeof(uint32_t) * 4 * S) &&
              alloc((void **)&ctx->chunks, sizeof(int2) * (size_t)ctx->max_chunks) &&
              alloc((void **)&ctx->grid, sizeof(GridDev) * S) &&
              alloc((void **)&ctx->counters, sizeof(Counters)) &&
              alloc((void **)&ctx->key, sizeof(int32_t) * A) &&
              alloc((void **)&ctx->rank, sizeof(int32_t) * A) &&
              alloc((void **)&ctx->counts, sizeof(int32_t) * (C + 1)) &&
              alloc((void **)&ctx->cell_start, sizeof(int32_t) * (C + 2)) &&
              alloc((void **)&ctx->partial, sizeof(uint32_t) * (size_t)ctx->n_tiles) &&
              alloc((void **)&ctx->sorted, sizeof(float4) * A) &&
              alloc((void **)&ctx->sid, sizeof(int32_t) * A) &&
              alloc((void **)&ctx->inv, sizeof(int32_t) * A) &&
              alloc((void **)&ctx->nbr, sizeof(int32_t) * A * (size_t)k_max) &&
              alloc((void **)&ctx->ncount, sizeof(int32_t) * A) &&
              alloc((void **)&ctx->fb_list, sizeof(orca::FallbackItem) * A) &&
              alloc((void **)&ctx->fb_key, sizeof(uint8_t) * A) &&
              alloc((void **)&ctx->fb_order, sizeof(int32_t) * A) &&
              alloc((void **)&ctx->stash_n, sizeof(double2) * A * (size_t)k_max) &&
              alloc((void **)&ctx->stash_b, sizeof(double) * A * (size_t)k_max) &&
              alloc((void **)&ctx->srad, sizeof(float) * A) &&
              alloc((void **)&ctx->nxt, sizeof(float4) * A) &&
              alloc((void **)&ctx->sid2, sizeof(int32_t) * A) &&
              alloc((void **)&ctx->sg[0], sizeof(float2) * A) &&
              alloc((void **)&ctx->sg[1], sizeof(float2) * A) &&
              alloc((void **)&ctx->fb_total, sizeof(unsigned long long)) &&
              alloc((void **)&ctx->acc, sizeof(double) * 4 * A) &&
              alloc((void **)&ctx->own, sizeof(double) * 4 * A) &&
              alloc((void **)&ctx->acc_scene, sizeof(double) * 2 * S);
    const size_t T = (size_t)tape_steps;
    if (ok && T > 0)
        ok = alloc((void **)&ctx->g4, sizeof(float4) * A) &&
             alloc((void **)&ctx->pref2, sizeof(float2) * A) &&
             alloc((void **)&ctx->g_pref2, sizeof(float2) * A) &&
             alloc((void **)&ctx->tape_state, sizeof(float4) * T * A) &&
             alloc((void **)&ctx->tape_nbr, sizeof(int32_t) * T * A * (size_t)k_max) &&
             alloc((void **)&ctx->tape_codes, sizeof(orca::TapeCode) * T * A) &&
             alloc((void **)&ctx->tape_sid, sizeof(int32_t) * T * A);
    if (!ok) {
        free_all(ctx);
        delete ctx;
        return ORCA_ENOMEM;
    }
    // counts start at zero and are kept zero between uses by the scan
    hipError_t e = hipMemsetAsync(ctx->counts, 0, sizeof(int32_t) * (C + 1), ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->counters, 0, sizeof(Counters), ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->acc, 0, sizeof(double) * 4 * A, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->acc_scene, 0, sizeof(double) * 2 * S, ctx->stream);
    if (e == hipSuccess) e = orca::launch_scene_map(ctx->off, max_scenes, ctx->agent_scene, 0,
                                                    ctx->bbox, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        free_all(ctx);
        delete ctx;
        return ORCA_EHIP;
    }
    *out = ctx;
    return ORCA_OK;
}

void orca_destroy(orca_ctx *ctx)
{
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    free_all(ctx);
    delete ctx;
}

int orca_set_stream(orca_ctx *ctx, void *hip_stream)
{
    if (!ctx) return ORCA_EINVAL;
    ctx->stream = (hipStream_t)hip_stream;
    return ORCA_OK;
}

int orca_build_grid(orca_ctx *ctx, int32_t n_scenes, const int64_t *scene_offsets,
                    const orca_params *params, const float *pos)
{
    if (!ctx) return ORCA_EINVAL;
    int rc = use_scenes(ctx, n_scenes, scene_offsets, params);
    if (rc != ORCA_OK) return rc;
    if (!pos && ctx->n > 0) return fail(ctx, ORCA_EINVAL, "pos must be non-NULL");
    const orca::Plan pl = make_plan(ctx);
    HIP_OK(orca::launch_grid(pl, pos, nullptr, false, ctx->stream));
    if (ctx->l_spawn) ctx->life_binned = true;
    ctx->grid_valid = true;
    ctx->grid_pos = pos;
    ctx->grid_radius = ctx->a_radius;
    return ORCA_OK;
}

int orca_set_agents(orca_ctx *ctx, const float *radius, const float *max_speed,
                    const float *pref_speed)
{
    if (!ctx) return ORCA_EINVAL;
    ctx->a_radius = radius;
    ctx->a_vmax = max_speed;
    ctx->a_speed = pref_speed;
    return ORCA_OK;
}

int orca_set_lifecycle(orca_ctx *ctx, const int32_t *spawn_step, uint8_t *state, int32_t t0)
{
    if (!ctx) return ORCA_EINVAL;
    if ((spawn_step == nullptr) != (state == nullptr))
        return fail(ctx, ORCA_EINVAL, "spawn_step and state must both be given or both be NULL");
    if (ctx->profiling) return fail(ctx, ORCA_ESTATE, "stop profiling before setting up spawning");
    ctx->l_spawn = spawn_step;
    ctx->l_state = state;
    ctx->grid_valid = false;
    ctx->life_binned = false;
    // step <- t0 (the staging word stays valid until the copy is done)
    HIP_OK(hipStreamSynchronize(ctx->stream));
    ctx->h_life = spawn_step ? t0 : 0;
    HIP_OK(hipMemcpyAsync(&ctx->counters->step, &ctx->h_life, sizeof(ctx->h_life),
                          hipMemcpyHostToDevice, ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    return ORCA_OK;
}

int orca_population(orca_ctx *ctx, int32_t *step, int64_t *present, int64_t *removed)
{
    if (!ctx) return ORCA_EINVAL;
    if (ctx->l_spawn && ctx->n > 0)
        HIP_OK(orca::launch_count_removed(ctx->l_state, (int32_t)ctx->n, ctx->counters,
                                          ctx->stream));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    Counters c;
    HIP_OK(hipMemcpy(&c, ctx->counters, sizeof(c), hipMemcpyDeviceToHost));
    int64_t np = ctx->n;
    if (ctx->l_spawn) {
        np = -1;
        if (ctx->life_binned && c.total_cells >= 1) {
            int32_t v = 0;
            HIP_OK(hipMemcpy(&v, ctx->cell_start + (c.total_cells - 1), sizeof(v),
                             hipMemcpyDeviceToHost));
            np = v;
        }
    }
    if (step) *step = ctx->l_spawn ? c.step : 0;
    if (present) *present = np;
    if (removed) *removed = ctx->l_spawn ? (int64_t)c.removed : 0;
    return ORCA_OK;
}

int orca_compute_velocities(orca_ctx *ctx, const float *pos, const float *vel,
                            const float *pref_vel, const float *goals, float *new_vel,
                            int32_t *nbr_out, uint8_t *lp_status)
{
    if (!ctx) return ORCA_EINVAL;
    if (!ctx->grid_valid || pos != ctx->grid_pos)
        return fail(ctx, ORCA_ESTATE, "orca_build_grid must be called first on the same pos");
    if (ctx->grid_radius != ctx->a_radius)
        return fail(ctx, ORCA_ESTATE, "per-agent radii changed since orca_build_grid");
    if (ctx->n > 0 && (!vel || !new_vel || (!goals && !pref_vel)))
        return fail(ctx, ORCA_EINVAL, "vel, new_vel and pref_vel (or goals) must be non-NULL");
    orca::Plan pl = make_plan(ctx);
    pl.out.new_vel = new_vel;
    pl.out.pref = const_cast<float *>(pref_vel);
    pl.out.goals = goals;
    pl.out.status = lp_status;
    pl.out.nbr_out = nbr_out;
    pl.out.krow = ctx->kmax_cur;
    HIP_OK(orca::launch_fill_vel(pl, vel, ctx->stream));
    return run_pass(ctx, pl, nullptr, nullptr);
}

int orca_step(orca_ctx *ctx, int32_t n_scenes, const int64_t *scene_offsets,
              const orca_params *params, float *pos, float *vel, float *pref_vel,
              const float *goals, int32_t n_steps, int32_t save_tape)
{
    if (!ctx) return ORCA_EINVAL;
    if (n_steps < 1) return fail(ctx, ORCA_EINVAL, "n_steps must be >= 1");
    if (save_tape != 0 && save_tape != 1) return fail(ctx, ORCA_EINVAL, "save_tape must be 0 or 1");
    int rc = use_scenes(ctx, n_scenes, scene_offsets, params);
    if (rc != ORCA_OK) return rc;
    if (ctx->n > 0 && (!pos || !vel || !pref_vel))
        return fail(ctx, ORCA_EINVAL, "pos, vel and pref_vel must be non-NULL");
    if (ctx->l_spawn && !goals)
        return fail(ctx, ORCA_EINVAL, "spawning and removal need goals");
    if (save_tape) {
        if (ctx->l_spawn)
            return fail(ctx, ORCA_EINVAL, "a recorded step cannot use spawning and removal");
        if (goals) return fail(ctx, ORCA_EINVAL, "a recorded step needs fixed preferred velocities");
        if (n_steps > ctx->tape_steps)
            return fail(ctx, ORCA_ECAPACITY, "n_steps %d exceeds tape_steps %d", n_steps,
                        ctx->tape_steps);
    }
    orca::Plan pl = make_plan(ctx);
    pl.out.pos = pos;
    pl.out.vel = vel;
    pl.out.pref = pref_vel;
    pl.out.goals = goals;
    ctx->grid_valid = false;
    if (save_tape) ctx->tape_len = 0;
    // the steps of a multi-step call run resident (resident_step), recorded
    // ones too (not with spawning and removal)
    const bool resident = n_steps > 1 && !ctx->l_spawn;
    for (int32_t t = 0; t < n_steps; ++t) {
        if (resident) resident_step(ctx, pl, t, n_steps, goals ? goals : pref_vel);
        if (save_tape) {
            // the step's neighbour lists and cell-order ids go straight to
            // the tape slot (a resident step takes the previous step's ids
            // from the previous slot); state and choices are written by
            // sorted index
            const size_t A = (size_t)ctx->max_agents;
            pl.out.tape_state = ctx->tape_state + (size_t)t * A;
            pl.out.tape_codes = ctx->tape_codes + (size_t)t * A;
            pl.nbr = ctx->tape_nbr + (size_t)t * A * (size_t)ctx->k_max;
            pl.sid = ctx->tape_sid + (size_t)t * A;
            if (resident && t > 0) pl.sid_prev = ctx->tape_sid + (size_t)(t - 1) * A;
        }
        rc = run_pass(ctx, pl, pos, vel);
        if (rc != ORCA_OK) return rc;
    }
    if (save_tape) {
        ctx->tape_len = n_steps;
        ctx->tape_scene_version = ctx->scene_version;
        ctx->tape_pref = pref_vel;
        ctx->tape_radius = ctx->a_radius;
        ctx->tape_vmax = ctx->a_vmax;
    }
    return ORCA_OK;
}

int orca_step_graph(orca_ctx *ctx, int32_t n_scenes, const int64_t *scene_offsets,
                    const orca_params *params, float *pos, float *vel, float *pref_vel,
                    const float *goals, int32_t n_steps)
{
    if (!ctx) return ORCA_EINVAL;
    if (n_steps < 1) return fail(ctx, ORCA_EINVAL, "n_steps must be >= 1");
    if (ctx->profiling) return fail(ctx, ORCA_ESTATE, "stop profiling before replaying a graph");
    int rc = use_scenes(ctx, n_scenes, scene_offsets, params);
    if (rc != ORCA_OK) return rc;
    if (ctx->n > 0 && (!pos || !vel || !pref_vel))
        return fail(ctx, ORCA_EINVAL, "pos, vel and pref_vel must be non-NULL");
    if (ctx->l_spawn && !goals)
        return fail(ctx, ORCA_EINVAL, "spawning and removal need goals");
    ctx->grid_valid = false;
    const void *key[9] = {pos,           vel,         pref_vel,     goals,      ctx->a_radius,
                          ctx->a_vmax,   ctx->a_speed, ctx->l_spawn, ctx->l_state};
    const bool fresh = ctx->graph_exec && memcmp(key, ctx->graph_key, sizeof(key)) == 0 &&
                       ctx->graph_scene_version == ctx->scene_version &&
                       ctx->graph_knn_block == ctx->knn_block &&
                       ctx->graph_fb == ctx->fb_waves_per_cu && ctx->graph_apl == ctx->vel_apl &&
                       ctx->graph_vw == ctx->vel_waves_per_cu &&
                       ctx->graph_wu == ctx->fb_work_units;
    // blocks of resident steps for plain steps (not with spawning and removal)
    const bool blocks = !ctx->l_spawn && n_steps >= kGraphBlock;
    if (!fresh) {
        drop_graph(ctx);
        memset(ctx->graph_key, 0, sizeof(ctx->graph_key));
    }
    if (!ctx->graph_exec || (blocks && !ctx->gblock_exec)) {
        if (!ctx->cap_stream) HIP_OK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        // the uploads of use_scenes must be done before the captured kernels replay
        HIP_OK(hipStreamSynchronize(ctx->stream));
        orca::Plan pl = make_plan(ctx);
        pl.out.pos = pos;
        pl.out.vel = vel;
        pl.out.pref = pref_vel;
        pl.out.goals = goals;
        // capture one step (nb == 1) or a block of nb resident steps
        auto capture = [&](int32_t nb, hipGraph_t *graph, hipGraphExec_t *exec) -> int {
            hipStream_t user = ctx->stream;
            ctx->stream = ctx->cap_stream;
            int r = ORCA_OK;
            hipError_t e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                orca::Plan q = pl;
                for (int32_t t = 0; t < nb && r == ORCA_OK; ++t) {
                    if (nb > 1) resident_step(ctx, q, t, nb, goals ? goals : pref_vel);
                    r = run_pass(ctx, q, pos, vel);
                }
                hipGraph_t g = nullptr;
                hipError_t e2 = hipStreamEndCapture(ctx->cap_stream, &g);
                *graph = g;
                if (r == ORCA_OK && e2 != hipSuccess) r = hip_fail(ctx, e2, "hipStreamEndCapture");
            } else {
                r = hip_fail(ctx, e, "hipStreamBeginCapture");
            }
            ctx->stream = user;
            if (r == ORCA_OK) {
                e = hipGraphInstantiate(exec, *graph, nullptr, nullptr, 0);
                if (e != hipSuccess) r = hip_fail(ctx, e, "hipGraphInstantiate");
            }
            return r;
        };
        if (!ctx->graph_exec) rc = capture(1, &ctx->graph, &ctx->graph_exec);
        if (rc == ORCA_OK && blocks && !ctx->gblock_exec)
            rc = capture(kGraphBlock, &ctx->gblock, &ctx->gblock_exec);
        if (rc != ORCA_OK) {
            drop_graph(ctx);
            return rc;
        }
        memcpy(ctx->graph_key, key, sizeof(key));
        ctx->graph_scene_version = ctx->scene_version;
        ctx->graph_knn_block = ctx->knn_block;
        ctx->graph_fb = ctx->fb_waves_per_cu;
        ctx->graph_apl = ctx->vel_apl;
        ctx->graph_vw = ctx->vel_waves_per_cu;
        ctx->graph_wu = ctx->fb_work_units;
    }
    int32_t t = 0;
    if (blocks)
        for (; t + kGraphBlock <= n_steps; t += kGraphBlock)
            HIP_OK(hipGraphLaunch(ctx->gblock_exec, ctx->stream));
    for (; t < n_steps; ++t) HIP_OK(hipGraphLaunch(ctx->graph_exec, ctx->stream));
    return ORCA_OK;
}

int orca_autotune(orca_ctx *ctx, const float *pos, const float *vel, const float *pref_vel,
                  const float *goals, float *new_vel, int32_t reps, int32_t *choice)
{
    if (!ctx) return ORCA_EINVAL;
    if (reps < 1) return fail(ctx, ORCA_EINVAL, "reps must be >= 1");
    if (!ctx->grid_valid || pos != ctx->grid_pos)
        return fail(ctx, ORCA_ESTATE, "orca_build_grid must be called first on the same pos");
    static const int32_t blocks[] = {64, 128, 256, 512};
    static const int32_t waves[] = {4, 8, 16, 32};
    static const int32_t apls[] = {1, 2, 4};
    static const int32_t vwaves[] = {8, 12};
    const bool was = ctx->profiling;
    int rc = orca_profile(ctx, 1);
    if (rc != ORCA_OK) return rc;
    const int32_t apl0 = ctx->vel_apl, vw0 = ctx->vel_waves_per_cu, wu0 = ctx->fb_work_units;
    const int32_t fb0 = ctx->fb_waves_per_cu;
    ctx->fb_work_units = 0;
    // one untimed pass with the candidate's shapes, then the fastest of reps
    // timed passes per stage (a sum would carry the noise of every pass)
    auto time_stages = [&](double (&best)[ORCA_PROF_STAGES]) {
        for (double &b : best) b = 1e300;
        for (int32_t r = 0; r <= reps && rc == ORCA_OK; ++r) {
            orca_profile(ctx, 1);
            rc = orca_compute_velocities(ctx, pos, vel, pref_vel, goals, new_vel, nullptr, nullptr);
            if (r > 0)
                for (int i = 0; i < ORCA_PROF_STAGES; ++i) best[i] = std::min(best[i], ctx->stage_ms[i]);
        }
    };
    // split kernels: neighbour block size and fallback waves (independent stages)
    double best_knn = 1e300, best_lp = 1e300, best_fb = 1e300;
    int32_t knn_block = ctx->knn_block, fb = ctx->fb_waves_per_cu;
    ctx->vel_apl = 0;
    for (int t = 0; t < 4 && rc == ORCA_OK; ++t) {
        ctx->knn_block = blocks[t];
        ctx->fb_waves_per_cu = waves[t];
        double st[ORCA_PROF_STAGES];
        time_stages(st);
        if (rc != ORCA_OK) break;
        if (st[1] < best_knn) {
            best_knn = st[1];
            knn_block = blocks[t];
        }
        best_lp = std::min(best_lp, st[2]);
        if (st[3] < best_fb) {
            best_fb = st[3];
            fb = waves[t];
        }
    }
    ctx->knn_block = knn_block;
    ctx->fb_waves_per_cu = fb;
    // the fused velocity kernel: agents per lane and waves per CU, against
    // the split kernels' neighbour + LP stages
    double best_vel = best_knn + best_lp;
    int32_t apl = 0, vw = vw0;
    for (int a = 0; a < 3 && rc == ORCA_OK; ++a)
        for (int w = 0; w < 2 && rc == ORCA_OK; ++w) {
            ctx->vel_apl = apls[a];
            ctx->vel_waves_per_cu = vwaves[w];
            double st[ORCA_PROF_STAGES];
            time_stages(st);
            if (rc == ORCA_OK && st[1] + st[2] < best_vel) {
                best_vel = st[1] + st[2];
                apl = apls[a];
                vw = vwaves[w];
            }
        }
    ctx->vel_apl = rc == ORCA_OK ? apl : apl0;
    ctx->vel_waves_per_cu = rc == ORCA_OK ? vw : vw0;
    // the fallback with work units (its LDS holds it to 6 waves per CU)
    int32_t wu = 0;
    if (rc == ORCA_OK && ctx->kmax_cur <= 16) {
        const int32_t fb_plain = ctx->fb_waves_per_cu;
        ctx->fb_work_units = 1;
        ctx->fb_waves_per_cu = 6;
        double st[ORCA_PROF_STAGES];
        time_stages(st);
        if (rc == ORCA_OK && st[3] < best_fb) wu = 1;
        else ctx->fb_waves_per_cu = fb_plain;
    }
    ctx->fb_work_units = rc == ORCA_OK ? wu : wu0;
    if (rc != ORCA_OK) ctx->fb_waves_per_cu = fb0;
    orca_profile(ctx, was ? 1 : 0);
    if (rc != ORCA_OK) return rc;
    if (choice) {
        choice[0] = ctx->knn_block;
        choice[1] = ctx->fb_waves_per_cu;
        choice[2] = ctx->vel_apl;
        choice[3] = ctx->vel_waves_per_cu;
        choice[4] = ctx->fb_work_units;
    }
    return ORCA_OK;
}

int orca_set_launch(orca_ctx *ctx, int32_t knn_block, int32_t fb_waves_per_cu)
{
    if (!ctx) return ORCA_EINVAL;
    if (knn_block != 64 && knn_block != 128 && knn_block != 256 && knn_block != 512)
        return fail(ctx, ORCA_EINVAL, "knn_block must be 64, 128, 256 or 512");
    if (fb_waves_per_cu < 1 || fb_waves_per_cu > 64)
        return fail(ctx, ORCA_EINVAL, "fb_waves_per_cu must be in 1..64");
    ctx->knn_block = knn_block;
    ctx->fb_waves_per_cu = fb_waves_per_cu;
    return ORCA_OK;
}

int orca_set_kernels(orca_ctx *ctx, int32_t agents_per_lane, int32_t velocity_waves_per_cu,
                     int32_t fallback_work_units)
{
    if (!ctx) return ORCA_EINVAL;
    if (agents_per_lane != 0 && agents_per_lane != 1 && agents_per_lane != 2 &&
        agents_per_lane != 4)
        return fail(ctx, ORCA_EINVAL, "agents_per_lane must be 0, 1, 2 or 4");
    if (velocity_waves_per_cu < 1 || velocity_waves_per_cu > 32)
        return fail(ctx, ORCA_EINVAL, "velocity_waves_per_cu must be in 1..32");
    if (fallback_work_units != 0 && fallback_work_units != 1)
        return fail(ctx, ORCA_EINVAL, "fallback_work_units must be 0 or 1");
    ctx->vel_apl = agents_per_lane;
    ctx->vel_waves_per_cu = velocity_waves_per_cu;
    ctx->fb_work_units = fallback_work_units;
    return ORCA_OK;
}

int orca_profile(orca_ctx *ctx, int32_t enable)
{
    if (!ctx) return ORCA_EINVAL;
    if (enable < 0 || enable > 2) return fail(ctx, ORCA_EINVAL, "enable must be 0, 1 or 2");
    if (enable == 1) {
        for (int i = 0; i <= ORCA_PROF_STAGES; ++i)
            if (!ctx->ev[i]) HIP_OK(hipEventCreate(&ctx->ev[i]));
    }
    if (enable == 2) {
        if (ctx->pev.empty()) {
            ctx->pev.assign((size_t)kProfPasses * (ORCA_PROF_STAGES + 1), nullptr);
            for (hipEvent_t &e : ctx->pev) HIP_OK(hipEventCreate(&e));
        }
        HIP_OK(hipMemsetAsync(ctx->fb_total, 0, sizeof(unsigned long long), ctx->stream));
    }
    ctx->profiling = enable != 0;
    ctx->prof_mode = enable;
    for (int i = 0; i < ORCA_PROF_STAGES; ++i) ctx->stage_ms[i] = 0.0;
    ctx->prof_steps = 0;
    ctx->prof_fallback = 0;
    return ORCA_OK;
}

int orca_profile_read(orca_ctx *ctx, double *stage_ms, int64_t *passes, int64_t *fallback_agents)
{
    if (!ctx || !stage_ms) return ORCA_EINVAL;
    if (ctx->profiling && ctx->prof_mode == 2) {
        // the recorded passes' events, summed once the stream has reached them
        HIP_OK(hipStreamSynchronize(ctx->stream));
        for (int i = 0; i < ORCA_PROF_STAGES; ++i) ctx->stage_ms[i] = 0.0;
        for (int64_t p = 0; p < ctx->prof_steps; ++p)
            for (int i = 0; i < ORCA_PROF_STAGES; ++i) {
                float ms = 0.f;
                HIP_OK(hipEventElapsedTime(&ms, ctx->pev[p * (ORCA_PROF_STAGES + 1) + i],
                                           ctx->pev[p * (ORCA_PROF_STAGES + 1) + i + 1]));
                ctx->stage_ms[i] += ms;
            }
        unsigned long long fb = 0;
        HIP_OK(hipMemcpy(&fb, ctx->fb_total, sizeof(fb), hipMemcpyDeviceToHost));
        ctx->prof_fallback = (int64_t)fb;
    }
    for (int i = 0; i < ORCA_PROF_STAGES; ++i) stage_ms[i] = ctx->stage_ms[i];
    if (passes) *passes = ctx->prof_steps;
    if (fallback_agents) *fallback_agents = ctx->prof_fallback;
    return ORCA_OK;
}

}  // extern "C"

namespace {

// Arguments of the adjoint of recorded step tape_step (agent-order [2, N]
// gradient arrays; the caller sets the by-id buffers of a run of steps).
orca::BackArgs back_args(const orca_ctx *ctx, int32_t tape_step, const float *g_pos_next,
                         const float *g_vel_next, float *g_pos, float *g_vel, float *g_pref_vel,
                         float *g_max_speed, float *g_time_horizon)
{
    const size_t A = (size_t)ctx->max_agents;
    orca::BackArgs a{};
    a.n = (int32_t)ctx->n;
    a.n_scenes = ctx->n_scenes;
    a.ld = (int32_t)A;
    a.agent_scene = ctx->agent_scene;
    a.sp = ctx->sp;
    a.state = ctx->tape_state + (size_t)tape_step * A;
    a.nbr = ctx->tape_nbr + (size_t)tape_step * A * (size_t)ctx->k_max;
    a.codes = ctx->tape_codes + (size_t)tape_step * A;
    a.sid = ctx->tape_sid + (size_t)tape_step * A;
    a.pref = ctx->tape_pref;
    a.g_pos_next = g_pos_next;
    a.g_vel_next = g_vel_next;
    a.g_pos = g_pos;
    a.g_vel = g_vel;
    a.g_pref = g_pref_vel;
    a.g_max_speed = g_max_speed;
    a.g_time_horizon = g_time_horizon;
    a.acc = ctx->acc;
    a.own = ctx->own;
    a.acc_scene = ctx->acc_scene;
    a.radius = ctx->tape_radius;
    a.max_speed = ctx->tape_vmax;
    return a;
}

int check_backward(orca_ctx *ctx, int32_t first, int32_t last, const float *g_pos_next,
                   const float *g_vel_next, const float *g_pos, const float *g_vel,
                   const float *g_pref_vel)
{
    if (first < 0 || last < first || last >= ctx->tape_len)
        return fail(ctx, ORCA_ESTATE, "no recorded steps %d..%d (the last recording holds %d)",
                    first, last, ctx->tape_len);
    if (ctx->tape_scene_version != ctx->scene_version)
        return fail(ctx, ORCA_ESTATE, "the scene set changed since the steps were recorded");
    if (ctx->n > 0 && (!g_pos_next || !g_vel_next || !g_pos || !g_vel || !g_pref_vel))
        return fail(ctx, ORCA_EINVAL, "gradient arrays must be non-NULL");
    return ORCA_OK;
}

}  // namespace

extern "C" {

int orca_backward(orca_ctx *ctx, int32_t tape_step, const float *g_pos_next,
                  const float *g_vel_next, float *g_pos, float *g_vel, float *g_pref_vel,
                  float *g_max_speed, float *g_time_horizon)
{
    if (!ctx) return ORCA_EINVAL;
    int rc = check_backward(ctx, tape_step, tape_step, g_pos_next, g_vel_next, g_pos, g_vel,
                            g_pref_vel);
    if (rc != ORCA_OK) return rc;
    const orca::BackArgs a = back_args(ctx, tape_step, g_pos_next, g_vel_next, g_pos, g_vel,
                                       g_pref_vel, g_max_speed, g_time_horizon);
    HIP_OK(orca::launch_backward(a, ctx->stream));
    return ORCA_OK;
}

int orca_backward_steps(orca_ctx *ctx, int32_t first, int32_t last, const float *g_pos_next,
                        const float *g_vel_next, float *g_pos, float *g_vel, float *g_pref_vel,
                        float *g_max_speed, float *g_time_horizon)
{
    if (!ctx) return ORCA_EINVAL;
    int rc = check_backward(ctx, first, last, g_pos_next, g_vel_next, g_pos, g_vel, g_pref_vel);
    if (rc != ORCA_OK) return rc;
    const int32_t n = (int32_t)ctx->n;
    // the gradients between the steps stay one float4 per agent id in g4
    // (each step reads and then writes each id's entry), the preferred
    // velocities and their gradient one float2 per agent id
    HIP_OK(orca::launch_backward_prep(ctx->tape_pref, ctx->pref2, ctx->g_pref2, n, ctx->stream));
    for (int32_t t = last; t >= first; --t) {
        orca::BackArgs a = back_args(ctx, t, g_pos_next, g_vel_next, g_pos, g_vel, g_pref_vel,
                                     g_max_speed, g_time_horizon);
        a.pref2 = ctx->pref2;
        a.g_pref2 = ctx->g_pref2;
        a.g_in4 = t == last ? nullptr : ctx->g4;
        a.g_out4 = t == first ? nullptr : ctx->g4;
        HIP_OK(orca::launch_backward(a, ctx->stream));
    }
    HIP_OK(orca::launch_backward_post(ctx->g_pref2, g_pref_vel, n, ctx->stream));
    return ORCA_OK;
}

}  // extern "C"
