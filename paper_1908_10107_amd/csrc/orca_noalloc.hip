// orca_noalloc.hip -- orca_step for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).
//
// The step's scratch (scene table, grid, counting-sort arrays, neighbour
// lists, fallback list and half-plane stash) lives in one file-scope device
// array, `scratch`, of fixed size, carved into the same buffers an orca_ctx
// allocates for kNoAllocAgents agents in one scene with neighbour caps up to
// kNoAllocK.  The step then runs the same kernels, with the same default
// launch shapes, as orca_step on a fresh context.
//
// In host code the array's name is only a stand-in for the symbol: its
// device address comes from hipGetSymbolAddress, taken once per device (with
// that device current) and kept.  Every call on a device shares that
// device's array and leaves the last call's contents in it; each call clears
// what must start at zero with kernels (no memset nodes, so the call can be
// captured into a graph).  Calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>

#include <math.h>
#include <mutex>

#include "orca.h"
#include "orca_internal.h"

namespace orca {
namespace {

constexpr int32_t kNoAllocAgents = ORCA_NOALLOC_MAX_AGENTS;
constexpr int32_t kNoAllocK = ORCA_NOALLOC_MAX_NEIGHBORS;
constexpr int32_t kMaxDevices = 64;
constexpr size_t kAlign = 256;

// Cell budget of a one-scene context of kNoAllocAgents agents (orca_create's
// rule: 4 cells per agent plus a per-scene margin).
constexpr uint32_t kNoAllocCells = 4u * kNoAllocAgents + 64u + 4096u;
constexpr int32_t kNoAllocTiles = (int32_t)((kNoAllocCells + 1 + kScanTile - 1) / kScanTile);
constexpr int32_t kNoAllocChunks = kNoAllocAgents / kBboxChunk + 2;

constexpr size_t up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// Byte offsets of the buffers inside scratch, in one fixed order.
struct Layout {
    size_t off, sp, agent_scene, bbox, chunks, grid, counters, key, rank, counts, cell_start,
        partial, sorted, sid, inv, nbr, ncount, fb_list, fb_key, fb_order, stash_n, stash_b, end;
};

constexpr Layout make_layout()
{
    const size_t A = (size_t)kNoAllocAgents, K = (size_t)kNoAllocK, C = (size_t)kNoAllocCells;
    Layout l{};
    size_t o = 0;
    l.off = o;          o += up(sizeof(int32_t) * 2);
    l.sp = o;           o += up(sizeof(SceneDev));
    l.agent_scene = o;  o += up(sizeof(int32_t) * A);
    l.bbox = o;         o += up(sizeof(uint32_t) * 4);
    l.chunks = o;       o += up(sizeof(int2) * (size_t)kNoAllocChunks);
    l.grid = o;         o += up(sizeof(GridDev));
    l.counters = o;     o += up(sizeof(Counters));
    l.key = o;          o += up(sizeof(int32_t) * A);
    l.rank = o;         o += up(sizeof(int32_t) * A);
    l.counts = o;       o += up(sizeof(int32_t) * (C + 1));
    l.cell_start = o;   o += up(sizeof(int32_t) * (C + 2));
    l.partial = o;      o += up(sizeof(uint32_t) * (size_t)kNoAllocTiles);
    l.sorted = o;       o += up(sizeof(float4) * A);
    l.sid = o;          o += up(sizeof(int32_t) * A);
    l.inv = o;          o += up(sizeof(int32_t) * A);
    l.nbr = o;          o += up(sizeof(int32_t) * A * K);
    l.ncount = o;       o += up(sizeof(int32_t) * A);
    l.fb_list = o;      o += up(sizeof(FallbackItem) * A);
    l.fb_key = o;       o += up(sizeof(uint8_t) * A);
    l.fb_order = o;     o += up(sizeof(int32_t) * A);
    l.stash_n = o;      o += up(sizeof(double2) * A * K);
    l.stash_b = o;      o += up(sizeof(double) * A * K);
    l.end = o;
    return l;
}

constexpr Layout kLayout = make_layout();
static_assert(kLayout.end == ORCA_NOALLOC_SCRATCH_BYTES,
              "ORCA_NOALLOC_SCRATCH_BYTES must state the scratch array's size");

}  // namespace

// The scratch of orca_step_noalloc: one copy per device, held until the
// process ends.  Host code must not pass this name to a kernel (it is a
// host-side stand-in); it uses the address hipGetSymbolAddress gives.
static __device__ __align__(256) unsigned char scratch[kLayout.end];

namespace {

// Per call: the scene's parameters, offsets and bounding-box chunks (passed
// by value, so no host buffer has to outlive the call), the cell counts and
// the counters cleared.
__global__ __launch_bounds__(256) void k_noalloc_setup(SceneDev p, int32_t n,
                                                       int32_t *__restrict__ off,
                                                       SceneDev *__restrict__ sp,
                                                       int2 *__restrict__ chunks,
                                                       int32_t *__restrict__ counts,
                                                       int32_t n_counts,
                                                       Counters *__restrict__ counters)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_counts) counts[i] = 0;
    if (i == 0) {
        off[0] = 0;
        off[1] = n;
        *sp = p;
        Counters c{};
        *counters = c;
    }
    if (i < (n + kBboxChunk - 1) / kBboxChunk) chunks[i] = make_int2(0, i * kBboxChunk);
}

struct DeviceScratch {
    unsigned char *ptr = nullptr;  // device address of scratch on this device
    int32_t cus = 0;
};

std::mutex g_mu;
DeviceScratch g_dev[kMaxDevices];

int say(char *err, int32_t len, int code, const char *fmt, ...)
{
    if (err && len > 0) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(err, (size_t)len, fmt, ap);
        va_end(ap);
    }
    return code;
}

// The device address of scratch on the current device (looked up once per
// device, with that device current) and its compute-unit count.
int device_scratch(DeviceScratch &out, char *err, int32_t len)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return say(err, len, ORCA_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return say(err, len, ORCA_EINVAL, "device %d is beyond the %d this library serves", dev,
                   kMaxDevices);
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceScratch &d = g_dev[dev];
    if (!d.ptr) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return say(err, len, ORCA_EHIP, "hipGetSymbolAddress(scratch): %s",
                       hipGetErrorString(e));
        int cus = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess)
            return say(err, len, ORCA_EHIP, "hipDeviceGetAttribute: %s", hipGetErrorString(e));
        d.cus = cus > 0 ? cus : 256;
        d.ptr = (unsigned char *)ptr;
    }
    out = d;
    return ORCA_OK;
}

bool finite_pos(float v) { return isfinite(v) && v > 0.0f; }
bool finite_nonneg(float v) { return isfinite(v) && v >= 0.0f; }

}  // namespace
}  // namespace orca

extern "C" int orca_step_noalloc(int64_t n_agents, const orca_params *params, float *pos,
                                 float *vel, float *pref_vel, const float *goals, int32_t n_steps,
                                 void *hip_stream, char *err, int32_t err_len)
{
    using namespace orca;
    if (err && err_len > 0) err[0] = '\0';
    if (n_agents < 0 || n_agents > kNoAllocAgents)
        return say(err, err_len, ORCA_ECAPACITY,
                   "n_agents %lld is outside 0 .. %d, the scratch array's capacity",
                   (long long)n_agents, kNoAllocAgents);
    if (!params) return say(err, err_len, ORCA_EINVAL, "params must be non-NULL");
    const orca_params &q = *params;
    if (!finite_nonneg(q.radius) || !finite_pos(q.max_speed) || !finite_pos(q.neighbor_dist) ||
        !finite_pos(q.time_horizon) || !finite_pos(q.dt) || !finite_nonneg(q.pref_speed) ||
        q.reserved != 0)
        return say(err, err_len, ORCA_EINVAL,
                   "radius, pref_speed must be finite and >= 0; max_speed, neighbor_dist, "
                   "time_horizon, dt finite and > 0; reserved 0");
    if (q.max_neighbors < 0 || q.max_neighbors > kNoAllocK)
        return say(err, err_len, q.max_neighbors < 0 ? ORCA_EINVAL : ORCA_ECAPACITY,
                   "max_neighbors %d is outside 0 .. %d, the scratch array's capacity",
                   q.max_neighbors, kNoAllocK);
    if (n_steps < 1) return say(err, err_len, ORCA_EINVAL, "n_steps must be >= 1");
    if (n_agents > 0 && (!pos || !vel || !pref_vel))
        return say(err, err_len, ORCA_EINVAL, "pos, vel and pref_vel must be non-NULL");
    DeviceScratch ds;
    int rc = device_scratch(ds, err, err_len);
    if (rc != ORCA_OK) return rc;

    const hipStream_t st = (hipStream_t)hip_stream;
    unsigned char *base = ds.ptr;
    auto at = [base](size_t o) { return (void *)(base + o); };
    const int32_t n = (int32_t)n_agents;

    SceneDev p;
    p.radius = q.radius;
    p.vmax = q.max_speed;
    p.nd = q.neighbor_dist;
    p.tau = q.time_horizon;
    p.dt = q.dt;
    p.pref_speed = q.pref_speed;
    volatile float nd = q.neighbor_dist;
    p.nd2 = nd * nd;  // float32 product, as every distance test rounds it
    p.k = q.max_neighbors;

    Plan pl{};
    pl.n = n;
    pl.n_scenes = 1;
    pl.ld = kNoAllocAgents;
    pl.cus = ds.cus;
    pl.n_chunks = (n + kBboxChunk - 1) / kBboxChunk;
    // the launch shapes of a fresh context
    pl.knn_block = 256;
    pl.fb_waves_per_cu = 16;
    pl.vel_apl = 0;
    pl.vel_waves_per_cu = 12;
    pl.fb_work_units = 0;
    pl.max_cells = kNoAllocCells;
    const Layout &L = kLayout;
    pl.off = (const int32_t *)at(L.off);
    pl.sp = (const SceneDev *)at(L.sp);
    pl.agent_scene = (int32_t *)at(L.agent_scene);
    pl.bbox = (uint32_t *)at(L.bbox);
    pl.chunks = (const int2 *)at(L.chunks);
    pl.grid = (GridDev *)at(L.grid);
    pl.counters = (Counters *)at(L.counters);
    pl.key = (int32_t *)at(L.key);
    pl.rank = (int32_t *)at(L.rank);
    pl.counts = (int32_t *)at(L.counts);
    pl.cell_start = (int32_t *)at(L.cell_start);
    pl.partial = (uint32_t *)at(L.partial);
    pl.sorted = (float4 *)at(L.sorted);
    pl.sid = (int32_t *)at(L.sid);
    pl.inv = (int32_t *)at(L.inv);
    pl.nbr = (int32_t *)at(L.nbr);
    pl.ncount = (int32_t *)at(L.ncount);
    pl.kcap = kNoAllocK;
    pl.fb_list = (FallbackItem *)at(L.fb_list);
    pl.fb_key = (uint8_t *)at(L.fb_key);
    pl.fb_order = (int32_t *)at(L.fb_order);
    pl.stash_n = (double2 *)at(L.stash_n);
    pl.stash_b = (double *)at(L.stash_b);
    pl.out.pos = pos;
    pl.out.vel = vel;
    pl.out.pref = pref_vel;
    pl.out.goals = goals;
    pl.out.life.sp = pl.sp;
    pl.out.life.agent_scene = pl.agent_scene;
    pl.out.life.counters = pl.counters;

    auto hip = [&](hipError_t e, const char *where) {
        return e == hipSuccess ? ORCA_OK
                               : say(err, err_len, ORCA_EHIP, "%s: %s", where, hipGetErrorString(e));
    };
    const int32_t n_counts = (int32_t)kNoAllocCells + 1;
    hipLaunchKernelGGL(k_noalloc_setup, dim3((n_counts + 255) / 256), dim3(256), 0, st, p, n,
                       (int32_t *)at(L.off), (SceneDev *)at(L.sp), (int2 *)at(L.chunks),
                       pl.counts, n_counts, pl.counters);
    if ((rc = hip(hipGetLastError(), "k_noalloc_setup")) != ORCA_OK) return rc;
    if ((rc = hip(launch_scene_map(pl.off, 1, pl.agent_scene, n, pl.bbox, st), "scene map")) !=
        ORCA_OK)
        return rc;
    if (n == 0) return ORCA_OK;
    for (int32_t t = 0; t < n_steps; ++t) {
        if ((rc = hip(launch_grid(pl, pos, vel, true, st), "binning")) != ORCA_OK) return rc;
        if ((rc = hip(launch_knn(pl, p.k, st), "neighbours")) != ORCA_OK) return rc;
        if ((rc = hip(launch_lp(pl, p.k, st), "2D LP")) != ORCA_OK) return rc;
        if ((rc = hip(launch_fallback(pl, p.k, st), "fallback")) != ORCA_OK) return rc;
    }
    return ORCA_OK;
}
