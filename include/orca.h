/*
 * orca.h -- C ABI of the MI355X (gfx950) ORCA crowd step.
 *
 * One timestep of optimal reciprocal collision avoidance as described in
 * Charlton et al., "Fast Simulation of Crowd Collision Avoidance":
 *   - agents are binned into a uniform grid of square cells a half, a third
 *     or a quarter as wide as the observation radius (section 3, Fig. 2:
 *     messages sorted into spatial bins, each agent reading its own and the
 *     nearby bins);
 *   - each agent keeps the K nearest others closer than the observation
 *     radius (Fig. 2's radius filter; the cap K is the memory remedy of
 *     section 5);
 *   - each kept neighbour contributes one half-plane of permitted velocities
 *     (Fig. 1(b)-(c)): the velocity obstacle for look-ahead tau, the shortest
 *     vector u from the relative velocity to its boundary, and the half-plane
 *     through v + u/2 whose normal points along u -- each agent takes half of
 *     the avoidance (section 2 on reciprocal velocity obstacles);
 *   - a linear program picks the permitted velocity closest to the preferred
 *     one inside the max-speed disc (section 3); if no velocity is permitted
 *     it picks the one that least penetrates the half-planes (section 3),
 *     then, within 1e-5 m/s of that least penetration, the one closest to the
 *     preferred velocity;
 *   - every agent is updated from the same state, then x += dt v'.
 *   Pairs already closer than their combined radius use dt in place of tau
 *   (they must separate within one step).  Exact head-on pairs dodge to
 *   their own right; coincident pairs split along x by agent index.
 *
 * Memory and layout
 *   - Every state array is a caller-owned DEVICE pointer to float32 in
 *     structure-of-arrays form [2, N]: element i holds x_i (or vx_i), element
 *     N + i holds y_i (or vy_i).  The library never frees caller memory.
 *   - Scenes: n_scenes independent crowds stored back to back; scene s owns
 *     agents scene_offsets[s] .. scene_offsets[s+1]-1 (host array, n_scenes+1
 *     entries, first entry 0, non-decreasing, last entry N).  Agents of
 *     different scenes never see each other.  Neighbour ids are global
 *     agent indices.
 *   - The context owns all scratch memory: it is allocated once by
 *     orca_create, so orca_build_grid, orca_compute_velocities and orca_step
 *     allocate nothing.
 *   - Every call only enqueues work on the context's HIP stream and returns;
 *     outputs are ready when that stream reaches them.
 *
 * Errors
 *   Every call returns ORCA_OK (0) or a negative code; orca_last_error gives a
 *   message.  Arguments are validated on the host before anything is
 *   enqueued.  NaN or infinite values in device data are not checked: the
 *   results are then unspecified, but every access stays in bounds.
 *
 * Precision
 *   State is float32.  Neighbour distances are compared in float32 (squared
 *   distance, each operation rounded separately); half-planes and linear
 *   programs are solved in float64 and the results rounded to float32.
 *   Outputs are bitwise reproducible run to run.
 */
#ifndef ORCA_H
#define ORCA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORCA_OK = 0,
    ORCA_EINVAL = -1,    /* bad argument (null pointer, non-finite or out-of-range value) */
    ORCA_ENOMEM = -2,    /* device allocation failed in orca_create */
    ORCA_ECAPACITY = -3, /* more agents, scenes or neighbours than the context was made for */
    ORCA_ESTATE = -4,    /* call order: velocities without a grid of the same positions */
    ORCA_EHIP = -5       /* a HIP runtime call or kernel launch failed */
};

/* Largest neighbour cap a context accepts. */
#define ORCA_K_LIMIT 32

typedef struct orca_ctx orca_ctx;

/* Per-scene parameters (host memory).  All agents of a scene share them. */
typedef struct orca_params {
    float radius;          /* agent radius r (m), >= 0; a pair's combined radius is 2r */
    float max_speed;       /* v_max (m/s), > 0: the velocity disc */
    float neighbor_dist;   /* observation radius (m), > 0; neighbours are strictly closer */
    float time_horizon;    /* look-ahead tau (s), > 0 */
    float dt;              /* time step (s), > 0 */
    float pref_speed;      /* walking speed for goal steering (m/s), >= 0 */
    int32_t max_neighbors; /* K, 0 .. the context's k_max */
    int32_t reserved;      /* must be 0 */
} orca_params;

/*
 * Create a context for up to max_agents agents in up to max_scenes scenes
 * with neighbour caps up to k_max (1 .. ORCA_K_LIMIT).  tape_steps reserves
 * room for that many recorded steps for orca_backward (0 = no tape).
 * hip_stream is a hipStream_t (NULL = the null stream) on the current device.
 * On success *out owns all device scratch; release it with orca_destroy.
 * Errors: EINVAL (out == NULL, sizes out of range), ECAPACITY (k_max above
 * ORCA_K_LIMIT), ENOMEM, EHIP.  On error *out is NULL.
 */
int orca_create(orca_ctx **out, int64_t max_agents, int32_t max_scenes, int32_t k_max,
                int32_t tape_steps, void *hip_stream);

/* Release a context (waits for its stream first).  NULL is ignored. */
void orca_destroy(orca_ctx *ctx);

/* Message of the last failed call on ctx (static text if ctx is NULL). */
const char *orca_last_error(const orca_ctx *ctx);

/* Make later calls enqueue on another stream of the same device. */
int orca_set_stream(orca_ctx *ctx, void *hip_stream);

/*
 * Bin the agents (section 3, Fig. 2).  pos: device [2, N] with
 * N = scene_offsets[n_scenes].  Per scene: bounding box, cells of side
 * neighbor_dist * (1 + 2^-10) / c with c = 2, 3 or 4 chosen from the
 * scene's mean density and K (so the 3 x 3 cells around an agent hold about
 * 2.75 K agents; a neighbour search reads the cells within c of its own),
 * wider cells if the context's cell budget would be exceeded, cell keys, a
 * counting sort of the agents into cell order.
 * The grid stays valid for orca_compute_velocities on the same pos pointer
 * until orca_step or another orca_build_grid.
 * Errors: EINVAL, ECAPACITY (N > max_agents, n_scenes > max_scenes,
 * max_neighbors > k_max), EHIP.
 */
int orca_build_grid(orca_ctx *ctx, int32_t n_scenes, const int64_t *scene_offsets,
                    const orca_params *params, const float *pos);

/*
 * New velocities from one state, without moving anyone (sections 3 and 5).
 * pos must be the pointer given to the last orca_build_grid (else ESTATE).
 * vel: current velocities [2, N].  Preferred velocities: if goals (device
 * [2, N]) is non-NULL each agent's preferred velocity points at its goal at
 * pref_speed (or covers the remaining offset in one dt when closer than
 * pref_speed * dt), else pref_vel [2, N] is used as given.
 * Outputs (original agent order):
 *   new_vel   [2, N] float32, required;
 *   nbr_out   [N, K_s] int32 per scene block (row i has K of agent i's scene
 *             entries: neighbour ids nearest first, ties by id, padded with
 *             -1); the rows are packed with stride k_row = max over scenes of
 *             max_neighbors; NULL to skip;
 *   lp_status [N] uint8: 0 = the 2D program was feasible, 1 = least
 *             penetration fallback, 2 = absent (spawning and removal: not
 *             yet spawned or removed; its new_vel is 0 and its nbr_out row
 *             all -1); NULL to skip.
 */
int orca_compute_velocities(orca_ctx *ctx, const float *pos, const float *vel,
                            const float *pref_vel, const float *goals, float *new_vel,
                            int32_t *nbr_out, uint8_t *lp_status);

/*
 * Advance n_steps (>= 1) synchronous steps in place.  Each step bins the
 * agents, picks every new velocity v' from the same state, then sets
 * x <- x + dt v' and v <- v' (float32 results of float64 sums).  With goals
 * (device [2, N], nullable) the preferred velocity is re-aimed at the goal at
 * the start of every step and written to pref_vel; without, pref_vel is read
 * only.  save_tape = 1 records the steps for orca_backward (needs tape_steps
 * >= n_steps at create); 0 records nothing.
 */
int orca_step(orca_ctx *ctx, int32_t n_scenes, const int64_t *scene_offsets,
              const orca_params *params, float *pos, float *vel, float *pref_vel,
              const float *goals, int32_t n_steps, int32_t save_tape);

/*
 * orca_step for many steps at the lowest launch cost: the first call captures
 * one whole step (every kernel of every scene; no host synchronisation and no
 * memory set nodes inside) into a HIP graph on a private capture stream, and
 * every step replays that graph on the context stream.  For 10 or more steps
 * without spawning and removal it also captures a block of 10 steps that, as
 * orca_step does, keeps the state in cell order between its steps; n_steps
 * then replays n_steps / 10 blocks and the rest one step at a time (the same
 * results bit for bit).  The graphs are captured again when pos / vel /
 * pref_vel / goals, the scene set or the launch shapes change.  A capture
 * waits for the context stream once.  Not available while profiling is on
 * (ESTATE).  No tape is recorded.
 */
int orca_step_graph(orca_ctx *ctx, int32_t n_scenes, const int64_t *scene_offsets,
                    const orca_params *params, float *pos, float *vel, float *pref_vel,
                    const float *goals, int32_t n_steps);

/*
 * Pick the launch shapes for the current workload by timing velocity passes
 * with HIP events (per candidate one untimed pass, then the fastest of reps
 * passes for each stage):
 *   - threads per neighbour block (64, 128, 256, 512) and persistent
 *     fallback waves per compute unit (4, 8, 16, 32, i.e. how many fallback
 *     agents each lane takes on);
 *   - the velocity kernels (see orca_set_kernels): the split neighbour and
 *     LP kernels, or the fused persistent kernel with 1, 2 or 4 agents per
 *     lane and 8 or 12 waves per compute unit, whichever runs the neighbour
 *     and LP stages fastest;
 *   - the fallback with or without work units (with: 6 waves per compute
 *     unit; neighbour caps up to 16).
 * Needs orca_build_grid on pos first; writes only new_vel (device [2, N],
 * scratch).  The choice is kept in the context and returned in choice[5]
 * (nullable): knn_block, fallback waves per CU, agents per lane (0 = split
 * kernels), velocity waves per CU, fallback work units (0 or 1).  Waits for
 * the stream.
 */
int orca_autotune(orca_ctx *ctx, const float *pos, const float *vel, const float *pref_vel,
                  const float *goals, float *new_vel, int32_t reps, int32_t *choice);

/*
 * Optional per-agent properties (section 4: people of different sizes and
 * speeds): device float32 arrays of at least N entries in agent order, each
 * nullable (NULL: the scene's radius / max_speed / pref_speed).  A pair's
 * combined radius is r_i + r_j; max_speed caps the agent's own velocity;
 * pref_speed is its walking speed toward its goal.  The context keeps the
 * pointers (the caller keeps the arrays alive and unchanged) and applies them
 * to every later orca_build_grid, orca_compute_velocities, orca_step and
 * orca_step_graph until set again; orca_compute_velocities returns ESTATE if
 * the radii changed since orca_build_grid.  orca_backward uses the radii and
 * max speeds of the recorded steps; an agent with its own max speed adds
 * nothing to its scene's max_speed gradient.  Errors: EINVAL (ctx NULL).
 */
int orca_set_agents(orca_ctx *ctx, const float *radius, const float *max_speed,
                    const float *pref_speed);

/*
 * Spawning and removal (section 4: crossings where people enter over time
 * and leave at their goal).  spawn_step: device int32 [N], the step index at
 * which each agent enters; state: device uint8 [N], 0 = not removed, 1 =
 * removed, read and written by the kernels.  At step index t an agent takes
 * part (is binned, seen as a neighbour, steered and moved) iff
 * spawn_step[i] <= t and state[i] == 0; absent agents keep their position
 * and velocity.  After each step's Euler update an agent whose goal lies
 * within its own radius of its new float32 position (|g - x|^2 <= r^2 in
 * float64) gets state 1.  The step index lives on the device: this call sets
 * it to t0 and every orca_step / orca_step_graph step advances it by one
 * (orca_build_grid evaluates presence at the current index without
 * advancing), so graph replays need no host round trip.  Both NULL turns the
 * feature off.  The context keeps the pointers (the caller keeps the arrays
 * alive); orca_step and orca_step_graph then need goals, and recorded steps
 * (save_tape) are refused.  Waits for the stream.  Errors: EINVAL (ctx NULL,
 * exactly one of the arrays NULL, or later: a step without goals or with
 * save_tape), ESTATE (profiling on).
 */
int orca_set_lifecycle(orca_ctx *ctx, const int32_t *spawn_step, uint8_t *state, int32_t t0);

/*
 * Read the spawning and removal counters (waits for the stream): *step = the
 * step index the next step evaluates presence at, *present = agents present
 * at the last binning (-1 if none has run since orca_set_lifecycle; N when
 * the feature is off), *removed = agents whose state is 1 (counted by a small
 * kernel on the context stream for this call; 0 when the feature is off).
 * Each output is nullable.  Errors: EINVAL (ctx NULL), EHIP.
 */
int orca_population(orca_ctx *ctx, int32_t *step, int64_t *present, int64_t *removed);

/*
 * Set the launch shapes directly (the two values orca_autotune picks):
 * knn_block in {64, 128, 256, 512} threads per neighbour block and
 * fb_waves_per_cu in 1..64 persistent fallback waves per compute unit.
 * Results do not depend on them.  Errors: EINVAL.
 */
int orca_set_launch(orca_ctx *ctx, int32_t knn_block, int32_t fb_waves_per_cu);

/*
 * Select kernel variants (results do not depend on them).
 * agents_per_lane: 0 runs the neighbour search and the half-planes + 2D LP
 *   (section 3) as two kernels with the neighbour lists stored in between
 *   (the default); 1, 2 or 4 runs both in one persistent kernel with each
 *   agent's neighbour list in registers: its one-wave blocks
 *   (velocity_waves_per_cu per compute unit, 1..32) take tiles of
 *   64 * agents_per_lane agents in cell order from one atomic queue per XCD
 *   (the XCD's contiguous share of the tiles, then the others' once its own
 *   is empty).  Plain passes only: recorded steps and steps with spawning
 *   and removal use the two kernels.
 * fallback_work_units: 1 runs the least-penetration fallback with work units
 *   (section 3: the recompute of a new velocity cut into equal pieces that
 *   idle threads take over; here the 1D programs on violated lines of the
 *   plane subproblems, split across groups of 4 lanes); 0 (the default) has
 *   each lane run its own.  Used for neighbour caps up to 16.
 * Errors: EINVAL.
 */
int orca_set_kernels(orca_ctx *ctx, int32_t agents_per_lane, int32_t velocity_waves_per_cu,
                     int32_t fallback_work_units);

/*
 * Vector-Jacobian product of recorded step tape_step (0-based, of the last
 * orca_step call with save_tape = 1; no goals).  Given the gradients of a loss
 * with respect to the state after the step (g_pos_next, g_vel_next, device
 * [2, N]), write the gradients with respect to the state before it (g_pos,
 * g_vel, device [2, N], overwritten) and ADD the gradients with respect to
 * the fixed preferred velocities (g_pref_vel [2, N]), each scene's max_speed
 * (g_max_speed [n_scenes]) and time_horizon (g_time_horizon [n_scenes]).
 * The discrete choices of the forward step (neighbour sets, half-plane
 * branches, active constraints) are held fixed.
 * Errors: EINVAL, ESTATE (no such recorded step), EHIP.
 */
int orca_backward(orca_ctx *ctx, int32_t tape_step, const float *g_pos_next,
                  const float *g_vel_next, float *g_pos, float *g_vel, float *g_pref_vel,
                  float *g_max_speed, float *g_time_horizon);

/*
 * orca_backward over the recorded steps last, last - 1, ..., first (0 <=
 * first <= last < the number of recorded steps): g_pos_next / g_vel_next are
 * the gradients after step last, g_pos / g_vel receive those before step
 * first, and the preferred-velocity, max_speed and time_horizon gradients of
 * every step are ADDED as orca_backward adds them.  The same products as
 * calling orca_backward for each step in turn (equal to float32 rounding of
 * the accumulation order): between the steps the gradients stay in the
 * context, one 16-byte entry per agent, so each step reads and writes one
 * line per agent instead of one per component.  The output arrays may be the
 * input arrays.  Errors: EINVAL, ESTATE (no such recorded steps), EHIP.
 */
int orca_backward_steps(orca_ctx *ctx, int32_t first, int32_t last, const float *g_pos_next,
                        const float *g_vel_next, float *g_pos, float *g_vel, float *g_pref_vel,
                        float *g_max_speed, float *g_time_horizon);

/*
 * Diagnostics: per-stage GPU time of every pass (orca_compute_velocities, or
 * one step of orca_step) measured with HIP events recorded on the context
 * stream between the stages.  Stages:
 *   0 binning (bounding box, keys, scan, scatter; 0 for orca_compute_velocities),
 *   1 neighbour gather, 2 half-planes + 2D LP, 3 least-penetration fallback.
 * orca_profile(ctx, 1) clears the sums and starts with each pass waiting for
 * its stream at the end (so the sums are always current); orca_profile(ctx,
 * 2) clears them and starts without waiting: the events of the first 1024
 * passes are recorded and the fallback agents counted on the device, and
 * orca_profile_read waits for the stream and sums them (use it around timed
 * work).  orca_profile(ctx, 0) stops.  orca_profile_read gives the summed
 * milliseconds per stage (stage_ms [ORCA_PROF_STAGES]), the number of passes,
 * and the total number of agents that took the fallback in them.
 */
#define ORCA_PROF_STAGES 4
int orca_profile(orca_ctx *ctx, int32_t enable);
int orca_profile_read(orca_ctx *ctx, double *stage_ms, int64_t *passes, int64_t *fallback_agents);

/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * orca_step for ONE scene of n_agents agents without a context: the same
 * kernels and results as orca_step on a fresh context (default launch
 * shapes, no tape, no per-agent properties, no spawning), with every scratch
 * buffer in a file-scope device array of ORCA_NOALLOC_SCRATCH_BYTES (about
 * 9.2 MiB) that each device the library runs on holds until the process
 * ends.  It calls no hipMalloc, hipFree or allocating library routine and
 * enqueues kernels only (no memset or copy nodes), so it can be captured.
 *   n_agents: 0 .. ORCA_NOALLOC_MAX_AGENTS; params: host, one scene with
 *   max_neighbors 0 .. ORCA_NOALLOC_MAX_NEIGHBORS; pos, vel, pref_vel,
 *   goals (nullable): caller-owned device [2, N] as for orca_step (goals
 *   given: pref_vel is overwritten with the steered preferred velocity);
 *   n_steps >= 1; hip_stream: a hipStream_t of the CURRENT device (NULL =
 *   null stream); err: nullable host buffer of err_len bytes for a message.
 * Every call on a device shares that device's array, which keeps the last
 * call's contents (each call clears what must start at zero): calls that
 * overlap on one device (other streams, other threads) race and must be
 * serialised by the caller.
 * Errors: ECAPACITY (n_agents or max_neighbors above the maximum), EINVAL,
 * EHIP.  Nothing is enqueued when the arguments are rejected.
 */
#define ORCA_NOALLOC_MAX_AGENTS 16384
#define ORCA_NOALLOC_MAX_NEIGHBORS 16
#define ORCA_NOALLOC_SCRATCH_BYTES 9685760
int orca_step_noalloc(int64_t n_agents, const orca_params *params, float *pos, float *vel,
                      float *pref_vel, const float *goals, int32_t n_steps, void *hip_stream,
                      char *err, int32_t err_len);

#ifdef __cplusplus
}
#endif

#endif /* ORCA_H */
