/*
 * mppi_jump.h - C ABI of the MI355X (gfx950) library for one iteration of
 * model predictive path-integral control on a jump-diffusion process
 * (Wang, Williams, Theodorou, "Information Theoretic Model Predictive
 * Control on Jump Diffusion Processes", arXiv 1807.06108).
 *
 * One iteration (Algorithm 1 of the paper) is:
 *   1. sample K perturbed control sequences: Gaussian noise plus
 *      compound-Poisson jumps (Sec. IV-B noise model, Algorithm 1 jump timer);
 *   2. roll out the K trajectories of the dynamics in parallel with explicit
 *      Euler steps and accumulate the modified path costs S~_k (eqs. (34)-(35));
 *   3. weights w_k = exp(-(S~_k - min S~)/lambda) / sum (eq. (37));
 *   4. U += alpha * sum_k w_k eps_k (eq. (36); step alpha of eq. (49)).
 * Between control steps the sequence is shifted: u_0 is executed, U moves one
 * step left and u_init is appended (Algorithm 1, Sec. V).
 *
 * Conventions shared by every entry point
 *   - All device pointers are plain device addresses (or, where stated,
 *     pinned host addresses that the device can access).  The caller owns
 *     all device memory; the library never allocates device memory and never
 *     synchronises a stream, except where an entry point says so.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Every entry point that takes a stream only enqueues work on it.
 *   - Every function returns an int status (MPPI_OK or a negative code); no
 *     C++ exception crosses this interface and the library never aborts.
 *     mppi_jump_last_error() gives a human-readable detail for the calling
 *     thread's last failure.
 *   - A context is not thread-safe; distinct contexts on distinct streams are
 *     independent.
 */
#ifndef MPPI_JUMP_H
#define MPPI_JUMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPPI_JUMP_ABI_VERSION 4

#define MPPI_JUMP_MAX_N 12      /* state dimension bound            */
#define MPPI_JUMP_MAX_M 4       /* control dimension bound          */
#define MPPI_JUMP_MAX_Q 3       /* jump-mark dimension bound        */
#define MPPI_JUMP_MAX_LEVELS 32 /* count-law inversion levels       */
#define MPPI_JUMP_MAX_K (1 << 24)
#define MPPI_JUMP_MAX_T 4096

/* status codes */
#define MPPI_OK 0
#define MPPI_EINVAL -1        /* invalid argument or configuration          */
#define MPPI_EWORKSPACE -2    /* workspace too small or misaligned          */
#define MPPI_EDEVICE -3       /* a HIP runtime call failed                  */
#define MPPI_ENONFINITE -4    /* every S~_k was non-finite; U left unchanged */
#define MPPI_EUNSUPPORTED -5  /* valid request this build does not support  */

/* dynamics ids: (n, m, q) = state, control and jump-mark dimensions */
#define MPPI_DYN_LINEAR 0     /* double integrator, (2, 1, 1)  */
#define MPPI_DYN_CARTPOLE 1   /* cartpole, (4, 1, 1)           */
#define MPPI_DYN_QUADROTOR 2  /* 12-state quadrotor, (12, 4, 3) */

/* jump count law (Sec. IV-B): Poisson(nu dt) or the zero-one law */
#define MPPI_COUNT_POISSON 0
#define MPPI_COUNT_ZERO_ONE 1

/* jump-mark law (Sec. II: the marks of the compound-Poisson process are
 * normal, N(0, diag sigma_J^2) per jump) */
#define MPPI_MARK_NORMAL 0

/* path-cost form: information-theoretic (eqs. (34)-(35), with the
 * importance-sampling terms) or stochastic-optimisation (Sec. IV: cost on the
 * applied control, no importance-sampling term) */
#define MPPI_COST_IT 0
#define MPPI_COST_SO 1

/* rollout schedules (identical results, different parallel decomposition):
 * one sample per lane, 256 samples per workgroup; or wave-specialised, 64
 * samples per workgroup of 8 wavefronts (7 draw noise, 1 runs the state
 * recursion), for latency when K does not fill the GPU.  AUTO picks
 * wave-specialised for K <= MPPI_JUMP_WS_MAX_K, or K <=
 * MPPI_JUMP_WS_MAX_K_MULTI for a model with several control channels (the
 * quadrotor: its heavier draws make the one-sample-per-lane schedule the
 * faster one sooner). */
#define MPPI_SCHED_AUTO 0
#define MPPI_SCHED_LANE 1
#define MPPI_SCHED_WAVE_SPECIALISED 2
#define MPPI_JUMP_WS_MAX_K 131072
#define MPPI_JUMP_WS_MAX_K_MULTI 98304

/* items of mppi_jump_get / mppi_jump_set */
#define MPPI_ITEM_U 0        /* float [T][m]                        get, set */
#define MPPI_ITEM_S 1        /* double [K] path costs S~_k          get, set */
#define MPPI_ITEM_W 2        /* double [K] normalised weights       get      */
#define MPPI_ITEM_STATS 3    /* mppi_jump_stats                     get      */
#define MPPI_ITEM_EPS 4      /* float [T][m][K] perturbations       get; see below */
#define MPPI_ITEM_DBG_ZD 5   /* float [K][T][m] standard normals z_D  (debug_dump) */
#define MPPI_ITEM_DBG_N 6    /* int32 [K][T] jump counts              (debug_dump) */
#define MPPI_ITEM_DBG_ZJ 7   /* float [K][T][q] standard normals z_J  (debug_dump) */
#define MPPI_ITEM_THRESH 8   /* uint64 [MPPI_JUMP_MAX_LEVELS] count thresholds; unused = 2^32 */

/*
 * Configuration: the "Given" block of Algorithm 1.  All floats are fp32.
 * Noise parameters are per-step control-space values: the sampled control is
 * U[t] + eps[k][t] with eps = sigma * z_D (+ a control-channel jump).
 */
typedef struct mppi_jump_config {
  int32_t abi_version;   /* must equal MPPI_JUMP_ABI_VERSION                   */
  int32_t dynamics;      /* MPPI_DYN_*                                         */
  int32_t K;             /* samples per iteration, 1..MPPI_JUMP_MAX_K          */
  int32_t T;             /* horizon steps, 1..MPPI_JUMP_MAX_T                  */
  float dt;              /* step length (s), > 0                               */
  float lambda;          /* temperature, > 0                                   */
  float alpha;           /* update step size (eq. (49)); 1 = Algorithm 1       */
  float c;               /* importance-sampling variance factor (eq. (35)), >0 */
  float nu;              /* jump rate (1/s), >= 0; count mean is nu*dt         */
  int32_t count_law;     /* MPPI_COUNT_*                                       */
  int32_t cost_form;     /* MPPI_COST_*                                        */
  int32_t debug_dump;    /* 1: also write z_D, N, z_J for every (k, t)         */
  float sigma[4];        /* Gaussian std per control channel, >= 0             */
  float sigma_J[4];      /* jump-mark std per mark channel, >= 0               */
  float u_init[4];       /* value appended by the shift                         */
  float R[4];            /* diagonal control cost (eq. (3))                    */
  float Q[12];           /* diagonal running state cost                        */
  float Qf[12];          /* diagonal terminal state cost                       */
  float x_goal[12];      /* target state x*                                    */
  float params[12];      /* dynamics constants (see below)                     */
  float crash_penalty;   /* quadrotor crash indicator weight                   */
  int32_t schedule;      /* MPPI_SCHED_*: rollout work split (same results)    */
  uint64_t seed;         /* Philox key                                         */
  uint64_t controller_id;/* < 2^24; part of the Philox counter                 */
  uint64_t start_iteration; /* iteration index of the first step, < 2^32      */
  int32_t full_sigma;    /* 0: Sigma_D = diag(sigma^2); 1: Sigma_D = L L^T     */
  float sigma_L[16];     /* full_sigma: Cholesky factor L of Sigma_D (Sec. IV-B
                            eps_D ~ N(0, Sigma_D)), row-major 4 x 4 of which
                            the leading m x m block is used: lower triangular,
                            diagonal > 0; sigma[] is then ignored            */
  int32_t sample_offset; /* global index of this controller's first sample:
                            sample k draws the noise of sample_offset + k, so
                            controllers with disjoint offsets are shards of
                            one larger sample set; >= 0, offset + K <= 2^31  */
  int32_t mark_law;      /* MPPI_MARK_*: distribution of a jump's mark          */
} mppi_jump_config;
/* params: cartpole  = {m_cart, m_pole, half_length, g}
 *         quadrotor = {mass, Jx, Jy, Jz, arm, k_yaw, g, tilt_max, z_min}
 *         linear    = unused                                                 */

typedef struct mppi_jump_stats {
  double rho;            /* min over finite S~_k                              */
  double eta;            /* sum_k exp(-(S~_k - rho)/lambda)                   */
  int32_t status;        /* MPPI_OK or MPPI_ENONFINITE of the last iteration  */
  int32_t n_finite;      /* number of finite S~_k                             */
  uint64_t iteration;    /* index of the next iteration                       */
} mppi_jump_stats;

typedef struct mppi_jump_ctx mppi_jump_ctx;

/* ABI version of the loaded library (MPPI_JUMP_ABI_VERSION). */
int mppi_jump_abi_version(void);

/* State, control and jump-mark dimensions of a dynamics id.
 * Pure host function.  EINVAL for an unknown id or NULL output. */
int mppi_jump_dims(int32_t dynamics, int32_t* n, int32_t* m, int32_t* q);

/* Device workspace a configuration needs (perturbations [T][m][K],
 * costs [K], reduction partials, statistics, control sequence, optional debug
 * dumps), in bytes, for a 256-byte aligned base.  Pure host function: it
 * validates the configuration and returns EINVAL for any invalid field. */
int mppi_jump_workspace_bytes(const mppi_jump_config* cfg, size_t* bytes);

/* Jump-count inversion table of a configuration (Sec. IV-B count law with
 * mean nu*dt): out[0..MPPI_JUMP_MAX_LEVELS) receives theta_j = floor(F(j) 2^32)
 * with F the CDF of the count law; entries from the closing level on are
 * 2^32.  The count drawn from a 32-bit word w is the number of j with
 * w >= theta_j.  Pure host function; EINVAL for an invalid configuration. */
int mppi_jump_count_thresholds(const mppi_jump_config* cfg, uint64_t* out);

/* Validate cfg, lay the caller's workspace out and enqueue its
 * initialisation on `stream`: U <- d_U0 ([T][m] fp32, read during this
 * enqueue's execution; NULL = u_init at every step), iteration counter <-
 * start_iteration.  Allocates only the host-side context (*out).
 * EWORKSPACE if ws_bytes is below mppi_jump_workspace_bytes or d_workspace
 * is not 256-byte aligned. */
int mppi_jump_init(const mppi_jump_config* cfg, void* d_workspace, size_t ws_bytes,
                   const float* d_U0, void* stream, mppi_jump_ctx** out);

/* Enqueue `iters` >= 1 iterations (Algorithm 1, sampling to update) from
 * the state d_x0 ([n] fp32 device), updating U in place.  Each iteration
 * draws fresh noise (its own iteration index).  If every S~_k of an
 * iteration is non-finite, that iteration leaves U unchanged and records
 * MPPI_ENONFINITE in the statistics (read with MPPI_ITEM_STATS).
 * With at most 256 rollout workgroups (wave-specialised schedule) or 64
 * (one sample per lane) the update of eqs. (36)-(37) runs in the rollout
 * kernel's epilogue (one kernel per iteration).  Beyond that,
 * each workgroup's epilogue publishes its weighted perturbation sums and a
 * second kernel combines them; a context with debug_dump runs the staged
 * pair (mppi_jump_rollout, mppi_jump_update) instead. */
int mppi_jump_step(mppi_jump_ctx* ctx, const float* d_x0, int32_t iters, void* stream);

/* One MPC control step (Algorithm 1 loop body, Sec. V): `iters` >= 1
 * iterations from d_x0 followed by the receding-horizon shift, with u_0 (the
 * control to execute, [m] fp32) written to d_u0_out (device memory; may be
 * NULL).  Equivalent to mppi_jump_step then mppi_jump_shift; when the
 * update is applied inside the rollout kernel (see mppi_jump_step) the
 * shift and the u_0 output are folded into the last iteration's kernel. */
int mppi_jump_control_step(mppi_jump_ctx* ctx, const float* d_x0, int32_t iters,
                           float* d_u0_out, void* stream);


/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one MPC
 * control step exactly as mppi_jump_control_step (same kernels, same
 * results) without a context or a caller workspace.  The scratch (costs,
 * perturbations, partials, statistics, counters) lives in a library-owned
 * static device array of MPPI_JUMP_STATIC_SCRATCH_BYTES per GPU, held until
 * the process ends; a configuration whose mppi_jump_workspace_bytes exceeds
 * it is refused with MPPI_EWORKSPACE.  The caller passes cfg (validated as
 * by mppi_jump_init; debug_dump must be 0, else MPPI_EUNSUPPORTED), the
 * control sequence d_U ([T][m] fp32 device memory, updated in place and
 * shifted), the state d_x0 ([n] fp32 device) and d_u0_out ([m] fp32 device,
 * may be NULL).  Iteration indices (the noise stream position) run from
 * cfg->start_iteration; a caller continuing a controller passes
 * start_iteration + iters on its next call.  Nothing is allocated: no
 * hipMalloc, no hipFree, no host heap.  The first call on a device resolves
 * the array's device address (hipGetSymbolAddress), so make one call
 * outside graph capture first.  Every call on one GPU shares that GPU's
 * array and leaves its contents behind (each call re-initialises what must
 * start at zero): calls that overlap on one GPU, on different streams or
 * threads, race and give undefined results. */
#define MPPI_JUMP_STATIC_SCRATCH_BYTES (16 << 20)
int mppi_jump_control_step_static(const mppi_jump_config* cfg, float* d_U, const float* d_x0,
                                  int32_t iters, float* d_u0_out, void* stream);

/* The two halves of one iteration, for callers that stage it:
 * rollout = sampling, propagation and path costs (fills S and eps, and the
 * min / normaliser statistics); update = weights and control update (reads
 * S and eps, updates U, advances the iteration counter).  step == rollout
 * followed by update. */
int mppi_jump_rollout(mppi_jump_ctx* ctx, const float* d_x0, void* stream);
int mppi_jump_update(mppi_jump_ctx* ctx, void* stream);

/* Enqueue the receding-horizon shift (Algorithm 1, after the update):
 * u0_out[0..m) <- U[0] by a stream-ordered copy (device or host memory; may
 * be NULL; a host destination is complete once the stream is synchronised),
 * then U[t] <- U[t+1] and U[T-1] <- u_init. */
int mppi_jump_shift(mppi_jump_ctx* ctx, float* u0_out, void* stream);

/* Enqueue a copy of an item (MPPI_ITEM_*) into dst (device or host memory).
 * EINVAL if dst_bytes is smaller than the item; EUNSUPPORTED for a debug
 * item of a context created without debug_dump, and for MPPI_ITEM_EPS after
 * an iteration that kept its perturbations on chip: the wave-specialised
 * iteration of mppi_jump_step / mppi_jump_control_step (without debug_dump)
 * holds its tile of perturbations in LDS until its weighted sums are formed
 * and never stores them, when the tile fits (T <= 496 for the one-channel
 * models, T <= 108 for the quadrotor);
 * every staged rollout (mppi_jump_rollout), unfused or lane-schedule
 * iteration, batch step and pool tick stores them.  MPPI_ITEM_W and
 * MPPI_ITEM_THRESH are computed at call time (W from the current S and
 * statistics).  A host dst is complete only after the stream is synchronised. */
int mppi_jump_get(mppi_jump_ctx* ctx, int32_t what, void* dst, size_t dst_bytes, void* stream);

/* Enqueue an overwrite of MPPI_ITEM_U ([T][m] fp32) or MPPI_ITEM_S ([K]
 * fp64, with the min / normaliser statistics recomputed from it) from src
 * (device or host).  Setting S between rollout and update lets a caller
 * supply its own path costs to the update. */
int mppi_jump_set(mppi_jump_ctx* ctx, int32_t what, const void* src, size_t src_bytes, void* stream);

/* Free the host-side context.  The caller frees the workspace after the
 * last enqueued work on it has finished. */
int mppi_jump_destroy(mppi_jump_ctx* ctx);

/* Static text for a status code; never NULL. */
const char* mppi_jump_strerror(int code);

/* Detail of the calling thread's last failure ("" if none). */
const char* mppi_jump_last_error(void);

/* ---- batched form: many controllers advanced by one launch ----
 * A batch groups contexts created with the same rollout schedule (each
 * whose own iteration is fused, see mppi_jump_step, and without debug_dump)
 * and advances all of them by one iteration per kernel launch: one grid
 * over every controller's tiles, longest first, driven by a device table of
 * their parameters and buffers.  Each controller keeps its own workspace,
 * iteration counter and noise stream, so a batched iteration gives exactly
 * the results of mppi_jump_step / mppi_jump_control_step on that controller
 * alone.  The tables are built once at creation; step calls take no
 * pointers and can be captured in a HIP graph and replayed. */
typedef struct mppi_jump_batch mppi_jump_batch;

/* Device scratch for a batch of n contexts (descriptor table, tile list,
 * u_0 outputs [n][4] fp32, work queue), for a 256-byte aligned base.  Pure host function.
 * EINVAL for NULL/mixed-schedule contexts; EUNSUPPORTED for a context whose
 * own iteration is not fused (more rollout workgroups than mppi_jump_step
 * fuses) or that has debug_dump set. */
int mppi_jump_batch_scratch_bytes(mppi_jump_ctx* const* ctxs, int32_t n, size_t* bytes);

/* Build a batch over ctxs[0..n) with states d_x0[i] ([n_i] fp32 device
 * pointers, read at every step); uploads the tables on `stream` and
 * synchronises it.  The caller keeps the contexts and the scratch alive for
 * the life of the batch. */
int mppi_jump_batch_create(mppi_jump_ctx* const* ctxs, const float* const* d_x0, int32_t n,
                           void* d_scratch, size_t scratch_bytes, void* stream,
                           mppi_jump_batch** out);

/* Enqueue `iters` iterations of every controller of the batch (one launch
 * per iteration); with shift != 0 the last one also shifts every sequence
 * and writes each controller's u_0 to its slot of the u_0 output array. */
int mppi_jump_batch_step(mppi_jump_batch* batch, int32_t iters, int32_t shift, void* stream);

/* Launch form of mppi_jump_batch_step (the same results either way):
 * MPPI_BATCH_GRID (the default) launches one workgroup per tile and lets the
 * hardware dispatcher start them in the longest-first order of the tile
 * list; MPPI_BATCH_PERSISTENT launches as many workgroups as the GPU holds at
 * once (the kernel's occupancy times the compute units), each taking the next
 * tile from a device work queue in the batch scratch until none is left.
 * EINVAL for another value; EDEVICE if the occupancy query fails. */
#define MPPI_BATCH_GRID 0
#define MPPI_BATCH_PERSISTENT 1
int mppi_jump_batch_set_launch(mppi_jump_batch* batch, int32_t launch);

/* Device address of the u_0 outputs, [n][4] fp32 (controller i at 4*i). */
int mppi_jump_batch_u0(mppi_jump_batch* batch, float** d_u0);

/* Free the host-side batch object. */
int mppi_jump_batch_destroy(mppi_jump_batch* batch);

/* ---- serving form: ticks over a resident pool ----
 *
 * A pool holds n contexts resident (each with its own workspace, U,
 * iteration counter and noise stream; the same conditions as a batch) and
 * advances any subset of them per tick: one MPC step per request (iters
 * iterations of Algorithm 1 from the request's state, then the shift), all
 * requests of a tick in one grid per iteration, longest first.  A request's
 * result depends only on its controller's own sequence of requests, never on
 * which other requests share its tick.
 *
 * A tick is staged through one of max_inflight slots: the host writes the
 * request record to the slot's part of the caller's pinned staging, the tick
 * uploads it, runs, and copies u_0 (and the plant's next state) back to the
 * staging; results are taken with mppi_jump_pool_results once the tick has
 * finished.  Ticks on different slots may be in flight together on different
 * streams; a controller may belong to one tick in flight at a time and a
 * slot holds one tick until its results are taken (both are checked: EINVAL).
 * Calls on one pool are not thread-safe.  While a context belongs to a pool,
 * the caller must not run it through other entry points concurrently. */
typedef struct mppi_jump_pool mppi_jump_pool;

#define MPPI_JUMP_POOL_MAX_INFLIGHT 16

/* Sizes for a pool over ctxs[0..n) with max_inflight slots: device scratch
 * (descriptor table and per-slot request records) and pinned host staging,
 * both for 256-byte aligned bases.  Pure host function.  Same context
 * conditions as mppi_jump_batch_scratch_bytes; EINVAL for max_inflight out
 * of [1, MPPI_JUMP_POOL_MAX_INFLIGHT]. */
int mppi_jump_pool_bytes(mppi_jump_ctx* const* ctxs, int32_t n, int32_t max_inflight,
                         size_t* device_bytes, size_t* pinned_host_bytes);

/* Build a pool: uploads the descriptor table on `stream`, synchronises it,
 * and zeroes the staging.  d_scratch is device memory, h_pinned is
 * page-locked host memory (e.g. hipHostMalloc); the caller owns both and the
 * contexts and keeps them alive for the life of the pool. */
int mppi_jump_pool_create(mppi_jump_ctx* const* ctxs, int32_t n, int32_t max_inflight,
                          void* d_scratch, size_t device_bytes, void* h_pinned,
                          size_t pinned_bytes, void* stream, mppi_jump_pool** out);

/* Enqueue a tick on `stream` through `slot`: for each request i < count,
 * controller ids[i] (distinct, in [0, n)) takes iters iterations from the
 * host state states[12 i .. 12 i + n_i) (fp32) and shifts.  With dist
 * (host, [count][8] fp32: words 0..3 added to the control channels, words
 * 4..6 a world-frame body force applied by the quadrotor model, word 7
 * unused) the tick then steps each request's simulated plant once from its
 * state under u_0 + dist.  Host arrays are read during the call only.
 * Asynchronous. */
int mppi_jump_pool_tick(mppi_jump_pool* pool, const int32_t* ids, const float* states,
                        const float* dist, int32_t count, int32_t iters, int32_t slot,
                        void* stream);

/* Put ctx at position `index` of the pool in place of its context, so that
 * a pool of fixed size can hold a changing set of resident controllers (a
 * server admitting a controller in place of one it evicted).  ctx must meet
 * the conditions of the pool's contexts (same rollout schedule; a fused
 * iteration; no debug_dump; diagonal covariance); the position
 * must not be in a tick in flight (EINVAL).  Uploads the position's
 * descriptor on `stream` and synchronises it, so later ticks on any stream
 * see the new context.
 * The caller keeps ctx and its workspace alive while the pool holds it. */
int mppi_jump_pool_replace(mppi_jump_pool* pool, int32_t index, mppi_jump_ctx* ctx, void* stream);

/* *finished = 1 when the slot holds no tick or its tick has finished on the
 * device, else 0.  Does not block. */
int mppi_jump_pool_query(mppi_jump_pool* pool, int32_t slot, int32_t* finished);

/* Take the results of the slot's finished tick, in the order of its
 * requests: ids [count], u_0 [count][4] fp32 (unused channels 0) and, if the
 * tick stepped the plant, the next plant states [count][12] fp32 (each
 * output may be NULL).  Frees the slot and its controllers for new ticks.
 * EINVAL if the slot holds no tick or the tick has not finished. */
int mppi_jump_pool_results(mppi_jump_pool* pool, int32_t slot, int32_t* ids, float* u0,
                           float* x_next, int32_t* count);

/* Free the host-side pool object (its events included). */
int mppi_jump_pool_destroy(mppi_jump_pool* pool);

/* ---- closed-loop and measurement helpers (not part of the method) ---- */

/* Simulated plant for closed-loop runs: one explicit Euler step of the
 * context's dynamics, x <- x + F(x, u + d) dt, on device state d_x ([n]),
 * applied control d_u ([m]) and disturbance d_dist ([m], added to the
 * control).  One GPU thread. */
int mppi_jump_plant_step(mppi_jump_ctx* ctx, float* d_x, const float* d_u,
                         const float* d_dist, void* stream);

/* The same plant step with a world-frame body force d_force ([3] fp32
 * device; NULL = none) for the models that take one (the quadrotor's gust;
 * the others ignore it), as the pool's plant step applies it. */
int mppi_jump_plant_step_force(mppi_jump_ctx* ctx, float* d_x, const float* d_u,
                               const float* d_dist, const float* d_force, void* stream);

/* Philox4x32-10 blocks of the library's generator for n caller-given
 * counters: d_out[4i..4i+4) = Philox(d_counters[4i..4i+4), key).  For
 * checking the generator against an independent implementation. */
int mppi_jump_philox(const uint32_t* d_counters, uint32_t key0, uint32_t key1,
                     uint32_t* d_out, int64_t n, void* stream);

/* Timing of the rollout kernel: when enabled, rollout launches are bracketed
 * by HIP events on their stream: the fused launches of one mppi_jump_step /
 * mppi_jump_control_step call (back-to-back rollout kernels) by one event
 * pair, any other rollout launch by its own.
 * profile_read synchronises on the recorded events and returns the summed
 * bracketed duration (ms), the number of rollout launches and the number of
 * iterations inside the brackets, then clears them.  At most 4096 brackets
 * are kept. */
int mppi_jump_profile(mppi_jump_ctx* ctx, int32_t enable);
int mppi_jump_profile_read(mppi_jump_ctx* ctx, double* total_ms, int64_t* launches,
                           int64_t* iterations);

#ifdef __cplusplus
}
#endif

#endif /* MPPI_JUMP_H */
