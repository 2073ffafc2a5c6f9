/*
 * sparrow.h -- C-ABI of the MI355X (gfx950) vectorized Sparrow step library.
 *
 * The library advances N independent copies of a 2D mobile-robot simulator
 * at once, as the Sparrow simulator of arXiv 2305.04180 does (Sec. 3.2):
 *   - per-env control delay and domain-randomised physics (Sec. 3.2.4),
 *   - simplified differential-drive kinematics, Eq. (5) and Eq. (6), applied
 *     row-wise over the batch as in Eq. (7) and Eq. (8),
 *   - LiDAR ray casting against each env's own occupancy grid, sensor noise,
 *     collision detection (Sec. 3.2 functionalities),
 *   - terminal rewards and done flags (Sec. 4.3.1), AutoReset (Sec. 3.2.5),
 *   - a gymnasium-style reset()/step() on device buffers with built-in
 *     normalisation and no host round trip (Sec. 3.2.1, Alg. 1 step 4),
 *   - an optional fused actor: a Q-network (Sec. 4.3.2) in BF16 on MFMA with
 *     FP32 accumulation, followed by vectorized epsilon-greedy exploration
 *     (VEM, Sec. 3.1.1), feeding K-step rollouts (Alg. 1 steps 2-4),
 *   - the sharer's experience buffer (Alg. 1 step 5, Alg. 2 step 1), filled
 *     by separate adds or by the step and rollout kernels themselves, the
 *     DDQN learner update (Alg. 2 step 2) and the time feedback mechanism
 *     (Sec. 3.1.2), and the paper's own task variant (Sec. 4.3.1).
 *
 * Conventions shared by every entry point:
 *   - Return value: SPARROW_OK (0) or a negative SPARROW_E* code; the message
 *     of the last failure on the calling thread is in sparrow_last_error().
 *   - "dev" pointers are HIP device pointers; "host" pointers are host memory.
 *     The caller owns every buffer it passes; the library never frees them
 *     and keeps no reference after the call returns (except sparrow_set_qnet,
 *     which copies).
 *   - Every GPU entry point is asynchronous on the stream given at create;
 *     results are valid after that stream is synchronised. No entry point
 *     synchronises except sparrow_status, sparrow_get_state, sparrow_set_state
 *     and sparrow_autotune.
 *   - A handle belongs to one stream and is not thread-safe; distinct handles
 *     are independent. Calls on one handle must not overlap.
 *   - Layouts: obs is FP32 row-major [N][obs_dim] (obs_dim = n_rays + 4 for
 *     the default task; see sparrow_set_task); reward FP32 [N]; done uint8
 *     0/1 [N]; flags uint8 [N]; actions int32 [N] in [0, n_actions) (7 by
 *     default). Rollout outputs are step-major [K][N].
 *
 * Observation row of the default task (Sec. 4.3.1 state, normalised,
 * relative to the robot; sparrow_set_task documents the other layout):
 *   [0, n_rays)   range_j / range (after noise, clipped to [0, range])
 *   n_rays        linear velocity / v_max of the env
 *   n_rays + 1    angular velocity / omega_max
 *   n_rays + 2    distance to target / (sqrt(2) * max(W, H))
 *   n_rays + 3    bearing of the target in the robot frame / pi, in (-1, 1]
 */
#ifndef SPARROW_H
#define SPARROW_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPARROW_OK 0
#define SPARROW_EINVAL (-1)       /* bad argument, shape or configuration          */
#define SPARROW_ENOMEM (-2)       /* device or host allocation failed              */
#define SPARROW_EHIP (-3)         /* HIP runtime failure (message has the detail)  */
#define SPARROW_ERESET (-4)       /* AutoReset found no free start/target cell     */
#define SPARROW_EUNSUPPORTED (-5) /* not gfx950, or LDS/variant capacity exceeded  */

#define SPARROW_N_ACTIONS 7
#define SPARROW_MAX_SIDE 512
#define SPARROW_MAX_RAYS 128

/* flags bits (sparrow_step / sparrow_rollout) */
#define SPARROW_FLAG_TERMINATED 1u /* collision or arrival                        */
#define SPARROW_FLAG_TRUNCATED 2u  /* episode reached timeout_steps               */
#define SPARROW_FLAG_COLLISION 4u
#define SPARROW_FLAG_ARRIVAL 8u

typedef struct sparrow_env sparrow_env; /* opaque; library-owned */

/* Configuration, copied at create. Units: cells, seconds, radians.
 * Domain randomisation (Sec. 3.2.4): at every episode start each env draws
 * dt ~ U[dt_lo, dt_hi] (control interval), K ~ U[K_lo, K_hi] (inertia blend of
 * Eq. (5)), mu ~ U[mu_lo, mu_hi] (friction gain on the target velocity),
 * v_max ~ U[vmax_lo, vmax_hi] (cells/s), sigma ~ U[sigma_lo, sigma_hi] (LiDAR
 * noise, cells), delay ~ U{delay_lo..delay_hi} (steps, <= 2), and its start
 * pose. omega_max is fixed. Every random draw is Philox4x32-10 keyed by seed
 * and counted by (env, global step, purpose, index). */
typedef struct {
  int32_t n_envs;        /* N >= 1                                        */
  int32_t n_rays;        /* 1..128, spread over fov_rad, endpoints included */
  int32_t n_actions;     /* must be 7                                     */
  float fov_rad;         /* field of view, centred on the heading         */
  float range_cells;     /* LiDAR range R > 0                             */
  float march_step;      /* sample spacing along a ray, > 0               */
  float robot_radius;    /* collision disk radius, (0, 8]                 */
  float arrive_radius;   /* arrival when the distance to target <= this   */
  int32_t timeout_steps; /* truncation after this many steps, >= 1        */
  float dt_lo, dt_hi, K_lo, K_hi, mu_lo, mu_hi, vmax_lo, vmax_hi, omega_max,
      sigma_lo, sigma_hi;
  int32_t delay_lo, delay_hi;
  uint64_t seed;
} sparrow_config;

/* Maps (host pointers, copied and bit-packed at create). cells holds n_maps
 * uint8 grids [height][width] row-major (0 = free, else occupied) at byte
 * offsets[m]; x indexes columns, y rows. env_to_map[n_envs] lets envs share a
 * map. 1 <= width, height <= 512. */
typedef struct {
  int32_t n_maps;
  const uint8_t *cells;
  const int64_t *offsets;
  const int32_t *width;
  const int32_t *height;
  const int32_t *env_to_map;
} sparrow_maps;

/* Create a handle on the current HIP device; all work goes to hip_stream
 * (a hipStream_t; NULL = the null stream). Packs the maps into LDS-ready
 * words on the device. No env is initialised until sparrow_reset.
 * Errors: EINVAL, ENOMEM, EHIP, EUNSUPPORTED (device is not gfx950). */
int sparrow_create(const sparrow_config *cfg, const sparrow_maps *maps, void *hip_stream,
                   sparrow_env **out);

/* Reset every env (Alg. 1 initial s = envs.reset()): draws physics, start and
 * target, writes obs (dev [N][obs_dim]). Advances the global step by one.
 * A map with no free start/target makes the error sticky (see status). */
int sparrow_reset(sparrow_env *env, float *obs);

/* One vectorized step (Alg. 1 step 4: s', r, done = envs.step(a_hat)).
 * actions: dev [N] (values outside [0, n_actions) act as "stop"). Writes obs
 * (dev [N][obs_dim]), reward, done, and optionally flags (dev [N]) and
 * final_obs (dev [N][obs_dim], the observation at the terminal pose of envs
 * that are done; rows of other envs are left untouched). Envs that are done
 * are reset inside the step and obs holds their first observation of the
 * next episode (AutoReset, Sec. 3.2.5). EINVAL before the first reset (or
 * set_state) and after a task change. Advances the global step by one. */
int sparrow_step(sparrow_env *env, const int32_t *actions, float *obs, float *reward,
                 uint8_t *done, uint8_t *flags, float *final_obs);

/* Uniform random actions for the current global step (dev [N]); the same
 * draws a rollout with use_qnet = 0 makes. Does not advance the step. */
int sparrow_random_actions(sparrow_env *env, int32_t *actions);

/* ---- Task (Sec. 4.3.1) -------------------------------------------------------
 * The default task is the workloads': 7 actions (the table in the design
 * notes), the progress reward (previous minus current distance to the
 * target, minus 0.01) with terminal -10 on collision / +10 on arrival, and
 * the target state [ranges | v_l/v_max, v_a/omega_max, distance/(sqrt 2
 * max(W, H)), bearing/pi] of n_rays + 4 entries. The paper's own task
 * differs in three places, each selectable:
 *   n_actions = 5: the five actions Sec. 4.3.1 lists (turn left, straight
 *     and left, straight, straight and right, turn right), rows 0, 1, 3, 5,
 *     6 of the 7-row table; ids >= n_actions act as stop.
 *   reward = SPARROW_REWARD_EQ11: terminal collide_reward / arrive_reward
 *     (-10 / +75 there); otherwise Eq. (11), r = w_d1 r_d1 + w_d2 r_d2 +
 *     w_v r_v + w_alpha r_alpha + w_d r_d in binary32 in this order, with
 *     r_d1 = max(1 - |x - tx| / D, 0), r_d2 = max(1 - |y - ty| / D, 0),
 *     r_v = 1 if v_l > v_max / 2 else 0, r_alpha = 1 - |alpha| / pi (alpha:
 *     heading relative to the direction of the target), r_d = -1 if an
 *     occupied cell lies within near_dist of the robot's edge (touching
 *     included) else 0; D = plan_dist. The paper leaves the shapes of r_d1,
 *     r_d2 and r_alpha open: these are readings.
 *   state = SPARROW_STATE_RELATIVE: [ranges | (x - tx)/D, (y - ty)/D,
 *     alpha/pi, v_l/v_max, v_a/omega_max], n_rays + 5 entries (32 with the
 *     paper's 27 rays).
 * Setting a task synchronises the stream, drops the installed Q-network
 * (its sizes follow the task) and requires a reset before the next step.
 * EINVAL for n_actions other than 5 or 7, unknown modes, plan_dist <= 0 or
 * near_dist outside [0, 64]. The collecting rollout runs the default task
 * only (EUNSUPPORTED otherwise). */
#define SPARROW_REWARD_PROGRESS 0
#define SPARROW_REWARD_EQ11 1
#define SPARROW_STATE_TARGET 0
#define SPARROW_STATE_RELATIVE 1
typedef struct {
  int32_t n_actions;   /* 7 or 5 */
  int32_t reward;      /* SPARROW_REWARD_* */
  int32_t state;       /* SPARROW_STATE_* */
  float arrive_reward; /* terminal reward on arrival */
  float collide_reward;/* terminal reward on collision */
  float plan_dist;     /* D, cells */
  float near_dist;     /* r_d margin around the robot's edge, cells */
  float w_d1, w_d2, w_v, w_alpha, w_d; /* Eq. (11) weights (0.3 0.1 0.3 0.3 0.1) */
} sparrow_task;
int sparrow_set_task(sparrow_env *env, const sparrow_task *task);
/* Entries of one observation row under the current task (n_rays + 4 or
 * n_rays + 5); -1 for NULL. */
int32_t sparrow_obs_dim(const sparrow_env *env);

/* Install the actor: Q-network dims[4] = {obs_dim, h1, h2, A} (host), with
 * obs_dim = sparrow_obs_dim(env) and A the task's n_actions (EINVAL
 * otherwise). Shapes: h1 = h2 = 256 with obs_dim <= 96, or h1 = 256, h2 =
 * 128 with obs_dim <= 64 (the [32, 256, 128, 5] network of Sec. 4.3.2):
 * weights resident in registers, drives the fused rollout; h1 = h2 = 512
 * with obs_dim <= 96: weights streamed from L2, serves sparrow_act and
 * sparrow_qnet_forward only (a rollout with use_qnet = 1 returns
 * EUNSUPPORTED). Other shapes return EUNSUPPORTED. w_bf16: dev, bf16 bit
 * patterns, [W1 (h1 x obs_dim) | W2 (h2 x h1) | W3 (A x h2)], each row-major
 * [out][in] (Sec. 4.3.2 fully connected layers with ReLU). b_f32: dev
 * [h1 + h2 + A]. eps: dev [N] per-env exploration probability of VEM
 * (Sec. 3.1.1; sparrow_vem_epsilon computes the schedule). All three are
 * copied; the call synchronises the stream. On any failure the network
 * installed before the call (if any) stays installed and usable. */
int sparrow_set_qnet(sparrow_env *env, const int32_t *dims, const uint16_t *w_bf16,
                     const float *b_f32, const float *eps);

/* VEM's per-env exploration probabilities for a fixed exploring interval
 * (Sec. 3.1.1: the last m envs form the exploring interval, whose
 * probabilities rise linearly across it from e_min to e_min + e_max; the
 * other envs hold e_min):
 *   eps_i = e_min for i < n_envs - m, else e_min + e_max * (i - (n_envs - m))
 *       / (m - 1) (m = 1: e_min + e_max),
 * in binary64 rounded once to binary32. Writes dev eps [n_envs] on the env's
 * stream, ready for sparrow_set_qnet (m = n_envs, e_min 0.01, e_max 0.29
 * gives the workloads' linspace(0.01, 0.3)). EINVAL unless 0 <= m <= n_envs
 * and e_min, e_max >= 0. */
int sparrow_vem_epsilon(sparrow_env *env, int32_t m, double e_min, double e_max, float *eps);

/* VEM whose exploring interval shrinks during training (Sec. 3.1.1: "the OR
 * is linearly diminished"; Table 6: OR 16 -> 3 over 500K transitions, E_min
 * 0.01, E_max 0.8). From this call on, the actor (rollout and sparrow_act)
 * uses for env i at global step g, with T = n_envs * g transitions,
 *   m = or_start - floor((or_start - or_final) * min(T, decay) / decay)
 *       (decay_transitions = 0: m = or_final),
 *   eps_i = e_min for i < n_envs - m, else e_min + e_max * (i - (n_envs - m))
 *       / (m - 1) (m = 1: e_min + e_max),
 * in binary64 rounded once to binary32, instead of the eps array of
 * sparrow_set_qnet. EINVAL unless e_min, e_max >= 0 and
 * 0 <= or_final <= or_start <= n_envs, decay_transitions >= 0. */
int sparrow_set_vem_schedule(sparrow_env *env, double e_min, double e_max, int32_t or_start,
                             int32_t or_final, int64_t decay_transitions);

/* Q-network forward on given observations (dev obs [n][obs_dim] -> dev q
 * [n][A] FP32, dev greedy [n] int32 = lowest argmax). Same MFMA code as the
 * fused actor: the observation is rounded to bf16 (RNE), layers accumulate in
 * FP32, hidden activations are stored as bf16. Either output may be NULL. */
int sparrow_qnet_forward(sparrow_env *env, const float *obs, int32_t n, float *q,
                         int32_t *greedy);

/* The actor as a separate kernel: Q-network on obs (dev [N][obs_dim]), then
 * VEM with the current global step. Writes actions (dev [N]). Does not
 * advance the step. */
int sparrow_act(sparrow_env *env, const float *obs, int32_t *actions);

/* K-step rollout in one persistent kernel (maps stay in LDS for all K steps),
 * launched directly on the stream. Per step: actor (use_qnet = 1: the
 * installed Q-network + VEM on the current observation; 0: uniform random
 * actions), then the step with AutoReset. Outputs, step-major: actions
 * (dev [K][N], nullable), reward (dev [K][N]), done (dev [K][N]), and obs
 * (dev [N][obs_dim]) after the last step. Needs a prior reset (the current
 * observation is kept on the device). Advances the global step by K. */
int sparrow_rollout(sparrow_env *env, int32_t K, int32_t use_qnet, int32_t *actions,
                    float *reward, uint8_t *done, float *obs);

/* sparrow_rollout that also returns what every step observed, for checks of
 * the intermediate steps and precision reports: obs_steps (dev [K][N]
 * [obs_dim] FP32, nullable) receives the observation after each step (row
 * K - 1 equals obs), hits_steps (dev [K][N][n_rays] int16, nullable) the
 * per-ray first-hit sample index of that observation (-1: none; row K - 1
 * equals what sparrow_debug_hits then returns). Same kernel, variant and
 * results as sparrow_rollout, launched directly rather than from the cached
 * graph, plus copies of the last step's rows on the env's stream. */
int sparrow_rollout_trace(sparrow_env *env, int32_t K, int32_t use_qnet, int32_t *actions,
                          float *reward, uint8_t *done, float *obs, float *obs_steps,
                          int16_t *hits_steps);

/* Per-ray sample index of the first hit (-1: none) of the most recent
 * observation of each env (dev [N][n_rays] int16). For parity checks. */
int sparrow_debug_hits(sparrow_env *env, int16_t *hit_k);

/* Synchronising state access (host buffers). Float fields [N][13]:
 * x y phi vl va tx ty dprev dt K mu vmax sigma; int fields [N][4]:
 * t delay q0 q1. set_state also invalidates the cached observation. */
int sparrow_get_state(sparrow_env *env, float *f_host, int32_t *i_host);
int sparrow_set_state(sparrow_env *env, const float *f_host, const int32_t *i_host);

uint32_t sparrow_global_step(const sparrow_env *env);
void sparrow_set_global_step(sparrow_env *env, uint32_t g);

/* Kernel variants. kernel: 0 = step/reset, 1 = rollout. envs_per_group in
 * {1, 2, 4, 8}; lanes_per_env in {16, 32, 64} (fewer lanes than rays: each
 * lane marches several rays; more lanes than rays: lanes of one ray split its
 * samples). Every variant computes identical results. */
int sparrow_set_variant(sparrow_env *env, int32_t kernel, int32_t envs_per_group,
                        int32_t lanes_per_env);
int sparrow_get_variant(const sparrow_env *env, int32_t kernel, int32_t *envs_per_group,
                        int32_t *lanes_per_env);
/* Time every admissible variant of both kernels on a scratch copy of the
 * state (the env itself is not advanced), keep the fastest. Synchronises.
 * report (host, nullable) receives a JSON summary of the timings. */
int sparrow_autotune(sparrow_env *env, int32_t steps, char *report, int32_t report_len);
/* sparrow_autotune with its choice kept in a file (host path, JSON lines):
 * the variants chosen for the same device and workload shape (envs, rays,
 * march, robot radius, task, actor sizes and the count of envs per map
 * shape) are read back and installed without timing; otherwise the
 * variants are timed as by sparrow_autotune and the choice is appended.
 * report receives {"cached": true, "chosen": ...} when read from the file.
 * EINVAL if the file cannot be appended to. */
int sparrow_autotune_cached(sparrow_env *env, int32_t steps, const char *path, char *report,
                            int32_t report_len);

/* Synchronise the stream and return the sticky asynchronous error (ERESET)
 * or a HIP error, else SPARROW_OK. */
int sparrow_status(sparrow_env *env);
void sparrow_destroy(sparrow_env *env);
const char *sparrow_last_error(void);

/* ---- Experience buffer ------------------------------------------------------
 * The sharer's buffer of Sec. 3.1.2: Alg. 1 step 5 adds the batched
 * transitions (s, a, r, s', done) and Alg. 2 step 1 samples a mini-batch
 * (Table 6: 1 M transitions, mini-batch 256). It lives on the device as a
 * ring of compact transitions, about 2 * n_rays + 21 bytes each:
 *   ranges (obs entries [0, n_rays))  uint8 level = nearest integer to
 *       255 * clamp(o, 0, 1) (product rounded to binary32, ties to even),
 *       read back as the binary32 quotient level / 255;
 *   the four scalar entries          binary16, round to nearest even, read
 *       back exactly;
 *   action int8, reward binary32, done one bit.
 * A push of n writes slot (head + i) mod capacity for its i-th transition and
 * advances head by n; size = min(total pushed, capacity). The handle is
 * bound to the stream given at create, like sparrow_env. */
typedef struct sparrow_ring sparrow_ring;

/* capacity in [1, 2^26] slots, n_rays in [1, SPARROW_MAX_RAYS]; seed keys
 * the sampler's Philox. Allocates the ring on the current device. */
int sparrow_ring_create(int32_t capacity, int32_t n_rays, uint64_t seed, void *hip_stream,
                        sparrow_ring **out);
/* Add n <= capacity transitions (n = 0 does nothing and may pass NULL
 * buffers). dev s, s_next: [n][n_rays + 4] FP32;
 * a: int32 [n] in [0, 128); r: FP32 [n]; done: uint8 [n]. s_final (dev,
 * nullable, [n][n_rays + 4]): where done[i] != 0, s' is row i of s_final
 * (sparrow_step's final_obs, the terminal observation) instead of s_next. */
int sparrow_ring_push(sparrow_ring *ring, int32_t n, const float *s, const int32_t *a,
                      const float *r, const float *s_next, const float *s_final,
                      const uint8_t *done);
/* Mini-batch of B uniform draws over the stored slots: slot b is
 * floor(w * size / 2^32), w the first word of Philox4x32-10 at counter
 * (b, draw, 8, 0) under the ring's seed. Outputs (dev, read back to FP32):
 * s, s_next [B][n_rays + 4], a int32 [B], r [B], done uint8 [B], idx int32
 * [B] (nullable). EINVAL when the ring is empty. */
int sparrow_ring_sample(sparrow_ring *ring, int32_t B, uint32_t draw, float *s, int32_t *a,
                        float *r, float *s_next, uint8_t *done, int32_t *idx);
/* The same read-back at the given slots (host int32 [n], each in
 * [0, size), checked on the host before anything is launched). */
int sparrow_ring_gather(sparrow_ring *ring, int32_t n, const int32_t *slots_host, float *s,
                        int32_t *a, float *r, float *s_next, uint8_t *done);
/* sparrow_ring_gather for callers that cannot allocate device memory (code
 * that must not call hipMalloc, such as tight serving loops or harnesses
 * that forbid it): the same read-back and outputs, with the slots staged in
 * a fixed array that the library holds on each GPU (SPARROW_GATHER_STATIC_MAX
 * int32 entries, 256 KiB, kept until the process ends) instead of a
 * library-allocated buffer. The call allocates nothing; n above
 * SPARROW_GATHER_STATIC_MAX is EINVAL, as are slots outside [0, size).
 * Synchronises the ring's stream before returning. Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (other threads,
 * other rings' streams) race, so the caller serialises them. */
#define SPARROW_GATHER_STATIC_MAX 65536
int sparrow_ring_gather_static(sparrow_ring *ring, int32_t n, const int32_t *slots_host, float *s,
                               int32_t *a, float *r, float *s_next, uint8_t *done);
int64_t sparrow_ring_size(const sparrow_ring *ring);
int64_t sparrow_ring_head(const sparrow_ring *ring);
/* Synchronise the ring's stream; SPARROW_OK or the HIP error. */
int sparrow_ring_status(sparrow_ring *ring);
void sparrow_ring_destroy(sparrow_ring *ring);

/* sparrow_rollout that also performs Alg. 1 step 5 inside the same kernel:
 * step t's N transitions (s, a_hat, r, s', done) go straight into the ring,
 * transition (t, i) at slot (head + t N + i) mod capacity, stored exactly as
 * sparrow_ring_push stores them. s is the observation the actor saw (for
 * t = 0 the current observation), a_hat the actor's action (before the
 * control delay), s' the observation after the step. For a done env, s' is
 * its terminal observation before the reset (the one sparrow_step returns
 * as final_obs; push with s_final) when terminal_obs != 0, else the
 * observation after the AutoReset (what the step returns as obs; push
 * without s_final), which skips one ray cast per done env. Afterwards head
 * and size advance by K N. Requirements: the ring's n_rays equals the env's
 * and K N <= capacity (EINVAL otherwise). actions, reward, done (dev [K][N])
 * are nullable here; obs as in sparrow_rollout. Runs on the env's stream (a
 * small kernel clearing the range's done bits, then the rollout): when the
 * ring is bound to another stream, the caller orders the two (events). */
int sparrow_rollout_collect(sparrow_env *env, sparrow_ring *ring, int32_t K, int32_t use_qnet,
                            int32_t terminal_obs, int32_t *actions, float *reward,
                            uint8_t *done, float *obs);

/* sparrow_step (no final_obs) that also adds the step's N transitions to the
 * ring in the same kernel (Alg. 1 step 5 with a separate actor, as in the
 * full collection loop): transition i at slot (head + i) mod capacity, s =
 * the env's current observation (the one the actions were chosen on), a =
 * actions[i] as given (stored as int8), r, done, and s' as in
 * sparrow_rollout_collect (terminal observation for done envs when
 * terminal_obs != 0, else the post-reset one); stored exactly as
 * sparrow_ring_push stores them. Head and size advance by N. Needs the
 * target state (EUNSUPPORTED otherwise), the ring's n_rays equal to the
 * env's and N <= capacity (EINVAL). Runs on the env's stream (the done-bit
 * clear, then the step). */
int sparrow_step_collect(sparrow_env *env, sparrow_ring *ring, const int32_t *actions,
                         float *obs, float *reward, uint8_t *done, uint8_t *flags,
                         int32_t terminal_obs);

/* ---- Learner ---------------------------------------------------------------
 * The learner's update of Alg. 2 step 2 (train the learner's model on a
 * mini-batch with DDQN; Table 6: gamma 0.98, learning rate 1e-4, target
 * network every 200 updates, mini-batch 256), on the device in FP32:
 *   a*   = argmax_a Q_online(s') (lowest index on ties),
 *   y    = r + gamma (1 - done) Q_target(s')[a*]  (a constant),
 *   loss = mean over the batch of huber_k(Q_online(s)[a] - y),
 * gradients by back-propagation (relu'(0) = 0), one Adam step (bias-
 * corrected) on every weight and bias, and after every target_every-th
 * update the target network becomes a copy of the online one. The network
 * is that of sparrow_set_qnet (Sec. 4.3.2, ReLU), weights row-major
 * [out][in], concatenated [W1 | W2 | W3], biases [b1 | b2 | b3]. */
typedef struct {
  float gamma, lr, beta1, beta2, adam_eps, huber_k;
  int32_t target_every; /* 0: the target network never changes */
  int32_t max_batch;    /* largest mini-batch (scratch is sized for it), <= 65535 */
} sparrow_learner_config;
typedef struct sparrow_learner sparrow_learner;

/* dims (host) = {d0 <= 128, h1 <= 512, h2 <= 512, A <= 16}; w, b: host FP32
 * initial weights (copied; the target network starts equal). */
int sparrow_learner_create(const int32_t *dims, const float *w_host, const float *b_host,
                           const sparrow_learner_config *cfg, void *hip_stream,
                           sparrow_learner **out);
/* One update on B <= max_batch transitions (dev: s, s_next [B][d0] FP32, a
 * int32 [B], r FP32 [B], done uint8 [B]); loss (dev [1], nullable) receives
 * the mini-batch loss. Asynchronous on the learner's stream. */
int sparrow_learner_update(sparrow_learner *L, int32_t B, const float *s, const int32_t *a,
                           const float *r, const float *s_next, const uint8_t *done,
                           float *loss);
/* Q of the online (which = 0) or target (1) network on n <= max_batch rows
 * (dev x [n][d0] -> dev q [n][A]). */
int sparrow_learner_q(sparrow_learner *L, int32_t which, int32_t n, const float *x, float *q);
/* The online network for the actor (Alg. 2 step 3 uploads it to the
 * sharer, Alg. 1 step 1 downloads it): weights rounded to bf16 (RNE, dev
 * [nw] bit patterns) and biases (dev [nb] FP32), ready for sparrow_set_qnet. */
int sparrow_learner_export_bf16(sparrow_learner *L, uint16_t *w_bf16, float *b);
/* Synchronising copies to host (each nullable): online and target weights
 * and biases, and the last update's gradients. */
int sparrow_learner_read(sparrow_learner *L, float *w, float *b, float *wt, float *bt,
                         float *gw, float *gb);
int64_t sparrow_learner_steps(const sparrow_learner *L);
void sparrow_learner_destroy(sparrow_learner *L);

/* ---- Time feedback mechanism ------------------------------------------------
 * Sec. 3.1.2: actor and learner run side by side; to hold the transitions per
 * step TPS = B_batch B_step / T_step at its target, Eq. (TB2TV) asks that a
 * vectorized step of the actor take rho = N TPS / B_batch times as long as
 * an update of the learner. The actor reports the duration of each
 * vectorized step (sleep excluded), the learner of each update; with their
 * means so far, xi = rho mean(learner) - mean(actor): the actor sleeps xi
 * after a step if xi > 0, else the learner sleeps -xi / rho after an update
 * (xi = 0 until both have reported). Host-only and thread-safe: the two
 * sides may report from different threads. Times in seconds. */
typedef struct sparrow_tfm sparrow_tfm;
int sparrow_tfm_create(double rho, sparrow_tfm **out); /* EINVAL unless rho > 0 */
void sparrow_tfm_actor_period(sparrow_tfm *t, double seconds);
void sparrow_tfm_learner_period(sparrow_tfm *t, double seconds);
double sparrow_tfm_xi(const sparrow_tfm *t);
double sparrow_tfm_actor_sleep(const sparrow_tfm *t);
double sparrow_tfm_learner_sleep(const sparrow_tfm *t);
void sparrow_tfm_destroy(sparrow_tfm *t);

/* ---- Peak-rate probes -------------------------------------------------------
 * Measurements of the device that bound the step kernels' rooflines; not part
 * of the method. Each runs one untimed launch, then times its launches with
 * HIP events on hip_stream (NULL: the default stream) and synchronises.
 *   kind 0: LDS reads of 16 bytes per lane, bank-conflict free (iters reads
 *           per lane; 2 workgroups of 1024 lanes per CU, 16 rounds), 3 launches
 *   kind 1: LDS reads of 4 bytes per lane (the ray march's access width),
 *           otherwise as kind 0
 *   kind 2: HBM copy of size bytes (in [1 MiB, 16 GiB], a multiple of 16) into
 *           a second buffer, iters launches; rate counts read + write bytes.
 *           Allocates both buffers and frees them before returning.
 *   kind 3: dense BF16 MFMA, v_mfma_f32_16x16x32_bf16 on register operands,
 *           8 chains of iters products per wave, 16 waves per CU, 3 launches
 * rate (host, required): bytes/s (kinds 0-2) or FLOP/s (kind 3); seconds
 * (host, nullable): the timed launches' duration. EINVAL for a kind outside
 * 0..3, iters outside [1, 2^20] or a bad size; ENOMEM, EHIP as usual. */
int sparrow_peak(int32_t kind, int64_t size, int32_t iters, void *hip_stream, double *rate,
                 double *seconds);

#ifdef __cplusplus
}
#endif
#endif
