/*
 * sparrow_oracle.h -- plain, slow CPU oracle of the vectorized Sparrow step.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path (the HIP library and
 * its Python binding) may include, link or call this code; only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark do. It shares no
 * source, header, table or constant generator with the GPU path.
 *
 * What it computes (arXiv 2305.04180):
 *   Sec. 3.2.2, Eq. (5)  velocity blend  v' = K v + (1-K) v_hat
 *   Sec. 3.2.2, Eq. (6)  pose update with the new velocity and the old heading
 *   Sec. 3.2.3, Eq. (7)/(8) the same rules row-wise over N copies (one loop)
 *   Sec. 3.2   LiDAR by ray casting on the occupancy grid, sensor noise,
 *              collision detection, AutoReset (Sec. 3.2.5), and per-episode
 *              domain randomisation of the world variable (Sec. 3.2.4)
 *   Sec. 4.3.1 terminal rewards on collision / arrival, discrete target
 *              velocities, normalised relative state
 *   Sec. 3.1.1 vectorized epsilon-greedy exploration (VEM)
 *   Sec. 4.3.2 fully connected Q-network mapping the state to actions
 * Details the paper leaves open (ray-march rule, collision geometry, RNG,
 * normalisation constants, reward shaping) follow one fixed reading, listed
 * in the repository's design notes.
 *
 * Floating point: every FP32 expression that can change a grid index or a
 * done flag is evaluated as separately rounded binary32 operations in the
 * written order (build with -ffp-contract=off -fno-fast-math). Noise,
 * bearing and the Q-network are evaluated in FP64 and rounded once.
 *
 * Parity pins: see the test suite (closed forms, hand-built maps, a
 * brute-force FP64 voxel walk, an independent Philox, libm sincos).
 */
#ifndef SPARROW_ORACLE_H
#define SPARROW_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_STOP = 7, ORC_NACT = 7 };
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ERESET = -4 };
/* Philox counter word 2 ("purpose") */
enum {
  ORC_P_RESET_DR = 1, ORC_P_RESET_START = 2, ORC_P_RESET_TARGET = 3,
  ORC_P_NOISE = 4, ORC_P_NOISE_RESET = 5, ORC_P_ACTION_UNIFORM = 6,
  ORC_P_EXPLORE = 7
};
/* flags bits */
enum { ORC_F_TERM = 1, ORC_F_TRUNC = 2, ORC_F_COLL = 4, ORC_F_ARRIVE = 8 };

typedef struct {
  int32_t n_envs, n_rays, n_actions;
  float fov, range, ds, robot_r, arrive_r;
  int32_t t_max;
  float dt_lo, dt_hi, K_lo, K_hi, mu_lo, mu_hi, vmax_lo, vmax_hi, omega_max,
      sigma_lo, sigma_hi;
  int32_t delay_lo, delay_hi;
  uint64_t seed;
} orc_config;

typedef struct {
  double max_rel_x, max_rel_y, max_rel_phi, max_rel_vl, max_rel_va;
  uint64_t ties_ray;     /* samples where floor(p32) != floor(p64) */
  uint64_t ties_coll;    /* collision tests where FP32 and FP64 disagree */
  uint64_t samples;      /* sum over marched rays of (k_hit + 1)         */
  uint64_t rays;         /* rays marched                                 */
  uint64_t kin_steps;    /* env-steps checked against the FP64 shadow    */
} orc_stats;

typedef struct orc_env orc_env;

/* cells: concatenated uint8 [H][W] row-major grids, 0 = free; offsets[m] is
 * the byte offset of map m. env_to_map[n_envs]. Copies everything. */
orc_env *orc_create(const orc_config *cfg, int32_t n_maps, const uint8_t *cells,
                    const int64_t *offsets, const int32_t *width,
                    const int32_t *height, const int32_t *env_to_map);
void orc_destroy(orc_env *e);
int32_t orc_status(const orc_env *e);
uint32_t orc_global_step(const orc_env *e);
void orc_set_global_step(orc_env *e, uint32_t g);
int32_t orc_obs_dim(const orc_env *e);

/* Task variant (Sec. 4.3.1). The default task is the workloads': 7 actions,
 * the progress reward (previous minus current distance to the target, minus
 * 0.01) with terminal -10 / +10, and the target state [ranges | v_l/v_max,
 * v_a/omega_max, distance/(sqrt 2 max(W, H)), bearing/pi]. The paper's own
 * formulation changes three things, selectable apart:
 *   n_actions = 5: the five actions it lists, rows {0,1,3,5,6} of the table;
 *   reward = ORC_REWARD_EQ11: Eq. (11) on steps that do not end the episode
 *     (see eq11_reward in the source for the reading of its terms), with
 *     the terminal rewards arrive_reward (+75 there) / collide_reward (-10);
 *   state = ORC_STATE_RELATIVE: [ranges | (x - tx)/D, (y - ty)/D, alpha/pi,
 *     v_l/v_max, v_a/omega_max], n_rays + 5 entries (27 + 5 = 32 there).
 * D = plan_dist (cells); near_dist (cells) is the r_d margin around the
 * robot's edge; w_* the Eq. (11) weights (0.3 0.1 0.3 0.3 0.1). Parity
 * against the paper is unpinned for this variant: the shapes of r_d1, r_d2
 * and r_alpha and the cell size are not stated. Returns ORC_EINVAL for
 * n_actions other than 5 or 7, unknown modes, plan_dist <= 0 or
 * near_dist < 0. orc_obs_dim follows the state. */
enum { ORC_REWARD_PROGRESS = 0, ORC_REWARD_EQ11 = 1 };
enum { ORC_STATE_TARGET = 0, ORC_STATE_RELATIVE = 1 };
typedef struct {
  int32_t n_actions, reward, state;
  float arrive_reward, collide_reward, plan_dist, near_dist;
  float w_d1, w_d2, w_v, w_alpha, w_d;
} orc_task;
int32_t orc_set_task(orc_env *e, const orc_task *t);
/* Disk test with radius robot_r + near_dist (the r_d term of Eq. (11)). */
int32_t orc_near(const orc_env *e, int32_t map, float px, float py);

/* Reset every env (draws use the current global step), write obs, advance. */
int32_t orc_reset(orc_env *e, float *obs, int16_t *hit_k);

/* One vectorized step of envs [e0, e1) at the current global step; does not
 * advance the global step (orc_advance does), so disjoint ranges may run on
 * different threads. final_obs, flags, hit_k, stats may be NULL. */
int32_t orc_step_range(orc_env *e, int32_t e0, int32_t e1, const int32_t *actions,
                       float *obs, float *reward, uint8_t *done, uint8_t *flags,
                       float *final_obs, int16_t *hit_k, orc_stats *stats);
void orc_advance(orc_env *e);
/* orc_step_range over all envs, then orc_advance */
int32_t orc_step(orc_env *e, const int32_t *actions, float *obs, float *reward,
                 uint8_t *done, uint8_t *flags, float *final_obs, int16_t *hit_k,
                 orc_stats *stats);

/* State access. Float fields, [n_envs][13]:
 *   x y phi vl va tx ty dprev dt K mu vmax sigma
 * Int fields, [n_envs][4]: t delay q0 q1 */
enum { ORC_NF = 13, ORC_NI = 4 };
void orc_get_state(const orc_env *e, float *f, int32_t *i);
void orc_set_state(orc_env *e, const float *f, const int32_t *i);

/* Building blocks exposed so the tests can pin them one by one. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_sincos_f32(float phi, float *s, float *c);
void orc_sincos_batch(int32_t n, const float *phi, float *s, float *c);
void orc_philox_batch(int32_t n, const uint32_t *ctr, const uint32_t key[2], uint32_t *out);
int32_t orc_collides(const orc_env *e, int32_t map, float px, float py);
int32_t orc_march(const orc_env *e, int32_t map, float x, float y, float ux, float uy);
void orc_ray_table(const orc_env *e, float *c, float *s);
uint16_t orc_bf16_rne(float f);

/* Q-network (Sec. 4.3.2 fully connected layers, ReLU). dims[4] = {d0,h1,h2,A}.
 * w: bf16 bits, [W1 (h1 x d0) | W2 (h2 x h1) | W3 (A x h2)], row-major
 * [out][in]; b: f32 [b1 | b2 | b3]. The observation is rounded to bf16 (RNE)
 * and everything after is FP64; round_act != 0 additionally rounds the two
 * hidden activations to bf16 after ReLU. q: [n][A]. */
void orc_qnet_f64(const int32_t dims[4], const uint16_t *w, const float *b,
                  int32_t n, const float *obs, int32_t round_act, double *q);
/* VEM (Sec. 3.1.1): greedy argmax (lowest index on ties), replaced by a
 * uniform random action with probability eps[i]. Uses the current global
 * step; does not advance. explore may be NULL. */
void orc_vem(const orc_env *e, const double *q, int32_t n_actions, const float *eps,
             int32_t *actions, uint8_t *explore);
void orc_uniform_actions(const orc_env *e, int32_t *actions);
/* VEM exploration noise per env: the last m envs form the exploring
 * interval, linear from e_min to e_min + e_max; the rest hold e_min. */
void orc_vem_epsilon(int32_t n, int32_t m, double e_min, double e_max, float *eps);
/* Size of the exploring interval after T transitions when it shrinks
 * linearly from or_start to or_final over `decay` transitions (Sec. 3.1.1;
 * Table 6 "Linear Decay Steps of OR"): or_start - floor((or_start -
 * or_final) * min(T, decay) / decay); decay = 0 gives or_final. */
int32_t orc_vem_or(int64_t T, int32_t or_start, int32_t or_final, int64_t decay);

#ifdef __cplusplus
}
#endif
#endif
