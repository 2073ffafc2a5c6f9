/*
 * learner_oracle.h -- plain CPU oracle of the learner update (arXiv
 * 2305.04180, Alg. 2 step 2: train the learner's model on a mini-batch with
 * DDQN; Table 6 gives gamma, the learning rate, the target-network update
 * period and the mini-batch size).
 *
 * TEST INFRASTRUCTURE ONLY: the product path never includes, links or calls
 * it.
 *
 * What it computes, in binary64 (one update on a mini-batch of B
 * transitions (s, a, r, s', done)):
 *   Q(x)    = W3 relu(W2 relu(W1 x + b1) + b2) + b3   (Sec. 4.3.2 network)
 *   a*_b    = argmax_a Q_online(s'_b)   (lowest index on ties; double DQN:
 *             the online network picks, the target network evaluates)
 *   y_b     = r_b + gamma (1 - done_b) Q_target(s'_b)[a*_b]
 *   delta_b = Q_online(s_b)[a_b] - y_b
 *   loss    = (1/B) sum_b huber(delta_b), huber(d) = d^2/2 for |d| <= k,
 *             k (|d| - k/2) otherwise; y is a constant (no gradient)
 *   gradients of the loss by back-propagation (relu'(0) = 0), then one Adam
 *   step on every weight and bias: m = b1 m + (1 - b1) g,
 *   v = b2 v + (1 - b2) g^2, w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 -
 *   b2^t)) + eps), t the update count; after every `target_every`-th update
 *   the target network becomes a copy of the online one.
 * Readings where the paper is silent: the Huber loss, Adam's beta1, beta2
 * and eps, relu'(0) = 0.
 * Weights: W_l row-major [out][in], concatenated [W1 | W2 | W3]; biases
 * [b1 | b2 | b3].
 */
#ifndef LEARNER_ORACLE_H
#define LEARNER_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double gamma, lr, beta1, beta2, adam_eps, huber_k;
  int32_t target_every;
} orc_learner_config;

typedef struct orc_learner orc_learner;

/* w, b: initial online weights (binary32, copied to binary64); the target
 * network starts as a copy. */
orc_learner *orc_learner_create(const int32_t dims[4], const float *w, const float *b,
                                const orc_learner_config *cfg);
void orc_learner_destroy(orc_learner *L);
/* One update. grad_w, grad_b (may be NULL) receive the gradients, loss the
 * mini-batch loss. Returns 0, or -1 for B < 1. */
int32_t orc_learner_update(orc_learner *L, int32_t B, const float *s, const int32_t *a,
                           const float *r, const float *s_next, const uint8_t *done,
                           double *loss, double *grad_w, double *grad_b);
/* Current parameters (binary64): online and target weights and biases. */
void orc_learner_get(const orc_learner *L, double *w, double *b, double *wt, double *bt);
int64_t orc_learner_steps(const orc_learner *L);
/* Forward pass of the online (which = 0) or target (1) network: q [n][A]. */
void orc_learner_q(const orc_learner *L, int32_t which, int32_t n, const float *x, double *q);

/* Time feedback mechanism (Sec. 3.1.2): the sharer keeps the mean period of
 * one vectorized step of the actor (V, sleep excluded) and of one update of
 * the learner (B); with rho = N TPS / B_batch, Eq. (TB2TV) asks V = rho B,
 * so xi = rho mean(B) - mean(V): the actor sleeps xi after a step when
 * xi > 0, the learner -xi / rho after an update otherwise. Means are over
 * every period recorded so far; xi is 0 until both have one. */
typedef struct {
  double rho, v_sum, b_sum;
  int64_t v_n, b_n;
} orc_tfm;
void orc_tfm_init(orc_tfm *t, double rho);
void orc_tfm_actor(orc_tfm *t, double seconds);
void orc_tfm_learner(orc_tfm *t, double seconds);
double orc_tfm_xi(const orc_tfm *t);

#ifdef __cplusplus
}
#endif
#endif
