/*
 * learner_oracle.c -- plain CPU oracle of the DDQN learner update (Alg. 2
 * step 2). TEST INFRASTRUCTURE ONLY. Definitions in learner_oracle.h.
 */
#include "learner_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

struct orc_learner {
  int32_t d0, h1, h2, A;
  size_t nw, nb;
  orc_learner_config cfg;
  double *w, *b, *wt, *bt;     /* online and target parameters */
  double *mw, *vw, *mb, *vb;   /* Adam moments */
  int64_t t;                   /* updates done */
};

static void forward(const orc_learner *L, const double *w, const double *b, const double *x,
                    double *z1, double *a1, double *z2, double *a2, double *q) {
  const int32_t d0 = L->d0, h1 = L->h1, h2 = L->h2, A = L->A;
  const double *W1 = w, *W2 = w + (size_t)h1 * d0, *W3 = W2 + (size_t)h2 * h1;
  const double *b1 = b, *b2 = b + h1, *b3 = b + h1 + h2;
  for (int32_t o = 0; o < h1; ++o) {
    double acc = b1[o];
    for (int32_t k = 0; k < d0; ++k) acc += W1[(size_t)o * d0 + k] * x[k];
    z1[o] = acc;
    a1[o] = acc > 0.0 ? acc : 0.0;
  }
  for (int32_t o = 0; o < h2; ++o) {
    double acc = b2[o];
    for (int32_t k = 0; k < h1; ++k) acc += W2[(size_t)o * h1 + k] * a1[k];
    z2[o] = acc;
    a2[o] = acc > 0.0 ? acc : 0.0;
  }
  for (int32_t o = 0; o < A; ++o) {
    double acc = b3[o];
    for (int32_t k = 0; k < h2; ++k) acc += W3[(size_t)o * h2 + k] * a2[k];
    q[o] = acc;
  }
}

orc_learner *orc_learner_create(const int32_t dims[4], const float *w, const float *b,
                                const orc_learner_config *cfg) {
  orc_learner *L = (orc_learner *)calloc(1, sizeof(orc_learner));
  if (!L) return NULL;
  L->d0 = dims[0];
  L->h1 = dims[1];
  L->h2 = dims[2];
  L->A = dims[3];
  L->nw = (size_t)L->h1 * L->d0 + (size_t)L->h2 * L->h1 + (size_t)L->A * L->h2;
  L->nb = (size_t)L->h1 + L->h2 + L->A;
  L->cfg = *cfg;
  double **bufs[8] = {&L->w, &L->b, &L->wt, &L->bt, &L->mw, &L->vw, &L->mb, &L->vb};
  const size_t sizes[8] = {L->nw, L->nb, L->nw, L->nb, L->nw, L->nw, L->nb, L->nb};
  for (int i = 0; i < 8; ++i) {
    *bufs[i] = (double *)calloc(sizes[i], sizeof(double));
    if (!*bufs[i]) {
      orc_learner_destroy(L);
      return NULL;
    }
  }
  for (size_t i = 0; i < L->nw; ++i) L->w[i] = L->wt[i] = (double)w[i];
  for (size_t i = 0; i < L->nb; ++i) L->b[i] = L->bt[i] = (double)b[i];
  return L;
}

void orc_learner_destroy(orc_learner *L) {
  if (!L) return;
  free(L->w); free(L->b); free(L->wt); free(L->bt);
  free(L->mw); free(L->vw); free(L->mb); free(L->vb);
  free(L);
}

int64_t orc_learner_steps(const orc_learner *L) { return L->t; }

void orc_learner_get(const orc_learner *L, double *w, double *b, double *wt, double *bt) {
  if (w) memcpy(w, L->w, sizeof(double) * L->nw);
  if (b) memcpy(b, L->b, sizeof(double) * L->nb);
  if (wt) memcpy(wt, L->wt, sizeof(double) * L->nw);
  if (bt) memcpy(bt, L->bt, sizeof(double) * L->nb);
}

void orc_learner_q(const orc_learner *L, int32_t which, int32_t n, const float *x, double *q) {
  const double *w = which ? L->wt : L->w, *b = which ? L->bt : L->b;
  double *xd = (double *)malloc(sizeof(double) * (size_t)L->d0);
  double *buf = (double *)malloc(sizeof(double) * 2 * (size_t)(L->h1 + L->h2));
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t k = 0; k < L->d0; ++k) xd[k] = (double)x[(size_t)i * L->d0 + k];
    forward(L, w, b, xd, buf, buf + L->h1, buf + 2 * L->h1, buf + 2 * L->h1 + L->h2,
            q + (size_t)i * L->A);
  }
  free(xd);
  free(buf);
}

static double huber(double d, double k) {
  const double a = fabs(d);
  return a <= k ? 0.5 * d * d : k * (a - 0.5 * k);
}
static double huber_grad(double d, double k) { return d > k ? k : (d < -k ? -k : d); }

int32_t orc_learner_update(orc_learner *L, int32_t B, const float *s, const int32_t *a,
                           const float *r, const float *s_next, const uint8_t *done,
                           double *loss, double *grad_w, double *grad_b) {
  if (B < 1) return -1;
  const int32_t d0 = L->d0, h1 = L->h1, h2 = L->h2, A = L->A;
  const double *W2 = L->w + (size_t)h1 * d0, *W3 = W2 + (size_t)h2 * h1;
  double *gw = (double *)calloc(L->nw, sizeof(double));
  double *gb = (double *)calloc(L->nb, sizeof(double));
  double *x = (double *)malloc(sizeof(double) * (size_t)d0);
  double *z1 = (double *)malloc(sizeof(double) * (size_t)h1);
  double *a1 = (double *)malloc(sizeof(double) * (size_t)h1);
  double *z2 = (double *)malloc(sizeof(double) * (size_t)h2);
  double *a2 = (double *)malloc(sizeof(double) * (size_t)h2);
  double *q = (double *)malloc(sizeof(double) * (size_t)A);
  double *qn = (double *)malloc(sizeof(double) * (size_t)A);
  double *qt = (double *)malloc(sizeof(double) * (size_t)A);
  double *d1 = (double *)malloc(sizeof(double) * (size_t)h1);
  double *d2 = (double *)malloc(sizeof(double) * (size_t)h2);
  double sum_loss = 0.0;
  double *gW1 = gw, *gW2 = gw + (size_t)h1 * d0, *gW3 = gW2 + (size_t)h2 * h1;
  double *gb1 = gb, *gb2 = gb + h1, *gb3 = gb + h1 + h2;
  for (int32_t i = 0; i < B; ++i) {
    /* the target: the online network picks a*, the target network values it */
    for (int32_t k = 0; k < d0; ++k) x[k] = (double)s_next[(size_t)i * d0 + k];
    forward(L, L->w, L->b, x, z1, a1, z2, a2, qn);
    forward(L, L->wt, L->bt, x, z1, a1, z2, a2, qt);
    int32_t best = 0;
    for (int32_t o = 1; o < A; ++o)
      if (qn[o] > qn[best]) best = o;
    const double y = (double)r[i] + L->cfg.gamma * (done[i] ? 0.0 : 1.0) * qt[best];
    /* the prediction, kept for back-propagation */
    for (int32_t k = 0; k < d0; ++k) x[k] = (double)s[(size_t)i * d0 + k];
    forward(L, L->w, L->b, x, z1, a1, z2, a2, q);
    const double delta = q[a[i]] - y;
    sum_loss += huber(delta, L->cfg.huber_k);
    const double g = huber_grad(delta, L->cfg.huber_k) / (double)B;  /* dloss/dQ[a_i] */
    const int32_t ai = a[i];
    /* layer 3 */
    gb3[ai] += g;
    for (int32_t k = 0; k < h2; ++k) gW3[(size_t)ai * h2 + k] += g * a2[k];
    for (int32_t k = 0; k < h2; ++k) d2[k] = z2[k] > 0.0 ? g * W3[(size_t)ai * h2 + k] : 0.0;
    /* layer 2 */
    for (int32_t o = 0; o < h2; ++o) {
      gb2[o] += d2[o];
      for (int32_t k = 0; k < h1; ++k) gW2[(size_t)o * h1 + k] += d2[o] * a1[k];
    }
    for (int32_t k = 0; k < h1; ++k) {
      double acc = 0.0;
      for (int32_t o = 0; o < h2; ++o) acc += d2[o] * W2[(size_t)o * h1 + k];
      d1[k] = z1[k] > 0.0 ? acc : 0.0;
    }
    /* layer 1 */
    for (int32_t o = 0; o < h1; ++o) {
      gb1[o] += d1[o];
      for (int32_t k = 0; k < d0; ++k) gW1[(size_t)o * d0 + k] += d1[o] * x[k];
    }
  }
  if (loss) *loss = sum_loss / (double)B;
  if (grad_w) memcpy(grad_w, gw, sizeof(double) * L->nw);
  if (grad_b) memcpy(grad_b, gb, sizeof(double) * L->nb);
  /* Adam */
  L->t += 1;
  const double c1 = 1.0 - pow(L->cfg.beta1, (double)L->t);
  const double c2 = 1.0 - pow(L->cfg.beta2, (double)L->t);
  for (int pass = 0; pass < 2; ++pass) {
    double *p = pass ? L->b : L->w, *m = pass ? L->mb : L->mw, *v = pass ? L->vb : L->vw;
    const double *gg = pass ? gb : gw;
    const size_t n = pass ? L->nb : L->nw;
    for (size_t i = 0; i < n; ++i) {
      m[i] = L->cfg.beta1 * m[i] + (1.0 - L->cfg.beta1) * gg[i];
      v[i] = L->cfg.beta2 * v[i] + (1.0 - L->cfg.beta2) * gg[i] * gg[i];
      p[i] -= L->cfg.lr * (m[i] / c1) / (sqrt(v[i] / c2) + L->cfg.adam_eps);
    }
  }
  if (L->cfg.target_every > 0 && L->t % L->cfg.target_every == 0) {
    memcpy(L->wt, L->w, sizeof(double) * L->nw);
    memcpy(L->bt, L->b, sizeof(double) * L->nb);
  }
  free(gw); free(gb); free(x); free(z1); free(a1); free(z2); free(a2);
  free(q); free(qn); free(qt); free(d1); free(d2);
  return 0;
}

void orc_tfm_init(orc_tfm *t, double rho) {
  memset(t, 0, sizeof(*t));
  t->rho = rho;
}
void orc_tfm_actor(orc_tfm *t, double seconds) {
  t->v_sum += seconds;
  t->v_n += 1;
}
void orc_tfm_learner(orc_tfm *t, double seconds) {
  t->b_sum += seconds;
  t->b_n += 1;
}
double orc_tfm_xi(const orc_tfm *t) {
  if (t->v_n == 0 || t->b_n == 0) return 0.0;
  return t->rho * (t->b_sum / (double)t->b_n) - t->v_sum / (double)t->v_n;
}
