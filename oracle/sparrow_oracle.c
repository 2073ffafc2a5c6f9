/*
 * sparrow_oracle.c -- plain CPU oracle of the vectorized Sparrow step.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline). See the header
 * for what it computes and which passages of arXiv 2305.04180 it follows.
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fPIC -shared -lm
 */
#include "sparrow_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Constants, each rounded once from double.                                 */
/* ------------------------------------------------------------------------ */
#define PI_D 3.14159265358979323846
static const float PI_F = (float)PI_D;
static const float TWO_PI_F = (float)(2.0 * PI_D);
static const float TWO_OVER_PI_F = (float)(2.0 / PI_D);
static const float TWO_M24 = 5.9604644775390625e-08f; /* 2^-24 */

/* Action table (Sec. 4.3.1 lists five target velocities as fractions of the
 * maximal linear velocity and +-1 rad/s; ids {0,1,3,5,6} are those five, ids
 * 2 and 4 add half turns). Entries: (A_v, A_w). */
static const float ACT_V[7] = {0.02f, 1.0f, 1.0f, 1.0f, 1.0f, 1.0f, 0.02f};
static const float ACT_W[7] = {1.0f, 1.0f, 0.5f, 0.0f, -0.5f, -1.0f, -1.0f};
/* The five actions of Sec. 4.3.1 in the order listed there (turn left, go
 * straight and turn left, go straight, go straight and turn right, turn
 * right) as rows of the table above. */
static const int32_t FIVE_ACTIONS[5] = {0, 1, 3, 5, 6};

struct orc_env {
  orc_config cfg;
  int32_t n_maps;
  uint8_t *cells;
  int64_t *offsets;
  int32_t *W, *H;
  float *inv_dn; /* per map: 1 / (sqrt(2) * max(W, H)) */
  int32_t *env_map;
  float *ray_c, *ray_s; /* cos / sin of each ray's offset from forward */
  int32_t M;            /* samples k = 0..M */
  float inv_R;
  orc_task task;
  float inv_D;          /* 1 / plan_dist, rounded once */
  float near_r;         /* robot_r + near_dist (binary32 sum) */
  uint32_t g;           /* global step counter */
  int32_t status;
  /* state */
  float *x, *y, *phi, *vl, *va, *tx, *ty, *dprev, *dt, *K, *mu, *vmax, *sigma;
  int32_t *t, *delay, *q0, *q1;
};

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplications,    */
/* a word permutation and a Weyl-sequence key schedule.                      */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += W0;
    k1 += W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(const orc_env *e, uint32_t env, uint32_t purpose, uint32_t sub,
                 uint32_t w[4]) {
  uint32_t ctr[4] = {env, e->g, purpose, sub};
  uint32_t key[2] = {(uint32_t)e->cfg.seed, (uint32_t)(e->cfg.seed >> 32)};
  orc_philox4x32_10(ctr, key, w);
}

/* 24-bit uniform in [0, 1): exact in binary32 */
static float unit24(uint32_t w) { return (float)(w >> 8) * TWO_M24; }
/* floor(w * n / 2^32): an integer in [0, n) */
static int32_t scale_u32(uint32_t w, uint32_t n) {
  return (int32_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

/* ------------------------------------------------------------------------ */
/* sincos_f32: Cody & Waite (1980) three-part reduction by pi/2, then Taylor */
/* polynomials of sin to r^11 and cos to r^10 with coefficients +-1/n!.      */
/* ------------------------------------------------------------------------ */
static float clear_low12(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  u &= ~0xFFFu;
  memcpy(&f, &u, 4);
  return f;
}

void orc_sincos_f32(float phi, float *s_out, float *c_out) {
  const float C1 = clear_low12((float)(PI_D / 2.0));
  const float C2 = clear_low12((float)(PI_D / 2.0 - (double)C1));
  const float C3 = (float)(PI_D / 2.0 - (double)C1 - (double)C2);
  const float S1 = (float)(-1.0 / 6.0), S2 = (float)(1.0 / 120.0),
              S3 = (float)(-1.0 / 5040.0), S4 = (float)(1.0 / 362880.0),
              S5 = (float)(-1.0 / 39916800.0);
  const float K1 = (float)(-1.0 / 2.0), K2 = (float)(1.0 / 24.0),
              K3 = (float)(-1.0 / 720.0), K4 = (float)(1.0 / 40320.0),
              K5 = (float)(-1.0 / 3628800.0);
  float kq = rintf(phi * TWO_OVER_PI_F);
  int32_t k = (int32_t)kq;
  float r = phi - kq * C1;
  r = r - kq * C2;
  r = r - kq * C3;
  float r2 = r * r;
  float ps = S5;
  ps = ps * r2 + S4;
  ps = ps * r2 + S3;
  ps = ps * r2 + S2;
  ps = ps * r2 + S1;
  float r3 = r * r2;
  float s = r + r3 * ps;
  float pc = K5;
  pc = pc * r2 + K4;
  pc = pc * r2 + K3;
  pc = pc * r2 + K2;
  pc = pc * r2 + K1;
  float c = 1.0f + r2 * pc;
  switch (k & 3) {
    case 0: *s_out = s; *c_out = c; break;
    case 1: *s_out = c; *c_out = -s; break;
    case 2: *s_out = -s; *c_out = -c; break;
    default: *s_out = -c; *c_out = s; break;
  }
}

/* ------------------------------------------------------------------------ */
/* Occupancy grid. Cells outside the map count as occupied.                  */
/* ------------------------------------------------------------------------ */
static int occupied(const orc_env *e, int32_t m, int32_t ix, int32_t iy) {
  if (ix < 0 || iy < 0 || ix >= e->W[m] || iy >= e->H[m]) return 1;
  return e->cells[e->offsets[m] + (int64_t)iy * e->W[m] + ix] != 0;
}

/* Collision (Sec. 3.2): the robot disk of radius r against every occupied
 * cell square [i, i+1] x [j, j+1] that meets the disk's bounding box
 * [x - r, x + r] (closed: i from ceil(x - r) - 1 to floor(x + r)); touching
 * (distance <= r) collides. */
static int32_t disk_hits(const orc_env *e, int32_t m, float px, float py, float r) {
  const float r2 = r * r;
  int32_t i0 = (int32_t)ceilf(px - r) - 1, i1 = (int32_t)floorf(px + r);
  int32_t j0 = (int32_t)ceilf(py - r) - 1, j1 = (int32_t)floorf(py + r);
  for (int32_t j = j0; j <= j1; ++j) {
    for (int32_t i = i0; i <= i1; ++i) {
      if (!occupied(e, m, i, j)) continue;
      float fi = (float)i, fj = (float)j;
      float dx = fmaxf(fmaxf(fi - px, 0.0f), px - (fi + 1.0f));
      float dy = fmaxf(fmaxf(fj - py, 0.0f), py - (fj + 1.0f));
      float d2 = dx * dx + dy * dy;
      if (d2 <= r2) return 1;
    }
  }
  return 0;
}

int32_t orc_collides(const orc_env *e, int32_t m, float px, float py) {
  return disk_hits(e, m, px, py, e->cfg.robot_r);
}

int32_t orc_near(const orc_env *e, int32_t m, float px, float py) {
  return disk_hits(e, m, px, py, e->near_r);
}

/* LiDAR ray (Sec. 3.2 ray casting on the grid): samples at t_k = k * ds for
 * k = 0..M along unit direction u; the first sample whose cell is occupied or
 * outside the map is the hit. Returns k_hit, or -1 when nothing is hit. */
int32_t orc_march(const orc_env *e, int32_t m, float x, float y, float ux, float uy) {
  const float W = (float)e->W[m], H = (float)e->H[m];
  for (int32_t k = 0; k <= e->M; ++k) {
    float tk = (float)k * e->cfg.ds;
    float px = x + tk * ux;
    float py = y + tk * uy;
    if (!(px >= 0.0f && px < W && py >= 0.0f && py < H)) return k;
    int32_t ix = (int32_t)floorf(px), iy = (int32_t)floorf(py);
    if (occupied(e, m, ix, iy)) return k;
  }
  return -1;
}

void orc_ray_table(const orc_env *e, float *c, float *s) {
  for (int32_t j = 0; j < e->cfg.n_rays; ++j) {
    c[j] = e->ray_c[j];
    s[j] = e->ray_s[j];
  }
}

/* ------------------------------------------------------------------------ */
/* create / destroy                                                          */
/* ------------------------------------------------------------------------ */
static void *xcalloc(size_t n, size_t sz) { return calloc(n ? n : 1, sz); }

orc_env *orc_create(const orc_config *cfg, int32_t n_maps, const uint8_t *cells,
                    const int64_t *offsets, const int32_t *width,
                    const int32_t *height, const int32_t *env_to_map) {
  if (!cfg || !cells || !offsets || !width || !height || !env_to_map) return NULL;
  if (cfg->n_envs <= 0 || cfg->n_rays <= 0 || cfg->n_actions != ORC_NACT || n_maps <= 0)
    return NULL;
  orc_env *e = (orc_env *)xcalloc(1, sizeof(orc_env));
  e->cfg = *cfg;
  e->n_maps = n_maps;
  int64_t total = 0;
  e->offsets = (int64_t *)xcalloc((size_t)n_maps, sizeof(int64_t));
  e->W = (int32_t *)xcalloc((size_t)n_maps, sizeof(int32_t));
  e->H = (int32_t *)xcalloc((size_t)n_maps, sizeof(int32_t));
  e->inv_dn = (float *)xcalloc((size_t)n_maps, sizeof(float));
  for (int32_t m = 0; m < n_maps; ++m) {
    e->W[m] = width[m];
    e->H[m] = height[m];
    e->offsets[m] = total;
    total += (int64_t)width[m] * height[m];
    int32_t side = width[m] > height[m] ? width[m] : height[m];
    e->inv_dn[m] = (float)(1.0 / (sqrt(2.0) * (double)side));
  }
  e->cells = (uint8_t *)xcalloc((size_t)total, 1);
  for (int32_t m = 0; m < n_maps; ++m)
    memcpy(e->cells + e->offsets[m], cells + offsets[m], (size_t)width[m] * height[m]);
  int32_t n = cfg->n_envs;
  e->env_map = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
  memcpy(e->env_map, env_to_map, sizeof(int32_t) * (size_t)n);
  /* ray offsets: endpoints of the field of view included, n-1 intervals */
  int32_t nr = cfg->n_rays;
  e->ray_c = (float *)xcalloc((size_t)nr, sizeof(float));
  e->ray_s = (float *)xcalloc((size_t)nr, sizeof(float));
  for (int32_t j = 0; j < nr; ++j) {
    double fov = (double)cfg->fov;
    double th = nr > 1 ? -fov / 2.0 + (double)j * fov / (double)(nr - 1) : 0.0;
    e->ray_c[j] = (float)cos(th);
    e->ray_s[j] = (float)sin(th);
  }
  e->M = (int32_t)floor((double)cfg->range / (double)cfg->ds);
  e->inv_R = (float)(1.0 / (double)cfg->range);
  float **fs[] = {&e->x, &e->y, &e->phi, &e->vl, &e->va, &e->tx, &e->ty,
                  &e->dprev, &e->dt, &e->K, &e->mu, &e->vmax, &e->sigma};
  for (size_t f = 0; f < sizeof(fs) / sizeof(fs[0]); ++f)
    *fs[f] = (float *)xcalloc((size_t)n, sizeof(float));
  int32_t **is[] = {&e->t, &e->delay, &e->q0, &e->q1};
  for (size_t f = 0; f < sizeof(is) / sizeof(is[0]); ++f)
    *is[f] = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
  orc_task t = {ORC_NACT, ORC_REWARD_PROGRESS, ORC_STATE_TARGET, 10.0f, -10.0f, 1.0f, 0.0f,
                0.3f, 0.1f, 0.3f, 0.3f, 0.1f};
  orc_set_task(e, &t);
  return e;
}

int32_t orc_set_task(orc_env *e, const orc_task *t) {
  if (!e || !t) return ORC_EINVAL;
  if ((t->n_actions != 5 && t->n_actions != 7) || t->reward < 0 || t->reward > 1 ||
      t->state < 0 || t->state > 1 || !(t->plan_dist > 0.0f) || !(t->near_dist >= 0.0f))
    return ORC_EINVAL;
  e->task = *t;
  e->inv_D = (float)(1.0 / (double)t->plan_dist);
  e->near_r = e->cfg.robot_r + t->near_dist;
  return ORC_OK;
}

void orc_destroy(orc_env *e) {
  if (!e) return;
  free(e->cells); free(e->offsets); free(e->W); free(e->H); free(e->inv_dn);
  free(e->env_map); free(e->ray_c); free(e->ray_s);
  free(e->x); free(e->y); free(e->phi); free(e->vl); free(e->va); free(e->tx);
  free(e->ty); free(e->dprev); free(e->dt); free(e->K); free(e->mu);
  free(e->vmax); free(e->sigma); free(e->t); free(e->delay); free(e->q0);
  free(e->q1);
  free(e);
}

int32_t orc_status(const orc_env *e) { return e->status; }
uint32_t orc_global_step(const orc_env *e) { return e->g; }
void orc_set_global_step(orc_env *e, uint32_t g) { e->g = g; }
int32_t orc_obs_dim(const orc_env *e) { return e->cfg.n_rays + 4 + e->task.state; }
void orc_advance(orc_env *e) { e->g += 1u; }

void orc_get_state(const orc_env *e, float *f, int32_t *iv) {
  for (int32_t i = 0; i < e->cfg.n_envs; ++i) {
    float *r = f + (size_t)i * ORC_NF;
    r[0] = e->x[i]; r[1] = e->y[i]; r[2] = e->phi[i]; r[3] = e->vl[i];
    r[4] = e->va[i]; r[5] = e->tx[i]; r[6] = e->ty[i]; r[7] = e->dprev[i];
    r[8] = e->dt[i]; r[9] = e->K[i]; r[10] = e->mu[i]; r[11] = e->vmax[i];
    r[12] = e->sigma[i];
    int32_t *q = iv + (size_t)i * ORC_NI;
    q[0] = e->t[i]; q[1] = e->delay[i]; q[2] = e->q0[i]; q[3] = e->q1[i];
  }
}

void orc_set_state(orc_env *e, const float *f, const int32_t *iv) {
  for (int32_t i = 0; i < e->cfg.n_envs; ++i) {
    const float *r = f + (size_t)i * ORC_NF;
    e->x[i] = r[0]; e->y[i] = r[1]; e->phi[i] = r[2]; e->vl[i] = r[3];
    e->va[i] = r[4]; e->tx[i] = r[5]; e->ty[i] = r[6]; e->dprev[i] = r[7];
    e->dt[i] = r[8]; e->K[i] = r[9]; e->mu[i] = r[10]; e->vmax[i] = r[11];
    e->sigma[i] = r[12];
    const int32_t *q = iv + (size_t)i * ORC_NI;
    e->t[i] = q[0]; e->delay[i] = q[1]; e->q0[i] = q[2]; e->q1[i] = q[3];
  }
}

/* ------------------------------------------------------------------------ */
/* AutoReset with per-episode domain randomisation (Sec. 3.2.4, 3.2.5).      */
/* ------------------------------------------------------------------------ */
static int32_t reset_env(orc_env *e, int32_t i) {
  const orc_config *c = &e->cfg;
  const int32_t m = e->env_map[i];
  uint32_t a[4], b[4];
  draw(e, (uint32_t)i, ORC_P_RESET_DR, 0, a);
  draw(e, (uint32_t)i, ORC_P_RESET_DR, 1, b);
  e->dt[i] = c->dt_lo + (c->dt_hi - c->dt_lo) * unit24(a[0]);
  e->K[i] = c->K_lo + (c->K_hi - c->K_lo) * unit24(a[1]);
  e->mu[i] = c->mu_lo + (c->mu_hi - c->mu_lo) * unit24(a[2]);
  e->vmax[i] = c->vmax_lo + (c->vmax_hi - c->vmax_lo) * unit24(a[3]);
  e->sigma[i] = c->sigma_lo + (c->sigma_hi - c->sigma_lo) * unit24(b[0]);
  e->delay[i] = c->delay_lo + scale_u32(b[1], (uint32_t)(c->delay_hi - c->delay_lo + 1));
  e->phi[i] = unit24(b[2]) * TWO_PI_F - PI_F;

  const uint32_t W = (uint32_t)e->W[m], H = (uint32_t)e->H[m];
  const float ra2 = c->arrive_r * c->arrive_r;
  int32_t rc = ORC_OK;
  /* start: the first collision-free candidate cell centre in counter order */
  float sx = 0, sy = 0;
  int found = 0;
  for (uint32_t n = 0; n < 16u * 64u && !found; ++n) {
    uint32_t w[4];
    draw(e, (uint32_t)i, ORC_P_RESET_START, n, w);
    float px = (float)scale_u32(w[0], W) + 0.5f;
    float py = (float)scale_u32(w[1], H) + 0.5f;
    if (n == 0) { sx = px; sy = py; }
    if (!orc_collides(e, m, px, py)) { sx = px; sy = py; found = 1; }
  }
  if (!found) rc = ORC_ERESET;
  /* target: same scheme, also farther than the arrival radius */
  float gx = 0, gy = 0;
  found = 0;
  for (uint32_t n = 0; n < 16u * 64u && !found; ++n) {
    uint32_t w[4];
    draw(e, (uint32_t)i, ORC_P_RESET_TARGET, n, w);
    float px = (float)scale_u32(w[0], W) + 0.5f;
    float py = (float)scale_u32(w[1], H) + 0.5f;
    if (n == 0) { gx = px; gy = py; }
    float dx = px - sx, dy = py - sy;
    float d2 = dx * dx + dy * dy;
    if (!orc_collides(e, m, px, py) && d2 > ra2) { gx = px; gy = py; found = 1; }
  }
  if (!found) rc = ORC_ERESET;
  e->x[i] = sx; e->y[i] = sy; e->tx[i] = gx; e->ty[i] = gy;
  e->vl[i] = 0.0f; e->va[i] = 0.0f; e->t[i] = 0;
  e->q0[i] = ORC_STOP; e->q1[i] = ORC_STOP;
  float dx = gx - sx, dy = gy - sy;
  e->dprev[i] = sqrtf(dx * dx + dy * dy);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Observation: normalised ranges, velocities, target distance and bearing   */
/* relative to the robot (Sec. 3.2.1 built-in normalisation; Sec. 4.3.1).    */
/* ------------------------------------------------------------------------ */
static void observe(const orc_env *e, int32_t i, uint32_t noise_purpose, float *o,
                    int16_t *hit_k, orc_stats *st) {
  const orc_config *c = &e->cfg;
  const int32_t m = e->env_map[i];
  const int32_t nr = c->n_rays;
  float s, co;
  orc_sincos_f32(e->phi[i], &s, &co);
  const float fx = -co, fy = -s; /* forward = direction of motion in Eq. (6) */
  for (int32_t j = 0; j < nr; ++j) {
    float ux = fx * e->ray_c[j] - fy * e->ray_s[j];
    float uy = fy * e->ray_c[j] + fx * e->ray_s[j];
    int32_t kh = orc_march(e, m, e->x[i], e->y[i], ux, uy);
    float d = kh < 0 ? c->range : (float)kh * c->ds;
    if (hit_k) hit_k[j] = (int16_t)kh;
    if (st) {
      int32_t last = kh < 0 ? e->M : kh;
      st->samples += (uint64_t)(last + 1);
      st->rays += 1;
      /* FP64 shadow of the same samples: count cell-boundary ties */
      double ph = (double)e->phi[i];
      double fxd = -cos(ph), fyd = -sin(ph);
      double th = nr > 1 ? -(double)c->fov / 2.0 + (double)j * (double)c->fov / (double)(nr - 1)
                         : 0.0;
      double uxd = fxd * cos(th) - fyd * sin(th), uyd = fyd * cos(th) + fxd * sin(th);
      for (int32_t k = 0; k <= last; ++k) {
        float tk = (float)k * c->ds;
        float px = e->x[i] + tk * ux, py = e->y[i] + tk * uy;
        double pxd = (double)e->x[i] + (double)k * (double)c->ds * uxd;
        double pyd = (double)e->y[i] + (double)k * (double)c->ds * uyd;
        if (floorf(px) != floor(pxd) || floorf(py) != floor(pyd)) st->ties_ray += 1;
      }
    }
    /* sensor noise (Sec. 3.2): additive Gaussian, Box-Muller in FP64 */
    uint32_t w[4];
    draw(e, (uint32_t)i, noise_purpose, (uint32_t)j, w);
    double u1 = (double)((w[0] >> 8) + 1u) * 0x1p-24;
    double u2 = (double)(w[1] >> 8) * 0x1p-24;
    float z = (float)(sqrt(-2.0 * log(u1)) * cos(2.0 * PI_D * u2));
    float dn = d + e->sigma[i] * z;
    dn = fminf(fmaxf(dn, 0.0f), c->range);
    o[j] = dn * e->inv_R;
  }
  float dx = e->tx[i] - e->x[i], dy = e->ty[i] - e->y[i];
  float bx = dx * fx + dy * fy; /* target in the robot frame */
  float by = dy * fx - dx * fy;
  float bearing = (float)(atan2((double)by, (double)bx) / PI_D);
  if (e->task.state == ORC_STATE_TARGET) {
    o[nr] = e->vl[i] / e->vmax[i];
    o[nr + 1] = e->va[i] / c->omega_max;
    float d2 = dx * dx + dy * dy;
    o[nr + 2] = sqrtf(d2) * e->inv_dn[m];
    o[nr + 3] = bearing;
  } else {
    /* Sec. 4.3.1 relative pose: the robot's position relative to the target
     * over the planning distance D, its orientation relative to the
     * direction of the target (alpha / pi), then the two velocities */
    o[nr] = (e->x[i] - e->tx[i]) * e->inv_D;
    o[nr + 1] = (e->y[i] - e->ty[i]) * e->inv_D;
    o[nr + 2] = bearing;
    o[nr + 3] = e->vl[i] / e->vmax[i];
    o[nr + 4] = e->va[i] / c->omega_max;
  }
}

int32_t orc_reset(orc_env *e, float *obs, int16_t *hit_k) {
  const int32_t n = e->cfg.n_envs, D = orc_obs_dim(e), nr = e->cfg.n_rays;
  int32_t rc = ORC_OK;
  for (int32_t i = 0; i < n; ++i) {
    if (reset_env(e, i) != ORC_OK) rc = ORC_ERESET;
    observe(e, i, ORC_P_NOISE_RESET, obs + (size_t)i * D, hit_k ? hit_k + (size_t)i * nr : NULL,
            NULL);
  }
  if (rc != ORC_OK) e->status = rc;
  orc_advance(e);
  return rc;
}

static double rel_err(double a, double b, double scale) {
  double den = fabs(b) > scale ? fabs(b) : scale;
  return fabs(a - b) / den;
}

/* ------------------------------------------------------------------------ */
/* Eq. (11) of Sec. 4.3.1 for a step that did not end the episode, at the    */
/* post-step pose:                                                           */
/*   r = w_d1 r_d1 + w_d2 r_d2 + w_v r_v + w_alpha r_alpha + w_d r_d         */
/* r_d1 = max(1 - d1 / D, 0), r_d2 = max(1 - d2 / D, 0) with d1 = |x - tx|,  */
/* d2 = |y - ty| (largest value 1, falling with the distance);               */
/* r_v = 1 if v_l > v_max / 2, else 0; r_alpha = 1 - |alpha| / pi, alpha the */
/* orientation relative to the direction of the target; r_d = -1 if an       */
/* occupied cell lies within near_dist of the robot's edge (within           */
/* robot_r + near_dist of its centre, touching included), else 0. Binary32   */
/* in this order; alpha / pi as in the observation (FP64, rounded once).     */
/* ------------------------------------------------------------------------ */
static float eq11_reward(const orc_env *e, int32_t i, int32_t m) {
  const orc_task *t = &e->task;
  const float x = e->x[i], y = e->y[i];
  const float d1 = fabsf(x - e->tx[i]), d2 = fabsf(y - e->ty[i]);
  const float rd1 = fmaxf(1.0f - d1 * e->inv_D, 0.0f);
  const float rd2 = fmaxf(1.0f - d2 * e->inv_D, 0.0f);
  const float rv = e->vl[i] > 0.5f * e->vmax[i] ? 1.0f : 0.0f;
  float s, co;
  orc_sincos_f32(e->phi[i], &s, &co);
  const float fx = -co, fy = -s;
  const float dx = e->tx[i] - x, dy = e->ty[i] - y;
  const float bx = dx * fx + dy * fy, by = dy * fx - dx * fy;
  const float alpha = (float)(atan2((double)by, (double)bx) / PI_D);
  const float ra = 1.0f - fabsf(alpha);
  const float rd = orc_near(e, m, x, y) ? -1.0f : 0.0f;
  float r = t->w_d1 * rd1;
  r = r + t->w_d2 * rd2;
  r = r + t->w_v * rv;
  r = r + t->w_alpha * ra;
  r = r + t->w_d * rd;
  return r;
}

/* ------------------------------------------------------------------------ */
/* One step of env i (Alg. 1 step 4: s', r, done = envs.step(a_hat)).        */
/* ------------------------------------------------------------------------ */
static int32_t step_env(orc_env *e, int32_t i, int32_t a_hat, float *o, float *reward,
                        uint8_t *done, uint8_t *flags, float *final_o, int16_t *hit_k,
                        orc_stats *st) {
  const orc_config *c = &e->cfg;
  const int32_t m = e->env_map[i];
  if (a_hat < 0 || a_hat >= e->task.n_actions) a_hat = ORC_STOP;
  else if (e->task.n_actions == 5) a_hat = FIVE_ACTIONS[a_hat];
  /* control delay: a FIFO of depth 0..2 holding not-yet-applied actions */
  int32_t a;
  if (e->delay[i] == 0) {
    a = a_hat;
  } else if (e->delay[i] == 1) {
    a = e->q0[i];
    e->q0[i] = a_hat;
  } else {
    a = e->q0[i];
    e->q0[i] = e->q1[i];
    e->q1[i] = a_hat;
  }
  /* target velocity of the applied action, scaled by the friction gain */
  float cl = 0.0f, ca = 0.0f;
  if (a != ORC_STOP) {
    cl = e->mu[i] * (ACT_V[a] * e->vmax[i]);
    ca = e->mu[i] * (ACT_W[a] * c->omega_max);
  }
  /* FP64 shadow inputs, taken before the update */
  const double x0 = e->x[i], y0 = e->y[i], p0 = e->phi[i], vl0 = e->vl[i], va0 = e->va[i];
  /* Eq. (5): velocity blend, then the velocity limits */
  const float K = e->K[i];
  const float omk = 1.0f - K;
  float vl = K * e->vl[i] + omk * cl;
  float va = K * e->va[i] + omk * ca;
  vl = fminf(fmaxf(vl, -e->vmax[i]), e->vmax[i]);
  va = fminf(fmaxf(va, -c->omega_max), c->omega_max);
  /* Eq. (6): pose with the new velocity and the old heading */
  float s, co;
  orc_sincos_f32(e->phi[i], &s, &co);
  const float dt = e->dt[i];
  float x = e->x[i] - dt * (vl * co);
  float y = e->y[i] - dt * (vl * s);
  float phi = e->phi[i] + dt * va;
  if (phi > PI_F) phi -= TWO_PI_F;
  else if (phi <= -PI_F) phi += TWO_PI_F;
  e->x[i] = x; e->y[i] = y; e->phi[i] = phi; e->vl[i] = vl; e->va[i] = va;
  e->t[i] += 1;

  if (st) {
    double Kd = K, cld = cl, cad = ca, vmd = e->vmax[i], wmd = c->omega_max;
    double vld = Kd * vl0 + (1.0 - Kd) * cld;
    double vad = Kd * va0 + (1.0 - Kd) * cad;
    vld = fmin(fmax(vld, -vmd), vmd);
    vad = fmin(fmax(vad, -wmd), wmd);
    double xd = x0 - (double)dt * vld * cos(p0);
    double yd = y0 - (double)dt * vld * sin(p0);
    double pd = p0 + (double)dt * vad;
    double dphi = (double)phi - pd;
    while (dphi > PI_D) dphi -= 2.0 * PI_D;
    while (dphi < -PI_D) dphi += 2.0 * PI_D;
    double ex = rel_err(x, xd, 1.0), ey = rel_err(y, yd, 1.0);
    double ep = fabs(dphi) / (fabs(pd) > 1.0 ? fabs(pd) : 1.0);
    double ev = rel_err(vl, vld, vmd), ew = rel_err(va, vad, wmd);
    if (ex > st->max_rel_x) st->max_rel_x = ex;
    if (ey > st->max_rel_y) st->max_rel_y = ey;
    if (ep > st->max_rel_phi) st->max_rel_phi = ep;
    if (ev > st->max_rel_vl) st->max_rel_vl = ev;
    if (ew > st->max_rel_va) st->max_rel_va = ew;
    st->kin_steps += 1;
  }

  /* collision, arrival, reward (Sec. 4.3.1: terminal -10 / +reward) */
  int32_t coll = orc_collides(e, m, x, y);
  if (st) {
    /* FP64 collision decision for the tie counter */
    double r = c->robot_r;
    int cd = 0;
    for (int32_t j = (int32_t)ceil((double)y - r) - 1; j <= (int32_t)floor((double)y + r) && !cd; ++j)
      for (int32_t ii = (int32_t)ceil((double)x - r) - 1; ii <= (int32_t)floor((double)x + r); ++ii) {
        if (!occupied(e, m, ii, j)) continue;
        double ddx = fmax(fmax(ii - (double)x, 0.0), (double)x - (ii + 1));
        double ddy = fmax(fmax(j - (double)y, 0.0), (double)y - (j + 1));
        if (ddx * ddx + ddy * ddy <= r * r) { cd = 1; break; }
      }
    if (cd != coll) st->ties_coll += 1;
  }
  float dx = e->tx[i] - x, dy = e->ty[i] - y;
  float d2 = dx * dx + dy * dy;
  int32_t arrived = d2 <= c->arrive_r * c->arrive_r;
  int32_t term = 0;
  float r;
  if (coll) {
    r = e->task.collide_reward;
    term = 1;
  } else if (arrived) {
    r = e->task.arrive_reward;
    term = 1;
  } else if (e->task.reward == ORC_REWARD_PROGRESS) {
    float dist = sqrtf(d2);
    r = (e->dprev[i] - dist) - 0.01f;
    e->dprev[i] = dist;
  } else {
    r = eq11_reward(e, i, m);
    e->dprev[i] = sqrtf(d2);
  }
  int32_t trunc = !term && e->t[i] >= c->t_max;
  int32_t dn = term || trunc;
  uint8_t fl = (uint8_t)((term ? ORC_F_TERM : 0) | (trunc ? ORC_F_TRUNC : 0) |
                         (coll ? ORC_F_COLL : 0) | (arrived && !coll ? ORC_F_ARRIVE : 0));
  *reward = r;
  *done = (uint8_t)dn;
  if (flags) *flags = fl;
  int32_t rc = ORC_OK;
  if (dn) {
    if (final_o) observe(e, i, ORC_P_NOISE, final_o, NULL, NULL);
    rc = reset_env(e, i);
    observe(e, i, ORC_P_NOISE_RESET, o, hit_k, st);
  } else {
    observe(e, i, ORC_P_NOISE, o, hit_k, st);
  }
  return rc;
}

int32_t orc_step_range(orc_env *e, int32_t e0, int32_t e1, const int32_t *actions,
                       float *obs, float *reward, uint8_t *done, uint8_t *flags,
                       float *final_obs, int16_t *hit_k, orc_stats *stats) {
  const int32_t D = orc_obs_dim(e), nr = e->cfg.n_rays;
  if (e0 < 0 || e1 > e->cfg.n_envs || e0 > e1) return ORC_EINVAL;
  int32_t rc = ORC_OK;
  for (int32_t i = e0; i < e1; ++i) {
    int32_t r = step_env(e, i, actions[i], obs + (size_t)i * D, reward + i, done + i,
                         flags ? flags + i : NULL,
                         final_obs ? final_obs + (size_t)i * D : NULL,
                         hit_k ? hit_k + (size_t)i * nr : NULL, stats);
    if (r != ORC_OK) rc = r;
  }
  if (rc != ORC_OK) e->status = rc;
  return rc;
}

int32_t orc_step(orc_env *e, const int32_t *actions, float *obs, float *reward,
                 uint8_t *done, uint8_t *flags, float *final_obs, int16_t *hit_k,
                 orc_stats *stats) {
  int32_t rc = orc_step_range(e, 0, e->cfg.n_envs, actions, obs, reward, done, flags,
                              final_obs, hit_k, stats);
  orc_advance(e);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Actor: Q-network forward (Sec. 4.3.2) and VEM (Sec. 3.1.1).              */
/* ------------------------------------------------------------------------ */
uint16_t orc_bf16_rne(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40u); /* NaN */
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return (uint16_t)(u >> 16);
}

static double bf16_to_f64(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return (double)f;
}

static double round_bf16_d(double v) { return bf16_to_f64(orc_bf16_rne((float)v)); }

void orc_qnet_f64(const int32_t dims[4], const uint16_t *w, const float *b, int32_t n,
                  const float *obs, int32_t round_act, double *q) {
  const int32_t d0 = dims[0], h1 = dims[1], h2 = dims[2], A = dims[3];
  const uint16_t *W1 = w, *W2 = w + (size_t)h1 * d0, *W3 = W2 + (size_t)h2 * h1;
  const float *b1 = b, *b2 = b + h1, *b3 = b + h1 + h2;
  double *x0 = (double *)malloc(sizeof(double) * (size_t)d0);
  double *a1 = (double *)malloc(sizeof(double) * (size_t)h1);
  double *a2 = (double *)malloc(sizeof(double) * (size_t)h2);
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t k = 0; k < d0; ++k) x0[k] = bf16_to_f64(orc_bf16_rne(obs[(size_t)i * d0 + k]));
    for (int32_t o = 0; o < h1; ++o) {
      double acc = (double)b1[o];
      for (int32_t k = 0; k < d0; ++k) acc += bf16_to_f64(W1[(size_t)o * d0 + k]) * x0[k];
      acc = acc > 0.0 ? acc : 0.0;
      a1[o] = round_act ? round_bf16_d(acc) : acc;
    }
    for (int32_t o = 0; o < h2; ++o) {
      double acc = (double)b2[o];
      for (int32_t k = 0; k < h1; ++k) acc += bf16_to_f64(W2[(size_t)o * h1 + k]) * a1[k];
      acc = acc > 0.0 ? acc : 0.0;
      a2[o] = round_act ? round_bf16_d(acc) : acc;
    }
    for (int32_t o = 0; o < A; ++o) {
      double acc = (double)b3[o];
      for (int32_t k = 0; k < h2; ++k) acc += bf16_to_f64(W3[(size_t)o * h2 + k]) * a2[k];
      q[(size_t)i * A + o] = acc;
    }
  }
  free(x0); free(a1); free(a2);
}

void orc_vem(const orc_env *e, const double *q, int32_t n_actions, const float *eps,
             int32_t *actions, uint8_t *explore) {
  for (int32_t i = 0; i < e->cfg.n_envs; ++i) {
    const double *qi = q + (size_t)i * n_actions;
    int32_t g = 0;
    for (int32_t a = 1; a < n_actions; ++a)
      if (qi[a] > qi[g]) g = a;
    uint32_t w[4];
    draw(e, (uint32_t)i, ORC_P_EXPLORE, 0, w);
    int32_t ex = unit24(w[0]) < eps[i];
    actions[i] = ex ? scale_u32(w[1], (uint32_t)n_actions) : g;
    if (explore) explore[i] = (uint8_t)ex;
  }
}

void orc_uniform_actions(const orc_env *e, int32_t *actions) {
  for (int32_t i = 0; i < e->cfg.n_envs; ++i) {
    uint32_t w[4];
    draw(e, (uint32_t)i, ORC_P_ACTION_UNIFORM, 0, w);
    actions[i] = scale_u32(w[0], (uint32_t)e->task.n_actions);
  }
}

void orc_vem_epsilon(int32_t n, int32_t m, double e_min, double e_max, float *eps) {
  for (int32_t i = 0; i < n; ++i) {
    if (i < n - m) {
      eps[i] = (float)e_min;
    } else {
      double frac = m > 1 ? (double)(i - (n - m)) / (double)(m - 1) : 1.0;
      eps[i] = (float)(e_min + e_max * frac);
    }
  }
}

int32_t orc_vem_or(int64_t T, int32_t or_start, int32_t or_final, int64_t decay) {
  if (decay <= 0) return or_final;
  const int64_t t = T < decay ? T : decay;
  return or_start - (int32_t)(((int64_t)(or_start - or_final) * t) / decay);
}

void orc_sincos_batch(int32_t n, const float *phi, float *s, float *c) {
  for (int32_t i = 0; i < n; ++i) orc_sincos_f32(phi[i], s + i, c + i);
}

void orc_philox_batch(int32_t n, const uint32_t *ctr, const uint32_t key[2], uint32_t *out) {
  for (int32_t i = 0; i < n; ++i) orc_philox4x32_10(ctr + 4 * (size_t)i, key, out + 4 * (size_t)i);
}
