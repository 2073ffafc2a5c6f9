/*
 * ring_oracle.c -- plain CPU oracle of the experience buffer (Sec. 3.1.2,
 * Alg. 1 step 5 and Alg. 2 step 1). TEST INFRASTRUCTURE ONLY.
 * The storage format and the sampling rule are stated in ring_oracle.h.
 */
#include "ring_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "sparrow_oracle.h"

struct orc_ring {
  int64_t cap, head, size;
  int32_t nr;
  uint32_t key[2];
  uint8_t *ranges_s, *ranges_sn;   /* [cap][nr] */
  uint16_t *scal_s, *scal_sn;      /* [cap][4] binary16 bits */
  int8_t *act;                     /* [cap] */
  float *rew;                      /* [cap] */
  uint8_t *done;                   /* [cap] (one flag per slot here) */
};

/* ---- conversions ------------------------------------------------------- */

/* binary32 -> binary16, round to nearest, ties to even (IEEE 754-2008). */
uint16_t orc_f16_rne(float f) {
  uint32_t x;
  memcpy(&x, &f, 4);
  const uint16_t sign = (uint16_t)((x >> 16) & 0x8000u);
  const uint32_t ax = x & 0x7fffffffu;
  if (ax > 0x7f800000u) return (uint16_t)(sign | 0x7e00u);  /* NaN stays NaN */
  /* 65520 = 65504 + half an ulp of binary16 at the top binade: from there
   * up (and infinity) the nearest value is infinity */
  if (ax >= 0x477ff000u) return (uint16_t)(sign | 0x7c00u);
  const uint32_t e = ax >> 23;
  if (e < 113) {
    /* |f| < 2^-14: a binary16 subnormal (or zero) in units of 2^-24 */
    if (e == 0) return sign; /* binary32 zero or subnormal: below 2^-126 */
    const uint32_t m = (ax & 0x7fffffu) | 0x800000u;  /* f = m * 2^(e-150) */
    const uint32_t shift = 126u - e;                   /* f / 2^-24 = m / 2^shift */
    if (shift > 24) return sign;                       /* below 2^-25: rounds to 0 */
    uint32_t q = m >> shift;
    const uint32_t rem = m & ((1u << shift) - 1u), half = 1u << (shift - 1u);
    if (rem > half || (rem == half && (q & 1u))) ++q;  /* may carry to 2^-14 */
    return (uint16_t)(sign | q);
  }
  /* normal: 10 of the 23 fraction bits survive, the low 13 round */
  uint32_t h = ((e - 112u) << 10) | ((ax & 0x7fffffu) >> 13);
  const uint32_t rem = ax & 0x1fffu;
  if (rem > 0x1000u || (rem == 0x1000u && (h & 1u))) ++h;  /* carry may bump the exponent */
  return (uint16_t)(sign | h);
}

float orc_f16_to_f32(uint16_t h) {
  const uint32_t sign = (uint32_t)(h & 0x8000u) << 16;
  const uint32_t e = (h >> 10) & 0x1fu, m = h & 0x3ffu;
  uint32_t x;
  if (e == 0) {
    const float v = (float)m * 0x1p-24f;  /* exact */
    return (h & 0x8000u) ? -v : v;
  }
  if (e == 31)
    x = sign | 0x7f800000u | (m << 13);
  else
    x = sign | ((e + 112u) << 23) | (m << 13);
  float f;
  memcpy(&f, &x, 4);
  return f;
}

uint8_t orc_quant_u8(float o) {
  const float c = fminf(fmaxf(o, 0.0f), 1.0f);
  const float p = c * 255.0f;      /* one binary32 rounding */
  return (uint8_t)rintf(p);        /* nearest, ties to even (default mode) */
}

float orc_dequant_u8(uint8_t q) { return (float)q / 255.0f; }

/* ---- the ring ---------------------------------------------------------- */

orc_ring *orc_ring_create(int64_t capacity, int32_t n_rays, uint64_t seed) {
  if (capacity <= 0 || n_rays <= 0) return NULL;
  orc_ring *r = (orc_ring *)calloc(1, sizeof(orc_ring));
  if (!r) return NULL;
  r->cap = capacity;
  r->nr = n_rays;
  r->key[0] = (uint32_t)seed;
  r->key[1] = (uint32_t)(seed >> 32);
  r->ranges_s = (uint8_t *)calloc((size_t)capacity * n_rays, 1);
  r->ranges_sn = (uint8_t *)calloc((size_t)capacity * n_rays, 1);
  r->scal_s = (uint16_t *)calloc((size_t)capacity * ORC_RING_SCALARS, 2);
  r->scal_sn = (uint16_t *)calloc((size_t)capacity * ORC_RING_SCALARS, 2);
  r->act = (int8_t *)calloc((size_t)capacity, 1);
  r->rew = (float *)calloc((size_t)capacity, 4);
  r->done = (uint8_t *)calloc((size_t)capacity, 1);
  if (!r->ranges_s || !r->ranges_sn || !r->scal_s || !r->scal_sn || !r->act || !r->rew ||
      !r->done) {
    orc_ring_destroy(r);
    return NULL;
  }
  return r;
}

void orc_ring_destroy(orc_ring *r) {
  if (!r) return;
  free(r->ranges_s);
  free(r->ranges_sn);
  free(r->scal_s);
  free(r->scal_sn);
  free(r->act);
  free(r->rew);
  free(r->done);
  free(r);
}

int64_t orc_ring_size(const orc_ring *r) { return r->size; }
int64_t orc_ring_head(const orc_ring *r) { return r->head; }

static void store_obs(const orc_ring *r, int64_t slot, const float *o, uint8_t *ranges,
                      uint16_t *scal) {
  for (int32_t j = 0; j < r->nr; ++j) ranges[slot * r->nr + j] = orc_quant_u8(o[j]);
  for (int32_t j = 0; j < ORC_RING_SCALARS; ++j)
    scal[slot * ORC_RING_SCALARS + j] = orc_f16_rne(o[r->nr + j]);
}

int32_t orc_ring_push(orc_ring *r, int32_t n, const float *s, const int32_t *a,
                      const float *rew, const float *s_next, const float *s_final,
                      const uint8_t *done) {
  if (n < 0 || n > r->cap) return -1;
  const int32_t D = r->nr + ORC_RING_SCALARS;
  for (int32_t i = 0; i < n; ++i) {
    const int64_t slot = (r->head + i) % r->cap;
    const float *sn = (done[i] && s_final) ? s_final + (size_t)i * D : s_next + (size_t)i * D;
    store_obs(r, slot, s + (size_t)i * D, r->ranges_s, r->scal_s);
    store_obs(r, slot, sn, r->ranges_sn, r->scal_sn);
    r->act[slot] = (int8_t)a[i];
    r->rew[slot] = rew[i];
    r->done[slot] = done[i] ? 1 : 0;
  }
  r->head = (r->head + n) % r->cap;
  r->size = r->size + n < r->cap ? r->size + n : r->cap;
  return 0;
}

static void load_obs(const orc_ring *r, int64_t slot, const uint8_t *ranges,
                     const uint16_t *scal, float *o) {
  for (int32_t j = 0; j < r->nr; ++j) o[j] = orc_dequant_u8(ranges[slot * r->nr + j]);
  for (int32_t j = 0; j < ORC_RING_SCALARS; ++j)
    o[r->nr + j] = orc_f16_to_f32(scal[slot * ORC_RING_SCALARS + j]);
}

int32_t orc_ring_gather(const orc_ring *r, int32_t n, const int64_t *slots, float *s,
                        int32_t *a, float *rew, float *s_next, uint8_t *done) {
  const int32_t D = r->nr + ORC_RING_SCALARS;
  for (int32_t b = 0; b < n; ++b)
    if (slots[b] < 0 || slots[b] >= r->size) return -1;
  for (int32_t b = 0; b < n; ++b) {
    const int64_t k = slots[b];
    if (s) load_obs(r, k, r->ranges_s, r->scal_s, s + (size_t)b * D);
    if (s_next) load_obs(r, k, r->ranges_sn, r->scal_sn, s_next + (size_t)b * D);
    if (a) a[b] = r->act[k];
    if (rew) rew[b] = r->rew[k];
    if (done) done[b] = r->done[k];
  }
  return 0;
}

int32_t orc_ring_sample(const orc_ring *r, int32_t B, uint32_t draw, float *s, int32_t *a,
                        float *rew, float *s_next, uint8_t *done, int64_t *idx) {
  if (r->size <= 0 || B < 0) return -1;
  int64_t *slots = (int64_t *)malloc(sizeof(int64_t) * (size_t)(B > 0 ? B : 1));
  if (!slots) return -1;
  for (int32_t b = 0; b < B; ++b) {
    const uint32_t ctr[4] = {(uint32_t)b, draw, ORC_P_RING_SAMPLE, 0u};
    uint32_t w[4];
    orc_philox4x32_10(ctr, r->key, w);
    slots[b] = (int64_t)(((uint64_t)w[0] * (uint64_t)r->size) >> 32);
    if (idx) idx[b] = slots[b];
  }
  const int32_t rc = orc_ring_gather(r, B, slots, s, a, rew, s_next, done);
  free(slots);
  return rc;
}
