/*
 * ring_oracle.h -- plain CPU oracle of the experience buffer that the actor
 * fills and the learner samples (arXiv 2305.04180, Sec. 3.1.2: Alg. 1 step 5
 * adds the batched transitions (s, a, r, s', done) to the sharer's buffer;
 * Alg. 2 step 1 samples a mini-batch from it; Table 6 gives the buffer size
 * and the mini-batch size).
 *
 * TEST INFRASTRUCTURE ONLY, like sparrow_oracle.h: the product path never
 * includes, links or calls it.
 *
 * Reading of the storage format (the paper stores full-precision tensors;
 * the device buffer stores a compact transition):
 *   - ranges (the first n_rays observation entries, each in [0, 1]) as
 *     uint8 q = nearest integer to 255 * clamp(o, 0, 1), ties to even, with
 *     the product rounded to binary32 first; read back as the binary32
 *     quotient q / 255;
 *   - the four scalar entries (speeds, target distance, bearing) as IEEE
 *     binary16, round to nearest even; read back exactly;
 *   - the action as int8, the reward as binary32, done as one bit.
 * Slots form a ring: the i-th transition of a push goes to slot
 * (head + i) mod capacity, then head advances by n; the stored count is
 * min(total pushed, capacity). For an env that is done, s' is its final
 * (pre-reset) observation when one is supplied.
 * Sampling draws each index uniformly from the stored slots:
 * Philox4x32-10 with counter (b, draw, ORC_P_RING_SAMPLE, 0) and the ring's
 * key gives word w; the slot is floor(w * size / 2^32).
 */
#ifndef RING_ORACLE_H
#define RING_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_P_RING_SAMPLE = 8, ORC_RING_SCALARS = 4 };

typedef struct orc_ring orc_ring;

orc_ring *orc_ring_create(int64_t capacity, int32_t n_rays, uint64_t seed);
void orc_ring_destroy(orc_ring *r);
int64_t orc_ring_size(const orc_ring *r);
int64_t orc_ring_head(const orc_ring *r);
/* s, s_next, s_final: [n][n_rays + 4]; s_final may be NULL. Returns 0, or
 * -1 when n is negative or above the capacity. */
int32_t orc_ring_push(orc_ring *r, int32_t n, const float *s, const int32_t *a,
                      const float *rew, const float *s_next, const float *s_final,
                      const uint8_t *done);
/* Transitions at the given slots, read back to binary32. Any output may be
 * NULL. Returns -1 when a slot is outside [0, size). */
int32_t orc_ring_gather(const orc_ring *r, int32_t n, const int64_t *slots, float *s,
                        int32_t *a, float *rew, float *s_next, uint8_t *done);
/* B uniform draws (see above), then a gather. idx may be NULL. Returns -1
 * when the ring is empty. */
int32_t orc_ring_sample(const orc_ring *r, int32_t B, uint32_t draw, float *s, int32_t *a,
                        float *rew, float *s_next, uint8_t *done, int64_t *idx);

/* Storage conversions, exposed for the pins. */
uint16_t orc_f16_rne(float f);
float orc_f16_to_f32(uint16_t h);
uint8_t orc_quant_u8(float o);
float orc_dequant_u8(uint8_t q);

#ifdef __cplusplus
}
#endif
#endif
