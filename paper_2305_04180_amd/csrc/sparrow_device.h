// sparrow_device.h -- gfx950 device code of the vectorized Sparrow step.
//
// Method (arXiv 2305.04180): Sec. 3.2.2 Eq. (5)/(6) kinematics applied per
// env as in Eq. (7)/(8); Sec. 3.2 LiDAR ray casting, noise and collision on
// the occupancy grid; Sec. 3.2.4 per-episode domain randomisation; Sec. 3.2.5
// AutoReset; Sec. 4.3.1 state, actions and terminal rewards; Sec. 3.1.1 VEM.
//
// Execution model. A workgroup owns a group of envs whose bit-packed maps it
// stages into LDS. Each env is served by L consecutive lanes of one wave
// (L = 16, 32 or 64); those lanes hold the env's scalar state redundantly, so
// kinematics need no broadcast, and split the per-ray and per-cell work:
// a lane marches one ray (or several, or half the samples of one ray when
// L exceeds the ray count) and wave ballots give first hits, collision and
// the lowest accepted reset candidate.
//
// Floating point: everything that can move a grid index or a done flag is
// evaluated as separately rounded binary32 operations in a fixed order
// (built with -ffp-contract=off), so hit cells and done flags are exact.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sparrow_ring_dev.h"

namespace sp {

constexpr int kStop = 7;
constexpr int kNumActions = 7;  // the largest action set (the 7-row table)

// Philox counter word 2 ("purpose") of each random draw.
enum : uint32_t {
  kResetDR = 1, kResetStart = 2, kResetTarget = 3, kNoise = 4,
  kNoiseReset = 5, kActionUniform = 6, kExplore = 7
};

constexpr double kPiD = 3.14159265358979323846;
constexpr float kPiF = (float)kPiD;
constexpr float kTwoPiF = (float)(2.0 * kPiD);
constexpr float kTwoOverPiF = (float)(2.0 / kPiD);
constexpr float kInvPiF = (float)(1.0 / kPiD);
constexpr float kTwoM24 = 5.9604644775390625e-08f;
constexpr float kMinusTwoLn2 = (float)(-2.0 * 0.69314718055994530942);

// Target velocity of action a: (fraction of v_max, fraction of omega_max) =
// (0.02, 1) (1, 1) (1, 0.5) (1, 0) (1, -0.5) (1, -1) (0.02, -1); evaluated
// with selects so no table is read from memory inside the step.
__device__ __forceinline__ float act_v(int a) { return (a == 0 || a == 6) ? 0.02f : 1.0f; }
__device__ __forceinline__ float act_w(int a) {
  return a <= 1 ? 1.0f : a == 2 ? 0.5f : a == 3 ? 0.0f : a == 4 ? -0.5f : -1.0f;
}

// ------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11), counter (env, step, purpose, sub).
// ------------------------------------------------------------------------
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // each 64-bit product in one v_mad_u64_u32 (not a low and a high multiply)
    const uint64_t m0 = (uint64_t)0xD2511F53u * c0, m1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t lo0 = (uint32_t)m0, hi0 = (uint32_t)(m0 >> 32);
    const uint32_t lo1 = (uint32_t)m1, hi1 = (uint32_t)(m1 >> 32);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

// float -> bf16 bits, round to nearest even (v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint16_t bf16_rne(float f) {
  return __builtin_bit_cast(uint16_t, (__bf16)f);
}

__device__ __forceinline__ float unit24(uint32_t w) { return (float)(w >> 8) * kTwoM24; }
__device__ __forceinline__ int scale_u32(uint32_t w, uint32_t n) {
  return (int)__umulhi(w, n);  // floor(w * n / 2^32)
}

// ------------------------------------------------------------------------
// sincos: Cody-Waite three-part reduction by pi/2, Taylor polynomials of
// sin (to r^11) and cos (to r^10) with coefficients +-1/n!.
// ------------------------------------------------------------------------
constexpr float clear12(float f) {
  return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, f) & ~0xFFFu);
}
constexpr float kRedA = clear12((float)(kPiD / 2.0));
constexpr float kRedB = clear12((float)(kPiD / 2.0 - (double)kRedA));
constexpr float kRedC = (float)(kPiD / 2.0 - (double)kRedA - (double)kRedB);

__device__ __forceinline__ void sincos_f32(float phi, float& s_out, float& c_out) {
  const float s1 = (float)(-1.0 / 6.0), s2 = (float)(1.0 / 120.0),
              s3 = (float)(-1.0 / 5040.0), s4 = (float)(1.0 / 362880.0),
              s5 = (float)(-1.0 / 39916800.0);
  const float c1 = (float)(-1.0 / 2.0), c2 = (float)(1.0 / 24.0), c3 = (float)(-1.0 / 720.0),
              c4 = (float)(1.0 / 40320.0), c5 = (float)(-1.0 / 3628800.0);
  const float kq = __builtin_rintf(phi * kTwoOverPiF);
  const int k = (int)kq;
  float r = phi - kq * kRedA;
  r = r - kq * kRedB;
  r = r - kq * kRedC;
  const float r2 = r * r;
  float ps = s5;
  ps = ps * r2 + s4;
  ps = ps * r2 + s3;
  ps = ps * r2 + s2;
  ps = ps * r2 + s1;
  const float s = r + (r * r2) * ps;
  float pc = c5;
  pc = pc * r2 + c4;
  pc = pc * r2 + c3;
  pc = pc * r2 + c2;
  pc = pc * r2 + c1;
  const float c = 1.0f + r2 * pc;
  const int quad = k & 3;
  s_out = quad == 0 ? s : quad == 1 ? c : quad == 2 ? -s : -c;
  c_out = quad == 0 ? c : quad == 1 ? -s : quad == 2 ? -c : s;
}

// ------------------------------------------------------------------------
// Kernel parameters (passed by value).
// ------------------------------------------------------------------------
struct State {  // structure of arrays, [N] each
  float *x, *y, *phi, *vl, *va, *tx, *ty, *dprev, *dt, *K, *mu, *vmax, *sigma;
  int32_t* t;
  uint32_t* ctl;  // delay | q0 << 8 | q1 << 16
};

struct MapMeta {  // packed map m: words [off, off + 1 + (H + 2) * wpr), 16-byte padded
  uint32_t off;
  int32_t W, H, wpr;
};

struct Params {
  State s;
  const uint32_t* words;    // all packed maps
  const MapMeta* meta;      // [n_maps]
  const float* inv_dn;      // [n_maps]
  const int32_t* env_map;   // [N]
  const float2* rays;       // [n_rays] (cos, sin) of each ray's offset angle
  const int4* slots;        // [n_groups][epw]: {env (-1: empty), map, LDS word offset, words}
  int32_t n_groups, epw;
  int32_t n_envs, n_rays, obs_dim, M, t_max, delay_lo, delay_hi;
  int32_t k_free;           // samples with t_k (1 + 1e-6) + 1e-3 <= robot radius
  // task (Sec. 4.3.1): actions 7 (the table) or 5 (its rows 0, 1, 3, 5, 6);
  // reward 0 progress, 1 Eq. (11); state 0 target distance/bearing, 1
  // relative pose
  int32_t n_actions, reward_mode, state_mode;
  float r_arrive, r_collide;  // terminal rewards
  float inv_D;              // 1 / planning distance
  float near_r;             // robot radius + the r_d margin
  float w_d1, w_d2, w_v, w_a, w_d;  // Eq. (11) weights
  int32_t win_rows;         // rows staged on each side of the robot's row (windowed step)
  // k_rollout: set words before and after the group's maps in LDS (0: no
  // padding, the march clamps), and the words of the maps region
  int32_t march_pad, maps_words;
  float ds, range, inv_R, robot_r, arrive_r, omega_max;
  float dt_lo, dt_span, K_lo, K_span, mu_lo, mu_span, vmax_lo, vmax_span, sigma_lo,
      sigma_span;
  uint32_t key0, key1;
  uint32_t g;               // global step of this launch (rollout: of its first step)
  int32_t K_steps;          // rollout length
  // step / reset I/O
  const int32_t* actions;   // [N]
  float* obs;               // [N][obs_dim]
  float* cur_obs;           // library copy of the latest observation
  float* reward;
  uint8_t* done;
  uint8_t* flags;
  float* final_obs;
  int16_t* hit_k;           // [N][n_rays]
  int32_t* err;             // sticky error word
  // rollout I/O ([K][N])
  int32_t* r_actions;
  float* r_reward;
  uint8_t* r_done;
  // rollout trace (nullable): observation [K][N][obs_dim] and hit indices
  // [K][N][n_rays] of steps 0 .. K - 2 (the last step's are obs and hit_k)
  float* t_obs;
  int16_t* t_hits;
  // actor
  const float* eps;         // [N]
  // collecting rollout: the experience buffer and the slot of its next add
  RingDev ring;
  int32_t ring_head;
  int32_t ring_terminal;    // s' of a done transition: 1 terminal, 0 post-reset observation
};

// The task seen by a kernel instantiation: TK = false is the default task
// (7 actions, progress reward with -10 / +10, target state) fixed at compile
// time, so its kernels carry none of the other tasks' code; TK = true reads
// the task from the parameters.
template <bool TK>
struct TaskOf {
  static __device__ __forceinline__ int n_actions(const Params& p) {
    return TK ? p.n_actions : kNumActions;
  }
  static __device__ __forceinline__ int reward(const Params& p) { return TK ? p.reward_mode : 0; }
  static __device__ __forceinline__ int state(const Params& p) { return TK ? p.state_mode : 0; }
  static __device__ __forceinline__ float arrive(const Params& p) { return TK ? p.r_arrive : 10.0f; }
  static __device__ __forceinline__ float collide(const Params& p) {
    return TK ? p.r_collide : -10.0f;
  }
};

// Destination of one observation in the experience buffer (both NULL: none).
struct RingRow {
  uint8_t* r;   // [n_rays] range levels
  uint16_t* c;  // [4] binary16 scalars
};

__device__ __forceinline__ RingRow ring_row(uint8_t* r, uint16_t* c, int nr, int32_t slot) {
  return RingRow{r + (size_t)slot * nr, c + (size_t)slot * kRingScalars};
}

// ------------------------------------------------------------------------
// Per-env register state (every lane of the env holds a copy).
// ------------------------------------------------------------------------
struct Env {
  float x, y, phi, vl, va, tx, ty, dprev, dt, K, mu, vmax, sigma;
  int32_t t, delay, q0, q1;
  float sphi, cphi;  // sincos_f32(phi), kept current with phi
};

__device__ __forceinline__ Env load_env(const State& s, int i) {
  Env e;
  e.x = s.x[i]; e.y = s.y[i]; e.phi = s.phi[i]; e.vl = s.vl[i]; e.va = s.va[i];
  e.tx = s.tx[i]; e.ty = s.ty[i]; e.dprev = s.dprev[i]; e.dt = s.dt[i]; e.K = s.K[i];
  e.mu = s.mu[i]; e.vmax = s.vmax[i]; e.sigma = s.sigma[i]; e.t = s.t[i];
  const uint32_t c = s.ctl[i];
  e.delay = (int)(c & 0xFFu); e.q0 = (int)((c >> 8) & 0xFFu); e.q1 = (int)((c >> 16) & 0xFFu);
  sincos_f32(e.phi, e.sphi, e.cphi);
  return e;
}

__device__ __forceinline__ void store_env(const State& s, int i, const Env& e) {
  s.x[i] = e.x; s.y[i] = e.y; s.phi[i] = e.phi; s.vl[i] = e.vl; s.va[i] = e.va;
  s.tx[i] = e.tx; s.ty[i] = e.ty; s.dprev[i] = e.dprev; s.dt[i] = e.dt; s.K[i] = e.K;
  s.mu[i] = e.mu; s.vmax[i] = e.vmax; s.sigma[i] = e.sigma; s.t[i] = e.t;
  s.ctl[i] = (uint32_t)e.delay | ((uint32_t)e.q0 << 8) | ((uint32_t)e.q1 << 16);
}

// ------------------------------------------------------------------------
// Lane geometry of one env inside a wave.
// ------------------------------------------------------------------------
template <int L>
struct Lanes {
  int q;          // lane index within the env, [0, L)
  int seg;        // first wave lane of the env
  uint64_t mask;  // the env's lanes in a wave ballot
  __device__ __forceinline__ explicit Lanes(int tid) {
    q = tid & (L - 1);
    seg = (tid & 63) & ~(L - 1);
    if constexpr (L == 64) mask = ~0ull;
    else mask = ((1ull << L) - 1ull) << seg;
  }
  __device__ __forceinline__ uint64_t ballot(bool p) const {
    return (uint64_t)__ballot(p) & mask;
  }
};

// v_cvt_flr_i32_f32: floor and convert in one instruction (equal to
// (int)floorf(x) for |x| < 2^31; saturates beyond, and NaN gives 0).
__device__ __forceinline__ int cvt_flr(float x) {
  int r;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}
__device__ __forceinline__ int med3i(int x, int lo, int hi) {
  int r;
  asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "v"(hi));
  return r;
}

// A map slot. Row y (y = -1..H) is n = ceil((W + 2) / 32) words; cell
// x >= 0 is bit x & 31 of word x >> 5 of its row, and columns -1 and -2 are
// bits 31 and 30 of the previous row's last word (columns >= W, so set), with
// one set word in front of row -1. Every bit outside [0, W) x [0, H) is set,
// so a coordinate clamped to [-1, W] x [-1, H] reads as occupied: outside the
// map counts as an obstacle. w1 points at word 0 of row 0; the word of (x, y)
// is w1[y * n + (x >> 5)] with an arithmetic shift, its bit x & 31.
// A slot holds the whole map, or a window of rows y_lo..y_hi together with
// the word in front of row y_lo (the last word of row y_lo - 1, or the set
// word): [wlo, whi] = [y_lo n - 1, (y_hi + 1) n - 1] are the word indices
// it holds, relative to w1.
struct Slot {
  const uint32_t* w1;
  int32_t W, H, wpr;
  int32_t wlo, whi;
  // The march's address: no per-axis clamp, only the word index clamped to
  // the slot's words. Exact for a ray that starts inside the map:
  // consecutive samples move at most ds |u| <= 1 (+ rounding, < 2 cells) per
  // axis, so the first sample outside [0, W) x [0, H) lies within two cells
  // of the map and its word and bit are set ones (rows -1 and H; the two
  // padding columns, which are also columns -1 and -2 of the next row; the
  // set word or the clamp for row -2 and row H + 1). A window covers every
  // row within the range of the robot, so no sample up to the first hit
  // leaves it. Later samples of the same block may read any word of the
  // slot; they are past the first hit and never count.
  __device__ __forceinline__ const uint32_t* word_of_march(int ix, int iy, int& bit) const {
    bit = ix;  // the bit-field extract uses its low five bits
    int w = __mul24(iy, wpr) + (ix >> 5);
    w = med3i(w, wlo, whi);
    asm("" : "+v"(w));
    return w1 + w;
  }
  // The march's address with no clamp at all, for a whole-map slot staged
  // between set words (see k_rollout's LDS layout): every map of the env has
  // the same row length n, the slots sit back to back with their set
  // alignment words, and at least march_pad set words lie before the first
  // and after the last. Then rows -2 and H + 1 of a slot (and the word before
  // row -2) read as set, so the first sample outside the map (within two
  // cells of the last one inside) still reads its correct, set bit; later
  // samples of the block, at most P U + 1 cells further, stay within the
  // padding and never count.
  __device__ __forceinline__ const uint32_t* word_of_free(int ix, int iy, int& bit) const {
    bit = ix;
    int w = __mul24(iy, wpr) + (ix >> 5);
    asm("" : "+v"(w));
    return w1 + w;
  }
  __device__ __forceinline__ const uint32_t* word_of(int ix, int iy, int& bit) const {
    ix = med3i(ix, -1, W);
    iy = med3i(iy, -1, H);
    bit = ix;  // the bit-field extract uses its low five bits
    int w = __mul24(iy, wpr) + (ix >> 5);
    asm("" : "+v"(w));  // keep the word index whole: one shift-add forms the address
    return w1 + w;
  }
  __device__ __forceinline__ bool occ(int ix, int iy) const {
    int bit;
    const uint32_t word = *word_of(ix, iy, bit);
    return __builtin_amdgcn_ubfe(word, (uint32_t)bit, 1u) != 0u;
  }
};

// Same test with the cells spread over the env's L lanes.
template <int L>
__device__ __forceinline__ bool collides_env(const Lanes<L>& ln, const Slot& m, float px,
                                             float py, float r) {
  const float r2 = r * r;
  const int i0 = (int)ceilf(px - r) - 1, i1 = (int)floorf(px + r);
  const int j0 = (int)ceilf(py - r) - 1, j1 = (int)floorf(py + r);
  const int nx = i1 - i0 + 1, ny = j1 - j0 + 1, nc = nx * ny;
  auto test = [&](int i, int j) {
    if (!m.occ(i, j)) return false;
    const float fi = (float)i, fj = (float)j;
    const float dx = fmaxf(fmaxf(fi - px, 0.0f), px - (fi + 1.0f));
    const float dy = fmaxf(fmaxf(fj - py, 0.0f), py - (fj + 1.0f));
    const float d2 = dx * dx + dy * dy;
    return d2 <= r2;
  };
  bool hit = false;
  if (L == 64 && nx <= 8 && ny <= 8) {
    // one cell per lane: lane q takes column q & 7, row q >> 3 of the box
    const int cx = ln.q & 7, cy = ln.q >> 3;
    if (cx < nx && cy < ny) hit = test(i0 + cx, j0 + cy);
  } else {
    for (int c = ln.q; c < nc; c += L) hit |= test(i0 + c % nx, j0 + c / nx);
  }
  return ln.ballot(hit) != 0ull;
}

// Samples per lane per march iteration (independent LDS reads): 10 by
// default; the plain step also has a 16-sample instantiation for long ranges
// (the host picks the one that wastes fewer samples past the range).
constexpr int kUnroll = 10;
constexpr int kUnrollLong = 16;

// Sample addresses: per-axis clamp (any start), the word index clamped to
// the slot (a start inside the map), or no clamp (a start inside the map, in
// a padded whole-map layout).
enum : int { kAddrAxis = 0, kAddrWord = 1, kAddrFree = 2 };

// U samples k0 + u * stride of one ray: all addresses first, then all
// LDS reads, then the tests, so the reads are in flight together. Sample
// distances are t_k = (float)k * ds; with ds == 1 that is (float)k, exact
// for k < 2^24. Returns the smallest hitting k of the block, or k0 + U * stride (one past the
// block) when none hits; hits past M are the caller's to discard. ADDR is
// one of the address modes above.
template <bool UNIT, int ADDR, int U>
__device__ __forceinline__ int sample_block(const Slot& m, float x, float y, float ux, float uy,
                                            float ds, int k0, int stride) {
  static_assert(U <= 31, "hit bits of one block and the sentinel fit a word");
  const uint32_t* adr[U];
  int bit[U];
  const float tk0 = (float)k0, fst = (float)stride;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    // unit step: t_k = (float)k formed as stride * u + k0 in one fused
    // multiply-add, exact for the small integers involved
    const float tk = UNIT ? (u == 0 ? tk0 : __builtin_fmaf(fst, (float)u, tk0))
                          : (float)(k0 + u * stride) * ds;
    const float px = x + tk * ux;
    const float py = y + tk * uy;
    adr[u] = ADDR == kAddrAxis   ? m.word_of(cvt_flr(px), cvt_flr(py), bit[u])
             : ADDR == kAddrWord ? m.word_of_march(cvt_flr(px), cvt_flr(py), bit[u])
                                 : m.word_of_free(cvt_flr(px), cvt_flr(py), bit[u]);
  }
  uint32_t wv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) wv[u] = *adr[u];
  // hit bit u of the block: one shift-or per sample on the extracted bit
  uint32_t hits = 1u << U;  // sentinel: no hit -> one past the block
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint32_t b = __builtin_amdgcn_ubfe(wv[u], (uint32_t)bit[u], 1u);
    asm("v_lshl_or_b32 %0, %1, %2, %0" : "+v"(hits) : "v"(b), "I"(u));
  }
  return k0 + (int)__builtin_ctz(hits) * stride;
}

// First hit of one ray marched by one lane, from sample k_start (earlier
// samples are known to be free). Returns -1 when no sample up to M hits.
template <bool UNIT, int ADDR, int U>
__device__ __forceinline__ int march_lane(const Slot& m, float x, float y, float ux, float uy,
                                          float ds, int M, int k_start) {
  int k0 = k_start;
  for (;; k0 += U) {
    const int kh = sample_block<UNIT, ADDR, U>(m, x, y, ux, uy, ds, k0, 1);
    if (kh < k0 + U) return kh <= M ? kh : -1;
    if (k0 + U > M) return -1;
  }
}

// P lanes per ray (P = L / Lr, a power of two): in iteration `it` lane
// `phase` tests samples it*P*U + u*P + phase; the lanes of the ray then take
// the minimum, so the ray stops at the first iteration with any hit.
template <bool UNIT, int ADDR, int U>
__device__ __forceinline__ int march_split(const Slot& m, float x, float y, float ux, float uy,
                                           float ds, int M, int P, int phase, int Lr, int L,
                                           int k_start) {
  const int span = P * U;
  for (int kb = k_start;; kb += span) {
    // a lane with no hit reports kb + phase + span: past the block either way
    int kl = sample_block<UNIT, ADDR, U>(m, x, y, ux, uy, ds, kb + phase, P);
    if (L == 64 && Lr == 32) {
      // partner lane is lane ^ 32: v_permlane32_swap leaves {own, partner}
      // in the two results of every lane, with no LDS round trip
      const auto sw = __builtin_amdgcn_permlane32_swap((uint32_t)kl, (uint32_t)kl, false, false);
      kl = min((int)sw[0], (int)sw[1]);
    } else {
      for (int s = Lr; s < L; s <<= 1) kl = min(kl, __shfl_xor(kl, s));
    }
    if (kl < kb + span) return kl <= M ? kl : -1;
    if (kb + span > M) return -1;
  }
}

// ------------------------------------------------------------------------
// The lane's ray offset directions (cos, sin), loaded once per kernel.
// ------------------------------------------------------------------------
// At most 128 rays: a lane of an env on L lanes marches up to 128 / L rays.
template <int L>
struct RayDirs {
  static constexpr int kMaxRPL = 128 / L;
  float c[kMaxRPL], s[kMaxRPL];
};

template <int L>
__device__ __forceinline__ RayDirs<L> load_rays(const float2* rays, int nr, int q) {
  constexpr int kMaxRPL = RayDirs<L>::kMaxRPL;
  int R2 = 1;
  while (R2 < nr) R2 <<= 1;
  const int Lr = L >= R2 ? R2 : L;
  const int RPL = L >= R2 ? 1 : R2 / L;
  RayDirs<L> d;
#pragma unroll
  for (int rr = 0; rr < kMaxRPL; ++rr) {
    const int j = q % Lr + rr * Lr;
    float2 v = make_float2(0.0f, 0.0f);
    if (rr < RPL && j < nr) v = rays[j];
    d.c[rr] = v.x;
    d.s[rr] = v.y;
  }
  return d;
}

// ------------------------------------------------------------------------
// Observation of one env: rays (march + noise), velocities, target.
// ------------------------------------------------------------------------
// PADDED: the slot is a whole map in the padded layout (k_rollout); its
// start-inside march takes the unclamped address when p.march_pad > 0 and the
// per-axis clamp otherwise. Else (windowed slots) it takes the word clamp.
template <int L, bool TK = false, int U = kUnroll, bool PADDED = false>
__device__ __forceinline__ void observe(const Params& p, const Lanes<L>& ln, const RayDirs<L>& rd, const Slot& m,
                        Env& e, int i, uint32_t g, uint32_t purpose, float inv_dn,
                        float* dst, float* dst2, int16_t* hk, uint16_t* dst_bf16,
                        bool disk_free, RingRow qa = RingRow{nullptr, nullptr},
                        RingRow qb = RingRow{nullptr, nullptr}, bool dist_current = false) {
  // With the robot disk known to be collision-free, every sample closer to
  // the centre than the radius lies in a cell a collision test would have
  // flagged, so none of the first k_free samples can hit.
  const int k_start = disk_free ? p.k_free : 0;
  sincos_f32(e.phi, e.sphi, e.cphi);  // also the next step's Eq. (6) heading
  const float fx = -e.cphi, fy = -e.sphi;  // heading: direction of motion in Eq. (6)
  const int nr = p.n_rays;
  int R2 = 1;
  while (R2 < nr) R2 <<= 1;
  const int P = L >= R2 ? L / R2 : 1;   // lanes per ray
  const int Lr = L >= R2 ? R2 : L;      // rays handled side by side
  const int RPL = L >= R2 ? 1 : R2 / L; // rays per lane
  const int j0 = ln.q % Lr, phase = ln.q / Lr;
  const int cx = cvt_flr(e.x), cy = cvt_flr(e.y);
  const bool inside = cx >= 0 && cx < m.W && cy >= 0 && cy < m.H;
#pragma unroll
  for (int rr = 0; rr < RayDirs<L>::kMaxRPL; ++rr) {
    if (rr >= RPL) break;
    const int j = j0 + rr * Lr;
    const bool valid = j < nr;
    float ux = 0.0f, uy = 0.0f;
    if (valid) {
      ux = fx * rd.c[rr] - fy * rd.s[rr];
      uy = fy * rd.c[rr] + fx * rd.s[rr];
    }
    int kh = -1;
    if (valid) {
      // the unclamped march address needs a start inside the map and steps
      // of at most one cell (ds <= 1); anything else takes the clamped one
      // (the generic path gives the same t_k = (float)k * 1 when ds == 1;
      // 16-lane envs, which march several rays per lane, keep one path to
      // stay within the register budget)
      constexpr int kUnitAddr = PADDED ? kAddrFree : kAddrWord;
      if (L >= 32 && p.ds == 1.0f && inside && (!PADDED || p.march_pad > 0))
        kh = P == 1 ? march_lane<true, kUnitAddr, U>(m, e.x, e.y, ux, uy, p.ds, p.M, k_start)
                    : march_split<true, kUnitAddr, U>(m, e.x, e.y, ux, uy, p.ds, p.M, P, phase, Lr,
                                                      L, k_start);
      else
        kh = P == 1 ? march_lane<false, kAddrAxis, U>(m, e.x, e.y, ux, uy, p.ds, p.M, k_start)
                    : march_split<false, kAddrAxis, U>(m, e.x, e.y, ux, uy, p.ds, p.M, P, phase,
                                                       Lr, L, k_start);
    }
    if (valid && phase == 0) {
      const float d = kh < 0 ? p.range : (float)kh * p.ds;
      const U4 w = philox((uint32_t)i, g, purpose, (uint32_t)j, p.key0, p.key1);
      // Box-Muller with the hardware transcendentals: v_log_f32 is log2 and
      // v_cos_f32 takes revolutions, so cos(2 pi u2) needs no range reduction
      const float u1 = (float)((w.x >> 8) + 1u) * kTwoM24;
      const float u2 = (float)(w.y >> 8) * kTwoM24;
      const float rad = __builtin_amdgcn_sqrtf(kMinusTwoLn2 * __builtin_amdgcn_logf(u1));
      const float z = rad * __builtin_amdgcn_cosf(u2);
      float dn = d + e.sigma * z;
      dn = fminf(fmaxf(dn, 0.0f), p.range);
      const float o = dn * p.inv_R;
      if (dst) dst[j] = o;
      if (dst2) dst2[j] = o;
      if (dst_bf16) dst_bf16[j] = bf16_rne(o);
      if (hk) hk[j] = (int16_t)kh;
      if (qa.r) qa.r[j] = quant_u8(o);
      if (qb.r) qb.r[j] = quant_u8(o);
    }
  }
  if constexpr (PADDED) {
    if (ln.q == 0) {
      const float dx = e.tx - e.x, dy = e.ty - e.y;
      const float bx = dx * fx + dy * fy;
      const float by = dy * fx - dx * fy;
      const float bearing = atan2f(by, bx) * kInvPiF;
      float o[5];
      const int smode = TaskOf<TK>::state(p);
      if (smode == 0) {
        const float d2 = dx * dx + dy * dy;
        o[0] = e.vl / e.vmax;
        o[1] = e.va / p.omega_max;
        // dprev already holds sqrtf(d2) at this pose (same expression) after a
        // step that went on or after an AutoReset
        o[2] = (dist_current ? e.dprev : sqrtf(d2)) * inv_dn;
        o[3] = bearing;
        o[4] = 0.0f;
      } else {
        // relative pose (Sec. 4.3.1): position relative to the target over
        // the planning distance, orientation relative to the target, then the
        // velocities
        o[0] = (e.x - e.tx) * p.inv_D;
        o[1] = (e.y - e.ty) * p.inv_D;
        o[2] = bearing;
        o[3] = e.vl / e.vmax;
        o[4] = e.va / p.omega_max;
      }
      const int ns = 4 + smode;
      // the state's four leading values through one float4 store where the
      // row is 16-byte aligned, else one by one
      const float4 o4 = make_float4(o[0], o[1], o[2], o[3]);
      auto put = [&](float* row) {
        if ((reinterpret_cast<uintptr_t>(row + nr) & 15u) == 0u) {
          *reinterpret_cast<float4*>(row + nr) = o4;
        } else {
          for (int a = 0; a < 4; ++a) row[nr + a] = o[a];
        }
        if (ns == 5) row[nr + 4] = o[4];
      };
      if (dst) put(dst);
      if (dst2) put(dst2);
      if (dst_bf16) {
#pragma unroll
        for (int a = 0; a < 5; ++a) {
          if (a >= ns) break;
          dst_bf16[nr + a] = bf16_rne(o[a]);
        }
      }
      if (qa.c || qb.c) {
        // the four binary16 codes as one 8-byte store (rows are 8-byte aligned)
        const uint2 h = make_uint2((uint32_t)f16_bits(o[0]) | ((uint32_t)f16_bits(o[1]) << 16),
                                   (uint32_t)f16_bits(o[2]) | ((uint32_t)f16_bits(o[3]) << 16));
        if (qa.c) *reinterpret_cast<uint2*>(qa.c) = h;
        if (qb.c) *reinterpret_cast<uint2*>(qb.c) = h;
      }
    }
  } else {
    // the plain step: every lane computes the state values (the same issue
    // cost as one lane) and lane a < ns writes value a, one store
    // instruction per row
    const float dx = e.tx - e.x, dy = e.ty - e.y;
    const float bx = dx * fx + dy * fy;
    const float by = dy * fx - dx * fy;
    const float bearing = atan2f(by, bx) * kInvPiF;
    float o[5];
    const int smode = TaskOf<TK>::state(p);
    if (smode == 0) {
      const float d2 = dx * dx + dy * dy;
      o[0] = e.vl / e.vmax;
      o[1] = e.va / p.omega_max;
      o[2] = (dist_current ? e.dprev : sqrtf(d2)) * inv_dn;
      o[3] = bearing;
      o[4] = 0.0f;
    } else {
      o[0] = (e.x - e.tx) * p.inv_D;
      o[1] = (e.y - e.ty) * p.inv_D;
      o[2] = bearing;
      o[3] = e.vl / e.vmax;
      o[4] = e.va / p.omega_max;
    }
    const int ns = 4 + smode;
    const int a = ln.q;
    const float mine = a == 0 ? o[0] : a == 1 ? o[1] : a == 2 ? o[2] : a == 3 ? o[3] : o[4];
    if (a < ns) {
      if (dst) dst[nr + a] = mine;
      if (dst2) dst2[nr + a] = mine;
      if (dst_bf16) dst_bf16[nr + a] = bf16_rne(mine);
    }
    if (a == 0 && (qa.c || qb.c)) {
      const uint2 h = make_uint2((uint32_t)f16_bits(o[0]) | ((uint32_t)f16_bits(o[1]) << 16),
                                 (uint32_t)f16_bits(o[2]) | ((uint32_t)f16_bits(o[3]) << 16));
      if (qa.c) *reinterpret_cast<uint2*>(qa.c) = h;
      if (qb.c) *reinterpret_cast<uint2*>(qb.c) = h;
    }
  }
}

// ------------------------------------------------------------------------
// AutoReset of one env (Sec. 3.2.5) with per-episode randomisation (Sec.
// 3.2.4): physics draws, then start and target as the first collision-free
// candidate cell centre in counter order. The env's lanes draw the Philox
// words side by side: one stream gives the two physics draws (lanes 0 and 1)
// and start candidates 0 .. L - 3 (lane 2 + n), the next streams L
// candidates each (lane n - base); the candidates are then tested one after
// the other in counter order (most are accepted within a few), each by the
// env's L lanes splitting the disk's cells as in the per-step collision
// test. Returns false when no candidate was accepted.
// ------------------------------------------------------------------------
template <int L>
__device__ bool reset_env(const Params& p, const Lanes<L>& ln, const Slot& m, Env& e, int i,
                          uint32_t g) {
  const int q = ln.q;
  U4 cw = philox((uint32_t)i, g, q < 2 ? kResetDR : kResetStart, (uint32_t)(q < 2 ? q : q - 2),
                 p.key0, p.key1);
  auto from = [&](uint32_t v, int lane) { return (uint32_t)__shfl((int)v, ln.seg + lane); };
  e.dt = p.dt_lo + p.dt_span * unit24(from(cw.x, 0));
  e.K = p.K_lo + p.K_span * unit24(from(cw.y, 0));
  e.mu = p.mu_lo + p.mu_span * unit24(from(cw.z, 0));
  e.vmax = p.vmax_lo + p.vmax_span * unit24(from(cw.w, 0));
  e.sigma = p.sigma_lo + p.sigma_span * unit24(from(cw.x, 1));
  e.delay = p.delay_lo + scale_u32(from(cw.y, 1), (uint32_t)(p.delay_hi - p.delay_lo + 1));
  e.phi = unit24(from(cw.z, 1)) * kTwoPiF - kPiF;
  const uint32_t W = (uint32_t)m.W, H = (uint32_t)m.H;
  const float ra2 = p.arrive_r * p.arrive_r;
  bool ok = true;
  float pos[2][2];
#pragma unroll
  for (int which = 0; which < 2; ++which) {
    const uint32_t purpose = which == 0 ? kResetStart : kResetTarget;
    // counter of the stream's lane 0 (the start stream begins with the two
    // physics draws)
    int base = which == 0 ? -2 : 0;
    if (which == 1) cw = philox((uint32_t)i, g, purpose, (uint32_t)q, p.key0, p.key1);
    float bx = 0.0f, by = 0.0f;
    bool found = false;
    for (int n = 0; n < 16 * 64; ++n) {
      if (n - base >= L) {
        base = n;
        cw = philox((uint32_t)i, g, purpose, (uint32_t)(n + q), p.key0, p.key1);
      }
      const float px = (float)scale_u32(from(cw.x, n - base), W) + 0.5f;
      const float py = (float)scale_u32(from(cw.y, n - base), H) + 0.5f;
      if (n == 0) {
        bx = px;
        by = py;
      }
      bool acc = true;
      if (which == 1) {
        const float dx = px - pos[0][0], dy = py - pos[0][1];
        const float d2 = dx * dx + dy * dy;
        acc = d2 > ra2;
      }
      acc = acc && !collides_env<L>(ln, m, px, py, p.robot_r);
      if (acc) {
        bx = px;
        by = py;
        found = true;
        break;
      }
    }
    ok = ok && found;
    pos[which][0] = bx;
    pos[which][1] = by;
  }
  e.x = pos[0][0]; e.y = pos[0][1]; e.tx = pos[1][0]; e.ty = pos[1][1];
  e.vl = 0.0f; e.va = 0.0f; e.t = 0; e.q0 = kStop; e.q1 = kStop;
  const float dx = e.tx - e.x, dy = e.ty - e.y;
  e.dprev = sqrtf(dx * dx + dy * dy);
  return ok;
}

// ------------------------------------------------------------------------
// One step of one env (Alg. 1 step 4). Writes reward/done/flags through the
// lane with q == 0. Returns the done flag.
// ------------------------------------------------------------------------
struct StepOut {
  float reward;
  uint8_t done, flags;
};

// Control delay, command, Eq. (5) and Eq. (6): the part of the step that
// does not read the map. With five actions, action a is row a + (a >= 2) +
// (a >= 3) of the table: rows 0, 1, 3, 5, 6, the five actions of Sec. 4.3.1.
template <bool TK = false>
__device__ __forceinline__ void step_motion(const Params& p, Env& e, int a_hat) {
  const int n_actions = TaskOf<TK>::n_actions(p);
  if (a_hat < 0 || a_hat >= n_actions) a_hat = kStop;
  else if (n_actions == 5) a_hat += (a_hat >= 2 ? 1 : 0) + (a_hat >= 3 ? 1 : 0);
  int a;
  if (e.delay == 0) {
    a = a_hat;
  } else if (e.delay == 1) {
    a = e.q0;
    e.q0 = a_hat;
  } else {
    a = e.q0;
    e.q0 = e.q1;
    e.q1 = a_hat;
  }
  float cl = 0.0f, ca = 0.0f;
  if (a != kStop) {
    cl = e.mu * (act_v(a) * e.vmax);
    ca = e.mu * (act_w(a) * p.omega_max);
  }
  // Eq. (5)
  const float omk = 1.0f - e.K;
  float vl = e.K * e.vl + omk * cl;
  float va = e.K * e.va + omk * ca;
  vl = fminf(fmaxf(vl, -e.vmax), e.vmax);
  va = fminf(fmaxf(va, -p.omega_max), p.omega_max);
  // Eq. (6): new velocity, old heading (its sin/cos are current in e)
  e.x = e.x - e.dt * (vl * e.cphi);
  e.y = e.y - e.dt * (vl * e.sphi);
  float phi = e.phi + e.dt * va;
  if (phi > kPiF) phi -= kTwoPiF;
  else if (phi <= -kPiF) phi += kTwoPiF;
  e.phi = phi;
  e.vl = vl;
  e.va = va;
  e.t += 1;
}

// Whether any occupied cell square lies within distance r of (px, py): the
// decision of collides_env's per-cell test over the same box, one row of
// the box per lane. In a row the cells that pass form one run around the
// cell under px (dx grows monotonically away from it, and so does the FP32
// sum dx^2 + dy^2); the run's ends are estimated with a square root and
// settled by the exact per-cell test of their neighbours, then its bits are
// read word by word. Cells outside the map count as occupied.
template <int L>
__device__ __forceinline__ bool disk_any(const Lanes<L>& ln, const Slot& m, float px, float py,
                                         float r) {
  const float r2 = r * r;
  const int i0 = (int)ceilf(px - r) - 1, i1 = (int)floorf(px + r);
  const int j0 = (int)ceilf(py - r) - 1, j1 = (int)floorf(py + r);
  const int ic = cvt_flr(px);
  bool hit = false;
  for (int j = j0 + ln.q; j <= j1; j += L) {
    const float fj = (float)j;
    const float dy = fmaxf(fmaxf(fj - py, 0.0f), py - (fj + 1.0f));
    const float dy2 = dy * dy;
    if (!(dy2 <= r2)) continue;  // no cell of the row is close enough (or NaN)
    auto pass = [&](int i) {
      const float fi = (float)i;
      const float dx = fmaxf(fmaxf(fi - px, 0.0f), px - (fi + 1.0f));
      return dx * dx + dy2 <= r2;
    };
    const float t = sqrtf(r2 - dy2);
    int hi = min(max(cvt_flr(px + t), ic), i1);
    while (hi < i1 && pass(hi + 1)) ++hi;
    while (hi > ic && !pass(hi)) --hi;
    int lo = max(min((int)ceilf(px - t) - 1, ic), i0);
    while (lo > i0 && pass(lo - 1)) --lo;
    while (lo < ic && !pass(lo)) ++lo;
    // the cell under px always passes, so lo <= ic <= hi
    if (j < 0 || j >= m.H || lo < 0 || hi >= m.W) {
      hit = true;
      continue;
    }
    const uint32_t* row = m.w1 + j * m.wpr;
    for (int c = lo >> 5; c <= (hi >> 5); ++c) {
      uint32_t mask = ~0u;
      if (c == (lo >> 5)) mask &= ~0u << (lo & 31);
      if (c == (hi >> 5)) mask &= ~0u >> (31 - (hi & 31));
      hit = hit || (row[c] & mask) != 0u;
    }
  }
  return ln.ballot(hit) != 0ull;
}

// Eq. (11) of Sec. 4.3.1 on a step that did not end the episode, at the new
// pose: r = w_d1 r_d1 + w_d2 r_d2 + w_v r_v + w_alpha r_alpha + w_d r_d,
// r_d1 = max(1 - |x - tx| / D, 0), r_d2 = max(1 - |y - ty| / D, 0),
// r_v = [v_l > v_max / 2], r_alpha = 1 - |alpha| / pi (alpha: heading
// relative to the direction of the target), r_d = -1 when an occupied cell
// lies within the margin of the robot's edge (a disk test of radius
// robot_r + margin, touching included), else 0. (dx, dy) = target - pose.
template <int L>
__device__ __forceinline__ float eq11_reward(const Params& p, const Lanes<L>& ln, const Slot& m,
                                             const Env& e, float dx, float dy) {
  const float rd1 = fmaxf(1.0f - fabsf(dx) * p.inv_D, 0.0f);
  const float rd2 = fmaxf(1.0f - fabsf(dy) * p.inv_D, 0.0f);
  const float rv = e.vl > 0.5f * e.vmax ? 1.0f : 0.0f;
  float sn, cs;
  sincos_f32(e.phi, sn, cs);
  const float fx = -cs, fy = -sn;
  const float bx = dx * fx + dy * fy, by = dy * fx - dx * fy;
  const float ra = 1.0f - fabsf(atan2f(by, bx) * kInvPiF);
  const float rd = disk_any<L>(ln, m, e.x, e.y, p.near_r) ? -1.0f : 0.0f;
  float r = p.w_d1 * rd1;
  r = r + p.w_d2 * rd2;
  r = r + p.w_v * rv;
  r = r + p.w_a * ra;
  r = r + p.w_d * rd;
  return r;
}

// Collision, arrival, reward and truncation at the new pose (Sec. 4.3.1).
template <int L, bool TK = false>
__device__ __forceinline__ StepOut step_outcome(const Params& p, const Lanes<L>& ln,
                                                const Slot& m, Env& e) {
  const bool coll = collides_env<L>(ln, m, e.x, e.y, p.robot_r);
  const float dx = e.tx - e.x, dy = e.ty - e.y;
  const float d2 = dx * dx + dy * dy;
  const bool arrived = d2 <= p.arrive_r * p.arrive_r;
  bool term = false;
  float r;
  if (coll) {
    r = TaskOf<TK>::collide(p);
    term = true;
  } else if (arrived) {
    r = TaskOf<TK>::arrive(p);
    term = true;
  } else if (TaskOf<TK>::reward(p) == 0) {
    const float dist = sqrtf(d2);
    r = (e.dprev - dist) - 0.01f;
    e.dprev = dist;
  } else {
    r = eq11_reward<L>(p, ln, m, e, dx, dy);
    e.dprev = sqrtf(d2);
  }
  const bool trunc = !term && e.t >= p.t_max;
  StepOut o;
  o.reward = r;
  o.done = (uint8_t)(term || trunc);
  o.flags = (uint8_t)((term ? 1 : 0) | (trunc ? 2 : 0) | (coll ? 4 : 0) |
                      (arrived && !coll ? 8 : 0));
  return o;
}

template <int L, bool TK = false>
__device__ __forceinline__ StepOut step_env(const Params& p, const Lanes<L>& ln, const Slot& m,
                                            Env& e, int a_hat) {
  step_motion<TK>(p, e, a_hat);
  return step_outcome<L, TK>(p, ln, m, e);
}

// The whole packed map m in global memory as a slot (the AutoReset of the
// windowed step tests candidates anywhere on the map).
__device__ __forceinline__ Slot global_slot(const Params& p, const MapMeta& mm) {
  Slot s;
  s.w1 = p.words + mm.off + 1 + mm.wpr;
  s.W = mm.W;
  s.H = mm.H;
  s.wpr = mm.wpr;
  s.wlo = -1 - mm.wpr;
  s.whi = (mm.H + 1) * mm.wpr - 1;
  return s;
}

// Direct global-to-LDS load of 16 bytes per lane (global_load_lds_dwordx4):
// the wave's LDS destination is that of its first active lane, lane l's
// bytes land 16 l past it, so a full wave writes 1 KB in lane order.
__device__ __forceinline__ void lds_dma16(const uint4* src, uint4* dst) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
}

// Copy the rows of map mm within p.win_rows of the robot's row (clamped to
// the map's rows -1..H), with the word in front of the first, into the env's
// LDS buffer `buf`, by the env's own L lanes (one wave, so no workgroup
// barrier: the wave's LDS writes are done before its later LDS reads). The
// copy starts at the 16-byte boundary at or below that word; packed maps are
// 16-byte padded, so it never reads past the map. buf is 16-byte aligned.
template <int L>
__device__ __forceinline__ Slot stage_window(const Params& p, const Lanes<L>& ln,
                                             const MapMeta& mm, uint32_t* buf, float y) {
  const int n = mm.wpr;
  const int cy = med3i(cvt_flr(y), -1, mm.H);
  const int y_lo = max(-1, cy - p.win_rows), y_hi = min(mm.H, cy + p.win_rows);
  const uint32_t ws = mm.off + (uint32_t)((y_lo + 1) * n);  // the word in front of row y_lo
  const uint32_t we = mm.off + 1u + (uint32_t)((y_hi + 2) * n);
  const uint32_t ws4 = ws & ~3u;
  const int n4 = (int)((we - ws4 + 3u) >> 2);
  const uint4* src = reinterpret_cast<const uint4*>(p.words + ws4);
  uint4* dst = reinterpret_cast<uint4*>(buf);
  if constexpr (L == 64) {
    // the env is the whole wave: direct global-to-LDS loads of 1 KB pieces
    // (lane l's 16 bytes land at the piece's LDS base + 16 l), all in flight
    // before one wait
    for (int b = 0; b < n4; b += 64)
      if (b + ln.q < n4)
        lds_dma16(src + b + ln.q, dst + b);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the pieces are in LDS
  } else {
    // eight 16-byte loads in flight per lane before their LDS stores
    int k = ln.q;
    for (; k + 7 * L < n4; k += 8 * L) {
      uint4 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = src[k + u * L];
#pragma unroll
      for (int u = 0; u < 8; ++u) dst[k + u * L] = v[u];
    }
    for (; k + 3 * L < n4; k += 4 * L) {
      uint4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = src[k + u * L];
#pragma unroll
      for (int u = 0; u < 4; ++u) dst[k + u * L] = v[u];
    }
    for (; k < n4; k += L) dst[k] = src[k];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  Slot s;
  s.w1 = buf + (int)(ws - ws4) + 1 - y_lo * n;
  s.W = mm.W;
  s.H = mm.H;
  s.wpr = n;
  s.wlo = y_lo * n - 1;
  s.whi = (y_hi + 1) * n - 1;
  return s;
}

}  // namespace sp
