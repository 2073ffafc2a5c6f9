// sparrow_qnet.h -- the actor: Q-network forward in BF16 on MFMA (FP32
// accumulation) and vectorized epsilon-greedy exploration (VEM).
//
// The Q-network is the fully connected ReLU stack of Sec. 4.3.2 mapping the
// state to one value per discrete action; the actor takes its greedy action
// and VEM (Sec. 3.1.1) replaces it by a uniform random action with the env's
// own probability eps_i (Alg. 1 steps 2-3).
//
// Layout. Eight waves serve 16 rows (envs) at a time. Each wave keeps its
// slice of the weights resident in VGPRs for the whole kernel (weight-
// stationary): layer 1 and layer 2 are split by output tiles of 16 hidden
// units. Layer 2's output never leaves the registers: after bias, ReLU and
// bf16 rounding, the rows a lane holds of its wave's tiles are exactly a B
// fragment of a K = 32 (or K = 16) block, so one MFMA against the W3 columns
// of those units (also resident) gives the wave's share of layer 3; the
// eight partial [action][env] tiles meet in LDS and are summed in wave order.
// One v_mfma_f32_16x16x32_bf16 computes D[h][env] += W[h][k] * X[env][k] over
// a 16 x 16 x 32 block: A = weight rows, B = activation rows from LDS, D rows
// = hidden units, D columns = envs. Activations live in LDS as bf16 rows
// [env][k] padded by 16 bytes against bank conflicts; between layers they are
// rounded to bf16 (RNE) after bias and ReLU.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sparrow_device.h"

namespace sp {

constexpr int kQThreads = 512;  // eight waves
constexpr int kQWaves = 8;
constexpr int kQRows = 16;      // envs per MLP pass (MFMA N)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// VEM with a shrinking exploring interval (Sec. 3.1.1): after T = n * g
// transitions (g the global step) the last m(T) envs explore, m(T) =
// or_start - floor((or_start - or_final) * min(T, decay) / decay), with
// probabilities rising linearly across them from e_min to e_min + e_max.
// on = 0: the per-env probabilities of the eps array are used instead.
struct VemSchedule {
  int32_t on, n, or_start, or_final;
  int64_t decay;
  double e_min, e_max;
};

struct QParams {
  const uint16_t* w1;  // [h1][d0p] bf16, zero-padded columns
  const uint16_t* w2;  // [h2][h1]
  const uint16_t* w3;  // [16][h2], rows >= 7 zero
  const float* b1;     // [h1]
  const float* b2;     // [h2]
  const float* b3;     // [16], entries >= 7 zero
  int32_t d0, d0p, h1, h2;
  int32_t n_actions;       // outputs in use (5 or 7; rows of w3 past them are zero)
  int32_t lds_base_words;  // first LDS word of the actor's buffers
  VemSchedule vem;
};

// Exploration probability of env i at global step g: binary64 arithmetic in
// the order written, rounded once to binary32, so every draw compares
// against the same value the definition gives.
__device__ __forceinline__ float vem_eps(const VemSchedule& v, int i, uint32_t g) {
  int32_t m = v.or_final;
  if (v.decay > 0) {
    const int64_t T = (int64_t)v.n * (int64_t)g;
    const int64_t t = T < v.decay ? T : v.decay;
    m = v.or_start - (int32_t)(((int64_t)(v.or_start - v.or_final) * t) / v.decay);
  }
  if (i < v.n - m) return (float)v.e_min;
  const double frac = m > 1 ? (double)(i - (v.n - m)) / (double)(m - 1) : 1.0;
  return (float)(v.e_min + v.e_max * frac);
}

__device__ __forceinline__ float actor_eps(const QParams& q, const float* eps, int i, uint32_t g) {
  return q.vem.on ? vem_eps(q.vem, i, g) : eps[i];
}

// LDS: region A holds the bf16 input rows, region B the first hidden layer,
// region C the eight waves' partial layer-3 sums, FP32 [env][wave][action]
// with kQPartStride floats per env (4 more than 8 x 8, so the 16 env rows of
// one wave's 16-byte writes fall on distinct banks).
constexpr int kQPartStride = 8 * kQWaves + 4;
__host__ __device__ inline int qnet_stride0(const QParams& q) { return q.d0p + 8; }
__host__ __device__ inline int qnet_stride1(const QParams& q) { return q.h1 + 8; }
__host__ __device__ inline int qnet_region_a_bytes(const QParams& q) {
  return (kQRows * qnet_stride0(q) * 2 + 15) & ~15;
}
__host__ __device__ inline int qnet_region_b_bytes(const QParams& q) {
  return (kQRows * qnet_stride1(q) * 2 + 15) & ~15;
}
__host__ __device__ inline int qnet_region_c_bytes(const QParams&) {
  return kQRows * kQPartStride * 4;
}
__host__ __device__ inline size_t qnet_lds_bytes(const QParams& q) {
  return (size_t)qnet_region_a_bytes(q) + (size_t)qnet_region_b_bytes(q) +
         (size_t)qnet_region_c_bytes(q);
}

__device__ __forceinline__ uint16_t* qnet_region_a(const QParams& q, uint32_t* lds) {
  return reinterpret_cast<uint16_t*>(lds + q.lds_base_words);
}
__device__ __forceinline__ uint16_t* qnet_region_b(const QParams& q, uint32_t* lds) {
  return reinterpret_cast<uint16_t*>(reinterpret_cast<char*>(lds + q.lds_base_words) +
                                     qnet_region_a_bytes(q));
}
__device__ __forceinline__ float* qnet_region_c(const QParams& q, uint32_t* lds) {
  return reinterpret_cast<float*>(reinterpret_cast<char*>(lds + q.lds_base_words) +
                                  qnet_region_a_bytes(q) + qnet_region_b_bytes(q));
}
__device__ __forceinline__ uint16_t* qnet_input_row(const QParams& q, uint32_t* lds, int row) {
  return qnet_region_a(q, lds) + row * qnet_stride0(q);
}

// Weights resident in the VGPRs of one wave. D0P, H1, H2 fixed at compile time.
template <int D0P, int H1, int H2>
struct QNetCfg {
  static constexpr bool kOn = true;
  static constexpr int T1 = H1 / 16 / kQWaves;  // output tiles of layer 1 per wave
  static constexpr int K1 = D0P / 32;
  static constexpr int T2 = H2 / 16 / kQWaves;
  static constexpr int K2 = H1 / 32;
  // layer 3 over the wave's own units: pairs of tiles through K = 32 MFMAs,
  // or one tile through a K = 16 MFMA
  static constexpr int kW3Frags = T2 >= 2 ? T2 / 2 : 1;
  static constexpr bool kW3Half = T2 == 1;
  static_assert(T1 >= 1 && T2 >= 1, "hidden sizes must be multiples of 128");
  static_assert(T2 == 1 || T2 % 2 == 0, "layer-2 tiles per wave: 1 or even");
  static_assert(H1 % (16 * kQWaves) == 0 && H2 % (16 * kQWaves) == 0, "unsupported sizes");

  struct Weights {
    bf16x8 a1[T1][K1];
    bf16x8 a2[T2][K2];
    f32x4 bias1[T1];
    f32x4 bias2[T2];

    __device__ __forceinline__ void load(const QParams& q, int tid) {
      const int w = tid >> 6, l = tid & 63;
      const int r = l & 15, kq = (l >> 4) * 8;
#pragma unroll
      for (int t = 0; t < T1; ++t) {
        const int h = (w * T1 + t) * 16 + r;
#pragma unroll
        for (int ks = 0; ks < K1; ++ks)
          a1[t][ks] = *reinterpret_cast<const bf16x8*>(q.w1 + (size_t)h * D0P + ks * 32 + kq);
        const int hb = (w * T1 + t) * 16 + (l >> 4) * 4;
        bias1[t] = f32x4{q.b1[hb], q.b1[hb + 1], q.b1[hb + 2], q.b1[hb + 3]};
      }
#pragma unroll
      for (int t = 0; t < T2; ++t) {
        const int h = (w * T2 + t) * 16 + r;
#pragma unroll
        for (int ks = 0; ks < K2; ++ks)
          a2[t][ks] = *reinterpret_cast<const bf16x8*>(q.w2 + (size_t)h * H1 + ks * 32 + kq);
        const int hb = (w * T2 + t) * 16 + (l >> 4) * 4;
        bias2[t] = f32x4{q.b2[hb], q.b2[hb + 1], q.b2[hb + 2], q.b2[hb + 3]};
      }
    }
  };
};

struct NoQ {
  static constexpr bool kOn = false;
  static constexpr int kW3Frags = 1;
  static constexpr bool kW3Half = false;
  struct Weights {
    __device__ __forceinline__ void load(const QParams&, int) {}
  };
};

__device__ __forceinline__ f32x4 mfma16x16x32(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// ReLU, then two values to packed bf16 with round to nearest even
__device__ __forceinline__ uint32_t pack_relu_bf16x2(float lo, float hi) {
  const bf16x2 v = {(__bf16)fmaxf(lo, 0.0f), (__bf16)fmaxf(hi, 0.0f)};
  return __builtin_bit_cast(uint32_t, v);
}

// One dense layer for this wave's output tiles: out[env][h] = relu(W x + b).
template <int T, int KS, int AHEAD>
__device__ __forceinline__ void qnet_layer(const bf16x8 (&a)[T][KS], const f32x4 (&bias)[T],
                                           const uint16_t* in, int in_stride, uint16_t* out,
                                           int out_stride, int tile0, int l) {
  const int env = l & 15, kq = (l >> 4) * 8, hq = (l >> 4) * 4;
  f32x4 acc[T];
#pragma unroll
  for (int t = 0; t < T; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  // B fragments run up to AHEAD K steps ahead of the MFMAs that use them,
  // so the LDS reads overlap the multiplies (K outer, tiles inner); AHEAD = 1
  // reads each fragment in its own step
  constexpr int kAhead = KS < AHEAD ? KS : AHEAD;
  bf16x8 b[kAhead];
  if (kAhead > 1)
#pragma unroll
    for (int ks = 0; ks < kAhead; ++ks)
      b[ks] = *reinterpret_cast<const bf16x8*>(in + env * in_stride + ks * 32 + kq);
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const bf16x8 cur = kAhead == 1 ? *reinterpret_cast<const bf16x8*>(in + env * in_stride + ks * 32 + kq)
                                   : b[ks % kAhead];
    if (kAhead > 1 && ks + kAhead < KS)
      b[ks % kAhead] = *reinterpret_cast<const bf16x8*>(in + env * in_stride + (ks + kAhead) * 32 + kq);
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] = mfma16x16x32(a[t][ks], cur, acc[t]);
  }
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const f32x4 v4 = acc[t] + bias[t];
    uint2 v;
    v.x = pack_relu_bf16x2(v4[0], v4[1]);
    v.y = pack_relu_bf16x2(v4[2], v4[3]);
    *reinterpret_cast<uint2*>(out + env * out_stride + (tile0 + t) * 16 + hq) = v;
  }
}

typedef short bf16x4s __attribute__((ext_vector_type(4)));

// Accumulate this wave's output tiles of one dense layer (no bias, no store).
template <int T, int KS, int AHEAD>
__device__ __forceinline__ void qnet_accum(const bf16x8 (&a)[T][KS], const uint16_t* in,
                                           int in_stride, int l, f32x4 (&acc)[T]) {
  const int env = l & 15, kq = (l >> 4) * 8;
#pragma unroll
  for (int t = 0; t < T; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  constexpr int kAhead = KS < AHEAD ? KS : AHEAD;
  bf16x8 b[kAhead];
  if (kAhead > 1)
#pragma unroll
    for (int ks = 0; ks < kAhead; ++ks)
      b[ks] = *reinterpret_cast<const bf16x8*>(in + env * in_stride + ks * 32 + kq);
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const bf16x8 cur = kAhead == 1 ? *reinterpret_cast<const bf16x8*>(in + env * in_stride + ks * 32 + kq)
                                   : b[ks % kAhead];
    if (kAhead > 1 && ks + kAhead < KS)
      b[ks % kAhead] = *reinterpret_cast<const bf16x8*>(in + env * in_stride + (ks + kAhead) * 32 + kq);
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] = mfma16x16x32(a[t][ks], cur, acc[t]);
  }
}

// W3 columns of this wave's layer-2 units, in the order the lane holds the
// activations: for a pair of tiles (t, t + 1), units hq..hq + 3 of tile t
// then of tile t + 1 (a K = 32 A fragment); for a single tile its units
// hq..hq + 3 (K = 16). Row = action l % 16 (rows past the actions are zero).
// Loaded once per kernel: 4 (or 2) VGPRs per fragment.
template <class QC>
struct W3Frag {
  bf16x8 a[QC::kW3Frags];
  bf16x4s h;
  float b3;  // bias of action l % 8 (the action whose sum this lane forms)
};

template <class QC>
__device__ __forceinline__ void qnet_load_w3(const QParams& q, int tid, W3Frag<QC>& f) {
  if constexpr (QC::kOn) {
    const int w = tid >> 6, l = tid & 63;
    const int row = l & 15, hq = (l >> 4) * 4;
    if constexpr (QC::kW3Half) {
      const int h = w * 16 + hq;
      f.h = __builtin_bit_cast(bf16x4s, *reinterpret_cast<const uint2*>(q.w3 + (size_t)row * q.h2 + h));
    } else {
#pragma unroll
      for (int p = 0; p < QC::kW3Frags; ++p) {
        const int ha = (w * QC::T2 + 2 * p) * 16 + hq, hb = ha + 16;
        const uint2 wa = *reinterpret_cast<const uint2*>(q.w3 + (size_t)row * q.h2 + ha);
        const uint2 wb = *reinterpret_cast<const uint2*>(q.w3 + (size_t)row * q.h2 + hb);
        f.a[p] = __builtin_bit_cast(bf16x8, uint4{wa.x, wa.y, wb.x, wb.y});
      }
    }
    f.b3 = q.b3[l & 7];
  }
}

// Forward pass over the 16 input rows in LDS region A (the caller has made
// them visible with a barrier). Returns, in every lane, Q[a][col] with
// a = lane % 8 (bias included; a = 7 is a padding row of value 0 when seven
// actions are in use): col is the env column the lane's env occupies.
// Layer 3's eight wave partials are added in wave order 0..7, then the bias.
template <class QC, int AHEAD>
__device__ __forceinline__ float qnet_forward_sum(const QParams& q,
                                                  const typename QC::Weights& W,
                                                  const W3Frag<QC>& w3, uint32_t* lds, int tid,
                                                  int col) {
  float out = 0.0f;
  if constexpr (QC::kOn) {
    const int w = tid >> 6, l = tid & 63;
    uint16_t* ra = qnet_region_a(q, lds);
    uint16_t* rb = qnet_region_b(q, lds);
    float* rc = qnet_region_c(q, lds);
    qnet_layer<QC::T1, QC::K1, AHEAD>(W.a1, W.bias1, ra, qnet_stride0(q), rb, qnet_stride1(q),
                                      w * QC::T1, l);
    __syncthreads();
    f32x4 acc[QC::T2];
    qnet_accum<QC::T2, QC::K2, AHEAD>(W.a2, rb, qnet_stride1(q), l, acc);
    f32x4 q3 = {0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (QC::kW3Half) {
      const f32x4 v = acc[0] + W.bias2[0];
      const uint2 h2 = {pack_relu_bf16x2(v[0], v[1]), pack_relu_bf16x2(v[2], v[3])};
      q3 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w3.h, __builtin_bit_cast(bf16x4s, h2), q3,
                                                     0, 0, 0);
    } else {
#pragma unroll
      for (int p = 0; p < QC::kW3Frags; ++p) {
        const f32x4 va = acc[2 * p] + W.bias2[2 * p], vb = acc[2 * p + 1] + W.bias2[2 * p + 1];
        const uint4 h4 = {pack_relu_bf16x2(va[0], va[1]), pack_relu_bf16x2(va[2], va[3]),
                          pack_relu_bf16x2(vb[0], vb[1]), pack_relu_bf16x2(vb[2], vb[3])};
        q3 = mfma16x16x32(w3.a[p], __builtin_bit_cast(bf16x8, h4), q3);
      }
    }
    // lane l holds actions 4 (l / 16) .. + 3 of env column l % 16; actions
    // 8 .. 15 are zero rows, so only lanes below 32 store
    if (l < 32)
      *reinterpret_cast<f32x4*>(rc + (l & 15) * kQPartStride + w * 8 + (l >> 4) * 4) = q3;
    __syncthreads();
    const float* pc = rc + col * kQPartStride + (l & 7);
    float s = pc[0];
#pragma unroll
    for (int ww = 1; ww < kQWaves; ++ww) s += pc[ww * 8];
    out = w3.b3 + s;
  }
  return out;
}

// All Q values of env column col (bias included) from region C, summed in
// the same order as qnet_forward_sum; lowest index of the maximum over the
// first n_actions. For callers that hold one env per lane.
__device__ __forceinline__ int qnet_q_row(const QParams& q, uint32_t* lds, int col,
                                          float (&qa)[kNumActions], int n_actions) {
  const float* pc = qnet_region_c(q, lds) + col * kQPartStride;
  int best = 0;
#pragma unroll
  for (int a = 0; a < kNumActions; ++a) {
    float s = pc[a];
#pragma unroll
    for (int ww = 1; ww < kQWaves; ++ww) s += pc[ww * 8 + a];
    qa[a] = q.b3[a] + s;
    if (a < n_actions && qa[a] > qa[best]) best = a;
  }
  return best;
}

// Greedy action of the env whose lanes start at seg: the Q values sit in
// lanes seg + a (qnet_forward_sum); lowest index of the maximum.
template <int L>
__device__ __forceinline__ int qnet_greedy(float qsum, int seg, int n_actions) {
  int best = 0;
  float qb = 0.0f;
#pragma unroll
  for (int a = 0; a < kNumActions; ++a) {
    float v;
    if constexpr (L == 64) {
      v = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, qsum), a));
    } else {
      v = __shfl(qsum, seg + a);
    }
    if (a == 0) {
      qb = v;
    } else if (a < n_actions && v > qb) {
      qb = v;
      best = a;
    }
  }
  return best;
}

// VEM (Sec. 3.1.1): with probability eps the greedy action is replaced by a
// uniform random one; the draw is Philox (env, step, EXPLORE, 0). It does not
// depend on Q, so the rollout draws it ahead of the forward pass. Returns the random
// action, or -1 to keep the greedy one.
__device__ __forceinline__ int vem_draw(int env, uint32_t g, float eps, uint32_t key0,
                                        uint32_t key1, int n_actions) {
  const U4 w = philox((uint32_t)env, g, kExplore, 0u, key0, key1);
  return unit24(w.x) < eps ? scale_u32(w.y, (uint32_t)n_actions) : -1;
}

__device__ __forceinline__ int vem_select(int greedy, int env, uint32_t g, float eps,
                                          uint32_t key0, uint32_t key1, int n_actions) {
  const int d = vem_draw(env, g, eps, key0, key1, n_actions);
  return d >= 0 ? d : greedy;
}

}  // namespace sp
