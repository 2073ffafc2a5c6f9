// sparrow_mlp.h -- the actor's Q-network (Sec. 4.3.2 fully connected ReLU
// layers) for hidden widths whose weights do not fit in registers (512: the
// 68-512-512-7 network is 1.2 MB of bf16), in BF16 on MFMA with FP32
// accumulation, then VEM (Sec. 3.1.1). Same arithmetic as the register-
// resident actor: the observation is rounded to bf16, each layer accumulates
// in FP32, bias and ReLU follow, and hidden activations are rounded to bf16
// (RNE) before the next layer.
//
// Layout. A workgroup of eight waves takes 64 envs (four 16-env column tiles)
// per pass. The weights stream from L2 (every workgroup reads all of them
// once per pass, so a pass amortises them over 64 envs); activations stay on
// chip:
//   layer 1  wave w computes hidden tiles [w*T, w*T + T) (16 units each) for
//            all 64 envs: A = W1 fragments from global memory, B = the bf16
//            input rows in LDS; the result goes to LDS as bf16 rows [env][h].
//   layer 2  the same split over W2, reading layer 1 from LDS. Its output is
//            never stored: bias, ReLU and bf16 rounding happen in registers,
//            and the wave multiplies its own 16*T units straight into a
//            partial layer 3 (A = W3 columns of those units, B = the
//            activations as they sit in the accumulators).
//   layer 3  the eight partial [16 action][64 env] tiles meet in LDS (over
//            the space layer 1 used) and are summed in wave order.
// One v_mfma_f32_16x16x32_bf16 computes D[h][env] += W[h][k] X[env][k] over a
// 16 x 16 x 32 block; lane l holds A row l % 16 and B column l % 16, each
// with eight k values 8 (l / 16) .. + 7, and D rows 4 (l / 16) .. + 3 of
// column l % 16.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sparrow_device.h"
#include "sparrow_qnet.h"

namespace sp {

constexpr int kMWaves = 8;
constexpr int kMThreads = 64 * kMWaves;
constexpr int kMEnvTiles = 4;
constexpr int kMRows = 16 * kMEnvTiles;  // envs per pass

template <int D0P, int H>
struct MlpCfg {
  static constexpr int T = H / 16 / kMWaves;  // hidden tiles per wave
  static constexpr int K1 = D0P / 32;
  static constexpr int K2 = H / 32;
  static constexpr int XS = D0P + 8;  // LDS row stride of the input (bf16)
  static constexpr int HS = H + 8;    // LDS row stride of layer 1 (bf16)
  static_assert(T >= 2 && T % 2 == 0, "hidden width must be a multiple of 256");
  static constexpr int kXBytes = kMRows * XS * 2;
  static constexpr int kHBytes = kMRows * HS * 2;
  static constexpr int kQBytes = kMWaves * 16 * kMRows * 4;  // layer-3 partials
  static_assert(kQBytes <= kHBytes, "partials reuse the layer-1 space");
  static constexpr int kLdsBytes = kXBytes + kHBytes;
};

// Q-network + VEM over n observation rows. Outputs as k_qnet: q [n][7]
// (nullable), greedy [n] (nullable), actions [n] (nullable; eps, g, keys).
template <int D0P, int H>
__global__ void __launch_bounds__(kMThreads)
k_mlp(QParams qp, const float* __restrict__ obs, int32_t n, float* __restrict__ q,
      int32_t* __restrict__ greedy, const float* __restrict__ eps, uint32_t g, uint32_t key0,
      uint32_t key1, int32_t* __restrict__ actions) {
  using C = MlpCfg<D0P, H>;
  extern __shared__ uint32_t lds[];
  uint16_t* X = reinterpret_cast<uint16_t*>(lds);
  uint16_t* H1 = reinterpret_cast<uint16_t*>(reinterpret_cast<char*>(lds) + C::kXBytes);
  float* QP = reinterpret_cast<float*>(H1);
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int col = l & 15, kq = (l >> 4) * 8, hq = (l >> 4) * 4;
  const int h0 = w * C::T * 16;  // this wave's first hidden unit

  // padded input columns stay zero for the whole kernel
  for (int k = tid; k < C::kXBytes / 4; k += kMThreads) lds[k] = 0u;

  for (int r0 = blockIdx.x * kMRows; r0 < n; r0 += gridDim.x * kMRows) {
    __syncthreads();  // previous pass done with X and the partials
    for (int idx = tid; idx < kMRows * qp.d0; idx += kMThreads) {
      const int r = idx / qp.d0, k = idx - r * qp.d0;
      X[r * C::XS + k] = r0 + r < n ? bf16_rne(obs[(size_t)(r0 + r) * qp.d0 + k]) : 0;
    }
    __syncthreads();

    // ---- layer 1: H1[env][h] = relu(W1 x + b1) as bf16
    {
      f32x4 acc[C::T][kMEnvTiles];
#pragma unroll
      for (int t = 0; t < C::T; ++t)
#pragma unroll
        for (int e = 0; e < kMEnvTiles; ++e) acc[t][e] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < C::K1; ++ks) {
        bf16x8 a[C::T], b[kMEnvTiles];
#pragma unroll
        for (int t = 0; t < C::T; ++t)
          a[t] = *reinterpret_cast<const bf16x8*>(qp.w1 + (size_t)(h0 + t * 16 + col) * D0P +
                                                  ks * 32 + kq);
#pragma unroll
        for (int e = 0; e < kMEnvTiles; ++e)
          b[e] = *reinterpret_cast<const bf16x8*>(X + (e * 16 + col) * C::XS + ks * 32 + kq);
#pragma unroll
        for (int t = 0; t < C::T; ++t)
#pragma unroll
          for (int e = 0; e < kMEnvTiles; ++e) acc[t][e] = mfma16x16x32(a[t], b[e], acc[t][e]);
      }
#pragma unroll
      for (int t = 0; t < C::T; ++t) {
        const int hb = h0 + t * 16 + hq;
        const f32x4 bias = {qp.b1[hb], qp.b1[hb + 1], qp.b1[hb + 2], qp.b1[hb + 3]};
#pragma unroll
        for (int e = 0; e < kMEnvTiles; ++e) {
          const f32x4 v4 = acc[t][e] + bias;
          uint2 v;
          v.x = pack_relu_bf16x2(v4[0], v4[1]);
          v.y = pack_relu_bf16x2(v4[2], v4[3]);
          *reinterpret_cast<uint2*>(H1 + (e * 16 + col) * C::HS + hb) = v;
        }
      }
    }
    __syncthreads();

    // ---- layer 2 (+ this wave's share of layer 3)
    f32x4 q3[kMEnvTiles];
#pragma unroll
    for (int e = 0; e < kMEnvTiles; ++e) q3[e] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    {
      f32x4 acc[C::T][kMEnvTiles];
#pragma unroll
      for (int t = 0; t < C::T; ++t)
#pragma unroll
        for (int e = 0; e < kMEnvTiles; ++e) acc[t][e] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      // W2 fragments of the next K step are loaded while this one multiplies
      bf16x8 a_cur[C::T], a_nxt[C::T];
#pragma unroll
      for (int t = 0; t < C::T; ++t)
        a_cur[t] = *reinterpret_cast<const bf16x8*>(qp.w2 + (size_t)(h0 + t * 16 + col) * H + kq);
      for (int ks = 0; ks < C::K2; ++ks) {
        const int kn = ks + 1 < C::K2 ? ks + 1 : ks;
#pragma unroll
        for (int t = 0; t < C::T; ++t)
          a_nxt[t] = *reinterpret_cast<const bf16x8*>(qp.w2 + (size_t)(h0 + t * 16 + col) * H +
                                                      kn * 32 + kq);
        bf16x8 b[kMEnvTiles];
#pragma unroll
        for (int e = 0; e < kMEnvTiles; ++e)
          b[e] = *reinterpret_cast<const bf16x8*>(H1 + (e * 16 + col) * C::HS + ks * 32 + kq);
#pragma unroll
        for (int t = 0; t < C::T; ++t)
#pragma unroll
          for (int e = 0; e < kMEnvTiles; ++e) acc[t][e] = mfma16x16x32(a_cur[t], b[e], acc[t][e]);
#pragma unroll
        for (int t = 0; t < C::T; ++t) a_cur[t] = a_nxt[t];
      }
      // Layer 3 over this wave's units, two hidden tiles per MFMA: lane l's
      // eight k values are units hq + 0..3 of tile t and of tile t + 1 (the
      // accumulator rows it holds), so its W3 fragment takes the same units.
#pragma unroll
      for (int t = 0; t < C::T; t += 2) {
        const int ha = h0 + t * 16 + hq, hb = ha + 16;
        const f32x4 bias_a = {qp.b2[ha], qp.b2[ha + 1], qp.b2[ha + 2], qp.b2[ha + 3]};
        const f32x4 bias_b = {qp.b2[hb], qp.b2[hb + 1], qp.b2[hb + 2], qp.b2[hb + 3]};
        const uint2 wa = *reinterpret_cast<const uint2*>(qp.w3 + (size_t)col * H + ha);
        const uint2 wb = *reinterpret_cast<const uint2*>(qp.w3 + (size_t)col * H + hb);
        const uint4 w4 = {wa.x, wa.y, wb.x, wb.y};
        const bf16x8 a3 = __builtin_bit_cast(bf16x8, w4);
#pragma unroll
        for (int e = 0; e < kMEnvTiles; ++e) {
          const f32x4 va = acc[t][e] + bias_a, vb = acc[t + 1][e] + bias_b;
          const uint4 h4 = {pack_relu_bf16x2(va[0], va[1]), pack_relu_bf16x2(va[2], va[3]),
                            pack_relu_bf16x2(vb[0], vb[1]), pack_relu_bf16x2(vb[2], vb[3])};
          q3[e] = mfma16x16x32(a3, __builtin_bit_cast(bf16x8, h4), q3[e]);
        }
      }
    }
    __syncthreads();  // every wave is done reading layer 1: its space takes the partials
#pragma unroll
    for (int e = 0; e < kMEnvTiles; ++e)
#pragma unroll
      for (int i = 0; i < 4; ++i) QP[(w * 16 + hq + i) * kMRows + e * 16 + col] = q3[e][i];
    __syncthreads();
    if (tid < kMRows && r0 + tid < n) {
      const int row = r0 + tid;
      float qa[kNumActions];
      int best = 0;
#pragma unroll
      for (int a = 0; a < kNumActions; ++a) {
        float s = QP[a * kMRows + tid];
#pragma unroll
        for (int ww = 1; ww < kMWaves; ++ww) s += QP[(ww * 16 + a) * kMRows + tid];
        qa[a] = qp.b3[a] + s;
        if (a < qp.n_actions && qa[a] > qa[best]) best = a;
      }
      if (q)
        for (int a = 0; a < qp.n_actions; ++a) q[(size_t)row * qp.n_actions + a] = qa[a];
      if (greedy) greedy[row] = best;
      if (actions)
        actions[row] =
            vem_select(best, row, g, actor_eps(qp, eps, row, g), key0, key1, qp.n_actions);
    }
  }
}

}  // namespace sp
