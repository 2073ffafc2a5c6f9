// sparrow_learner.hip -- the learner's update (Alg. 2 step 2: a mini-batch
// sampled from the sharer's buffer trains the learner's model with DDQN;
// Table 6: gamma, learning rate, target-network period, mini-batch 256).
//
// One update on B transitions (s, a, r, s', done), all in FP32 with every sum
// in a fixed order, on the FP32 matrix cores (v_mfma_f32_16x16x4_f32), which
// keep it within FP32 rounding of binary64. A 256-row mini-batch through a
// 36-256-256-7 network is ~0.2 GFLOP per update, so the update is bound by
// launches and memory latency, not by arithmetic: it runs as three launches.
//   k_learn_fwd   per block of 16 rows and per pass -- the online network on
//                 s (activations kept for back-propagation), the online and
//                 the target network on s' -- all three layers with the
//                 block's activations in LDS: out = relu(b + W x), the last
//                 layer without relu
//   k_learn_rows  per block of 16 rows: a* = argmax Q_online(s') (lowest
//                 index on ties), y = r + gamma (1 - done) Q_target(s')[a*],
//                 delta = Q(s)[a] - y, g = dloss/dQ[a] = clip(delta, -k, k) /
//                 B, the block's Huber sum; the output error G[b][o] = [a_b ==
//                 o] g_b, da2[b][u] = [a2 > 0] g_b W3[a_b][u] and da1 = [a1 >
//                 0] (da2 W2)
//   k_learn_mm    the weight gradients gW3 = G^T a2, gW2 = da2^T a1, gW1 =
//                 da1^T s (each bias gradient the column sum of X, an extra
//                 column of ones in Y; relu'(0) = 0), each entry followed at
//                 once by its Adam step, and the mean loss; every
//                 target_every-th update the same launch writes the updated
//                 weights into the target network as well
// Weights are row-major [out][in], concatenated [W1 | W2 | W3]; biases
// [b1 | b2 | b3].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sparrow.h"
#include "sparrow_device.h"
#include "sparrow_host.h"

using namespace sp;

namespace {

constexpr int kMaxUnits = 512;

struct Dims {
  int32_t d0, h1, h2, A;
};

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kRB = 16;     // rows per block (the matrix-core tile side)
constexpr int kRWaves = 8;  // waves of k_learn_fwd and k_learn_rows
constexpr int kMaxCG = 8;   // column groups of the row-block kernels (four tiles each)

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// One Adam step (bias-corrected; c1, c2 = 1 - beta^t) on parameter p with
// gradient gi and moments m, v.
__device__ __forceinline__ float adam_step(float& m, float& v, float p, float gi, float lr,
                                           float beta1, float beta2, float eps, float c1,
                                           float c2) {
  m = beta1 * m + (1.0f - beta1) * gi;
  v = beta2 * v + (1.0f - beta2) * gi * gi;
  return p - lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// Tiles on the matrix cores (v_mfma_f32_16x16x4_f32): the sum over k of
// A[r][k] B(k, n0 + j) for the 16 x 16 tile of rows r = 0..15 of a block and
// columns n0..n0 + 15. A sits in LDS, row r at As + r sa, zero in columns K ..
// 16 ceil(K / 16) - 1; B(k, n) = Bp[k sk + n sn] in global memory, vb: sk ==
// 1 and 16-byte aligned rows (then four k in one load). Lane (i, g) = (lane %
// 16, lane / 16) holds A[i][k] and B(k, n0 + i) for k = 16 c + 4 g + t in
// instruction t of chunk c (both operands take the same k, so every k is
// summed once); the chunks are c0, c0 + dc, ... below c1. Element r of the
// result is row 4 g + r, column n0 + i. A column of B only reaches the same
// column of the result, so columns past N read column N - 1 and the caller
// drops them.

// The lane's column of B.
__device__ __forceinline__ const float* b_col(const float* Bp, int sn, int n0, int N) {
  return Bp + (size_t)min(n0 + ((int)threadIdx.x & 15), N - 1) * sn;
}

// B elements of up to PC chunks from cb.
template <int PC>
__device__ __forceinline__ void load_b(float (&bv)[PC][4], const float* bp, int sk, bool vb, int K,
                                       int cb, int c1, int dc) {
  const int g = ((int)threadIdx.x & 63) >> 4;
#pragma unroll
  for (int j = 0; j < PC; ++j) {
    const int c = cb + j * dc, k = 16 * c + 4 * g;
    if (c < c1) {
      if (vb && k + 3 < K) {
        const float4 v = *(const float4*)(bp + k);
        bv[j][0] = v.x, bv[j][1] = v.y, bv[j][2] = v.z, bv[j][3] = v.w;
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) bv[j][t] = k + t < K ? bp[(size_t)(k + t) * sk] : 0.0f;
      }
    }
  }
}

// The whole tile, PC chunks per register piece; bv holds the first piece
// already when pre is set.
template <int PC>
__device__ __forceinline__ f32x4 tile_mfma(float (&bv)[PC][4], bool pre, const float* As, int sa,
                                           const float* bp, int sk, bool vb, int K, int c0, int c1,
                                           int dc) {
  const int lane = (int)threadIdx.x & 63, i = lane & 15, g = lane >> 4;
  const float* ap = As + i * sa + 4 * g;
  f32x4 acc0 = {0.0f, 0.0f, 0.0f, 0.0f}, acc1 = acc0;
  for (int cb = c0; cb < c1; cb += PC * dc) {
    if (!(pre && cb == c0)) load_b<PC>(bv, bp, sk, vb, K, cb, c1, dc);
#pragma unroll
    for (int j = 0; j < PC; ++j) {
      const int c = cb + j * dc;
      if (c < c1) {
        const float4 av = *(const float4*)(ap + 16 * c);
        acc0 = mfma4(av.x, bv[j][0], acc0);
        acc1 = mfma4(av.y, bv[j][1], acc1);
        acc0 = mfma4(av.z, bv[j][2], acc0);
        acc1 = mfma4(av.w, bv[j][3], acc1);
      }
    }
  }
  return acc0 + acc1;
}

// LDS row stride for K columns: room for the zero columns up to a multiple of
// 16, plus 4 to spread the rows over the banks.
__host__ __device__ __forceinline__ int lds_stride(int K) { return ((K + 15) & ~15) + 4; }

// Tiles [tb, te) of nt in column group cg of n_cg.
__device__ __forceinline__ void group_tiles(int nt, int cg, int n_cg, int& tb, int& te) {
  tb = cg * nt / n_cg;
  te = (cg + 1) * nt / n_cg;
}

struct FwdArgs {
  Dims dm;
  int32_t B;
  int32_t pass0;       // the block's pass is pass0 + blockIdx.y
  const float* in[3];  // per pass: input rows [B][d0]
  const float* w[3];   // per pass: weights [W1 | W2 | W3]
  const float* b[3];   // per pass: biases [b1 | b2 | b3]
  int32_t vw;          // the three weight blocks take 16-byte loads
  float* a1;           // pass 0: [B][h1] activations (for back-propagation)
  float* a2;           // pass 0: [B][h2]
  float* q;            // partial sums [group][3][B][A] of the last layer over each
                       // group's units of layer 2, without the bias
};

// One block of 16 rows through the three layers of one pass, for one group
// of the second layer's units (blockIdx.z of gridDim.z): the whole first
// layer, the group's tiles of the second, and the last layer's sum over the
// group's units (the column groups' partial sums are added in group order by
// their reader). Eight waves: each takes every eighth tile of the first
// layer; a pair of waves takes one of the group's (at most four) tiles of the
// second; the last layer's chunks are spread over the waves and their partial
// tiles summed in wave order. Every wave issues the weight loads of its first
// tiles of all three layers before it stages the input, so that the block
// waits for memory about once.
__global__ void __launch_bounds__(kRWaves * 64) k_learn_fwd(FwdArgs f) {
  extern __shared__ __align__(16) float lds[];
  const Dims& d = f.dm;
  const int pass = f.pass0 + (int)blockIdx.y, cg = (int)blockIdx.z, n_cg = (int)gridDim.z;
  const int r0 = (int)blockIdx.x * kRB, rows = min(kRB, f.B - r0);
  const int tid = (int)threadIdx.x, wave = tid >> 6, lane = tid & 63, i = lane & 15, g = lane >> 4;
  const int sx = lds_stride(d.d0), s1 = lds_stride(d.h1), s2 = lds_stride(d.h2);
  float* xs = lds;
  float* h1s = xs + kRB * sx;
  float* h2s = h1s + kRB * s1;
  float* part = h2s + kRB * s2;  // [waves][16 x 16]
  const float* W1 = f.w[pass];
  const float* W2 = W1 + (size_t)d.h1 * d.d0;
  const float* W3 = W2 + (size_t)d.h2 * d.h1;
  const float* b1 = f.b[pass];
  const float* b2 = b1 + d.h1;
  const bool vw = f.vw != 0;
  const int nc0 = (d.d0 + 15) >> 4, nc1 = (d.h1 + 15) >> 4, nc2 = (d.h2 + 15) >> 4;
  const int nt1 = nc1;
  int tb, te;
  group_tiles(nc2, cg, n_cg, tb, te);
  // the wave's first tiles of the three layers
  // at most four second-layer tiles in the group (the host makes enough
  // groups): two waves per tile, each summing every other 16-deep chunk, the
  // partial tiles added in LDS
  const int kp = wave & 1, t2 = tb + (wave >> 1);
  // (the first two first-layer tiles, 64 inputs at a time)
  float p1a[4][4], p1b[4][4], p2[8][4], p3[2][4];
  if (wave < nt1) load_b<4>(p1a, b_col(W1, d.d0, 16 * wave, d.h1), 1, vw, d.d0, 0, nc0, 1);
  if (wave + kRWaves < nt1)
    load_b<4>(p1b, b_col(W1, d.d0, 16 * (wave + kRWaves), d.h1), 1, vw, d.d0, 0, nc0, 1);
  if (t2 < te) load_b<8>(p2, b_col(W2, d.h1, 16 * t2, d.h2), 1, vw, d.h1, kp, nc1, 2);
  load_b<2>(p3, b_col(W3, d.h2, 0, d.A), 1, vw, d.h2, tb + wave, te, kRWaves);
  const float* in = f.in[pass] + (size_t)r0 * d.d0;
  for (int e = tid; e < kRB * sx; e += blockDim.x) {
    const int r = e / sx, k = e % sx;
    xs[e] = (r < rows && k < d.d0) ? in[(size_t)r * d.d0 + k] : 0.0f;
  }
  __syncthreads();
  // out[r][n] = relu(b[n] + acc), written to LDS (zero past N) and, when out
  // is set, to global memory
  auto store = [&](f32x4 acc, int t, const float* bias, int N, float* Os, int so, float* out) {
    const int n = 16 * t + i;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 4 * g + r;
      const float v = n < N ? fmaxf(bias[n] + acc[r], 0.0f) : 0.0f;
      Os[row * so + n] = v;
      if (out && n < N && row < rows) out[(size_t)(r0 + row) * N + n] = v;
    }
  };
  float* a1 = pass == 0 && cg == 0 ? f.a1 : nullptr;
  for (int t = wave; t < nt1; t += kRWaves) {
    const float* bp = b_col(W1, d.d0, 16 * t, d.h1);
    const f32x4 acc = t == wave ? tile_mfma<4>(p1a, true, xs, sx, bp, 1, vw, d.d0, 0, nc0, 1)
                                : tile_mfma<4>(p1b, t == wave + kRWaves, xs, sx, bp, 1, vw, d.d0,
                                               0, nc0, 1);
    store(acc, t, b1, d.h1, h1s, s1, a1);
  }
  __syncthreads();
  {
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    if (t2 < te)
      acc = tile_mfma<8>(p2, true, h1s, s1, b_col(W2, d.h1, 16 * t2, d.h2), 1, vw, d.h1, kp, nc1, 2);
    if (kp == 1)
#pragma unroll
      for (int r = 0; r < 4; ++r) part[wave * 256 + (4 * g + r) * 16 + i] = acc[r];
    __syncthreads();
    if (kp == 0 && t2 < te) {
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] += part[(wave + 1) * 256 + (4 * g + r) * 16 + i];
      store(acc, t2, b2, d.h2, h2s, s2, pass == 0 ? f.a2 : nullptr);
    }
  }
  __syncthreads();  // h2s is complete; the partial tiles are written again
  {
    const f32x4 acc = tile_mfma<2>(p3, true, h2s, s2, b_col(W3, d.h2, 0, d.A), 1, vw, d.h2,
                                   tb + wave, te, kRWaves);
#pragma unroll
    for (int r = 0; r < 4; ++r) part[wave * 256 + (4 * g + r) * 16 + i] = acc[r];
  }
  __syncthreads();
  if (tid < 256) {
    const int row = tid >> 4, o = tid & 15;
    float sum = 0.0f;
    for (int w = 0; w < kRWaves; ++w) sum += part[w * 256 + tid];
    if (row < rows && o < d.A) f.q[(((size_t)cg * 3 + pass) * f.B + r0 + row) * d.A + o] = sum;
  }
}

struct RowsArgs {
  Dims dm;
  int32_t B;
  int32_t n_q;  // column groups of the forward's partial sums
  float gamma, k_h;
  const int32_t* a;
  const float* r;
  const uint8_t* done;
  const float* q;    // partial sums [n_q][3][B][A]
  const float* b3;   // online last-layer bias [A]
  const float* bt3;  // target last-layer bias [A]
  const float* W2;   // online [h2][h1]
  const float* W3;   // online [A][h2]
  const float* a1;   // [B][h1]
  const float* a2;   // [B][h2]
  float* G;          // [B][A]
  float* da2;        // [B][h2]
  float* da1;        // [B][h1]
  float* loss_part;  // [blocks]: the block's Huber sum
};

// Targets, Huber gradients and back-propagated errors of one block of 16 rows
// (see the file head), for one group of da1's columns (blockIdx.y of
// gridDim.y); group 0 also writes G, da2 and the block's Huber sum. Every
// global read that the block needs is issued first: Q (the forward's partial
// sums), the transitions' a, r and done, a2 and W3 into LDS, and each wave's
// W2 columns and relu' mask for its da1 tile.
__global__ void __launch_bounds__(kRWaves * 64) k_learn_rows(RowsArgs f) {
  extern __shared__ __align__(16) float lds[];
  __shared__ float gs[kRB], hub[kRB], qs[kRB][3][16], rs[kRB], part[kRWaves][256];
  __shared__ int32_t as[kRB], ds[kRB];
  const Dims& d = f.dm;
  const int cg = (int)blockIdx.y, n_cg = (int)gridDim.y;
  const int r0 = (int)blockIdx.x * kRB, rows = min(kRB, f.B - r0);
  const int tid = (int)threadIdx.x, wave = tid >> 6, lane = tid & 63, i = lane & 15, g = lane >> 4;
  const int s2 = lds_stride(d.h2);
  float* d2s = lds;             // [16][s2]: a2, then da2
  float* w3s = d2s + kRB * s2;  // [A][h2]
  const int nt1 = (d.h1 + 15) >> 4, nc2 = (d.h2 + 15) >> 4;
  int tb, te;
  group_tiles(nt1, cg, n_cg, tb, te);
  // at most four tiles in the group (the host makes enough groups): two waves
  // per da1 tile, each summing every other 16-deep chunk of h2, their partial
  // tiles added in LDS
  const int kp = wave & 1, t0 = tb + (wave >> 1);
  float pre[8][4];
  float mask[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  if (t0 < te) {
    load_b<8>(pre, b_col(f.W2, 1, 16 * t0, d.h1), d.h1, false, d.h2, kp, nc2, 2);
    const int n = 16 * t0 + i;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (n < d.h1 && 4 * g + r < rows) mask[r] = f.a1[(size_t)(r0 + 4 * g + r) * d.h1 + n];
  }
  // Q of the three passes: bias + the column groups' sums in group order
  for (int e = tid; e < kRB * 3 * d.A; e += blockDim.x) {
    const int r = e / (3 * d.A), pass = (e / d.A) % 3, o = e % d.A;
    if (r < rows) {
      const int b = r0 + r;
      // every group's load in flight together, then the sum in group order
      float v[kMaxCG];
#pragma unroll
      for (int c = 0; c < kMaxCG; ++c)
        v[c] = c < f.n_q ? f.q[(((size_t)c * 3 + pass) * f.B + b) * d.A + o] : 0.0f;
      float sum = 0.0f;
#pragma unroll
      for (int c = 0; c < kMaxCG; ++c) sum += v[c];
      qs[r][pass][o] = (pass == 2 ? f.bt3 : f.b3)[o] + sum;
    }
  }
  if (tid < rows) {
    as[tid] = f.a[r0 + tid];
    rs[tid] = f.r[r0 + tid];
    ds[tid] = f.done[r0 + tid];
  }
  for (int e = tid; e < kRB * s2; e += blockDim.x) {
    const int r = e / s2, u = e % s2;
    d2s[e] = (r < rows && u < d.h2) ? f.a2[(size_t)(r0 + r) * d.h2 + u] : 0.0f;
  }
  for (int e = tid; e < d.A * d.h2; e += blockDim.x) w3s[e] = f.W3[e];
  __syncthreads();
  if (tid < kRB) {
    float gv = 0.0f, hv = 0.0f;
    if (tid < rows) {
      int best = 0;
      for (int o = 1; o < d.A; ++o)
        if (qs[tid][1][o] > qs[tid][1][best]) best = o;
      const float y = rs[tid] + f.gamma * (ds[tid] ? 0.0f : 1.0f) * qs[tid][2][best];
      const float delta = qs[tid][0][as[tid]] - y;
      const float ad = fabsf(delta);
      hv = ad <= f.k_h ? 0.5f * delta * delta : f.k_h * (ad - 0.5f * f.k_h);
      gv = fminf(fmaxf(delta, -f.k_h), f.k_h) / (float)f.B;
    } else {
      as[tid] = 0;
    }
    gs[tid] = gv;
    hub[tid] = hv;
  }
  __syncthreads();
  if (cg == 0 && tid == 0) {
    float sum = 0.0f;
    for (int r = 0; r < kRB; ++r) sum += hub[r];
    f.loss_part[blockIdx.x] = sum;
  }
  if (cg == 0)
    for (int e = tid; e < rows * d.A; e += blockDim.x) {
      const int r = e / d.A, o = e % d.A;
      f.G[(size_t)(r0 + r) * d.A + o] = o == as[r] ? gs[r] : 0.0f;
    }
  for (int e = tid; e < kRB * s2; e += blockDim.x) {
    const int r = e / s2, u = e % s2;
    float v = 0.0f;
    if (r < rows && u < d.h2) {
      v = d2s[e] > 0.0f ? gs[r] * w3s[as[r] * d.h2 + u] : 0.0f;
      if (cg == 0) f.da2[(size_t)(r0 + r) * d.h2 + u] = v;
    }
    d2s[e] = v;
  }
  __syncthreads();
  // da1[r][n] = [a1[r][n] > 0] sum_u da2[r][u] W2[u][n]
  f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  if (t0 < te)
    acc = tile_mfma<8>(pre, true, d2s, s2, b_col(f.W2, 1, 16 * t0, d.h1), d.h1, false, d.h2, kp,
                       nc2, 2);
  if (kp == 1)
#pragma unroll
    for (int r = 0; r < 4; ++r) part[wave][(4 * g + r) * 16 + i] = acc[r];
  __syncthreads();
  if (kp == 0 && t0 < te) {
    const int n = 16 * t0 + i;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 4 * g + r;
      if (n < d.h1 && row < rows) {
        const size_t bn = (size_t)(r0 + row) * d.h1 + n;
        f.da1[bn] = mask[r] > 0.0f ? acc[r] + part[wave + 1][row * 16 + i] : 0.0f;
      }
    }
  }
}

// One weight-gradient product C[m][n] = sum_k X(k, m) Y(k, n) for m < M and
// n < N, X(k, m) = X[k sxk + m], Y(k, n) = Y[k syk + n]; Cb: Cb[m] =
// sum_k X(k, m), computed as column N of a Y with a column of ones (a bias
// gradient). Each entry, once summed, takes its Adam step at once: weight
// pw[m ldc + n] (moments pm, pv), bias qb[m] (moments qm, qv); tw, tb
// (nullable): the target network's copies, written with the new values.
// tile0: the first tile of this product in the launch.
struct MMOp {
  const float* X;
  const float* Y;
  float* C;
  float* Cb;
  float *pw, *pm, *pv, *tw;
  float *qb, *qm, *qv, *tb;
  int32_t sxk, syk, ldc;
  int32_t M, N, K;
  int32_t tiles_n, tile0;
};
struct MMBatch {
  MMOp op[3];
  int32_t n_ops;
  float lr, beta1, beta2, eps, c1, c2;
  const float* loss_part;  // the row blocks' Huber sums
  int32_t n_parts;
  float inv_b;
  float* loss;  // nullable: the mean loss
};

constexpr int kMT = 16;  // output tile side
constexpr int kGW = 4;   // waves per tile, each summing every fourth 16-deep chunk of K
constexpr int kGP = 4;   // chunks of a wave per register piece

// One 16 x 16 output tile per workgroup on the matrix cores (operand layout as
// in tile_mfma, both operands from global memory): each of the four waves
// takes every fourth 16-deep chunk of K, all of a piece's loads in flight
// together, and the four partial tiles are summed in wave order; then each
// thread takes one entry, with the Adam state it loaded first. Rows past M and
// columns past N read a clamped, valid row or column and are not stored.
__global__ void __launch_bounds__(kGW * 64) k_learn_mm(MMBatch bt) {
  __shared__ float part[kGW][256];
  int which = 0;
  for (int q = 1; q < bt.n_ops; ++q)
    if ((int)blockIdx.x >= bt.op[q].tile0) which = q;
  const MMOp& o = bt.op[which];
  const int t = (int)blockIdx.x - o.tile0;
  const int m0 = (t / o.tiles_n) * kMT, n0 = (t % o.tiles_n) * kMT;
  const int tid = (int)threadIdx.x, wave = tid >> 6, lane = tid & 63, i = lane & 15, g = lane >> 4;
  // the thread's entry: row m0 + tid / 16, column n0 + tid % 16
  const int em = m0 + (tid >> 4), en = n0 + (tid & 15);
  const bool eones = o.Cb != nullptr && en == o.N;
  float sm = 0.0f, sv = 0.0f, sp = 0.0f;
  if (em < o.M && en < o.N) {
    const size_t e = (size_t)em * o.ldc + en;
    sm = o.pm[e], sv = o.pv[e], sp = o.pw[e];
  } else if (em < o.M && eones) {
    sm = o.qm[em], sv = o.qv[em], sp = o.qb[em];
  }
  const bool ones = o.Cb != nullptr && n0 + i == o.N;
  const float* xp = o.X + min(m0 + i, o.M - 1);
  const float* yp = o.Y + min(n0 + i, o.N - 1);
  const int nc = (o.K + 15) >> 4;
  f32x4 acc0 = {0.0f, 0.0f, 0.0f, 0.0f}, acc1 = acc0;
  for (int cb = wave; cb < nc; cb += kGW * kGP) {
    float xa[kGP][4], yb[kGP][4];
#pragma unroll
    for (int j = 0; j < kGP; ++j) {
      const int c = cb + j * kGW;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = 16 * c + 4 * g + u;
        const bool in = c < nc && k < o.K;
        xa[j][u] = in ? xp[(size_t)k * o.sxk] : 0.0f;
        yb[j][u] = in ? (ones ? 1.0f : yp[(size_t)k * o.syk]) : 0.0f;
      }
    }
#pragma unroll
    for (int j = 0; j < kGP; ++j) {
      if (cb + j * kGW < nc) {
        acc0 = mfma4(xa[j][0], yb[j][0], acc0);
        acc1 = mfma4(xa[j][1], yb[j][1], acc1);
        acc0 = mfma4(xa[j][2], yb[j][2], acc0);
        acc1 = mfma4(xa[j][3], yb[j][3], acc1);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) part[wave][(4 * g + r) * 16 + i] = acc0[r] + acc1[r];
  if (blockIdx.x == 0 && tid == 0 && bt.loss) {
    // the row blocks' sums in block order, 16 loads in flight at a time
    float sum = 0.0f;
    for (int q0 = 0; q0 < bt.n_parts; q0 += 16) {
      float v[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = q0 + j < bt.n_parts ? bt.loss_part[q0 + j] : 0.0f;
#pragma unroll
      for (int j = 0; j < 16; ++j) sum += v[j];
    }
    bt.loss[0] = sum * bt.inv_b;
  }
  __syncthreads();
  if (em >= o.M) return;
  float gi = 0.0f;
#pragma unroll
  for (int w = 0; w < kGW; ++w) gi += part[w][tid];
  if (en < o.N) {
    const size_t e = (size_t)em * o.ldc + en;
    o.C[e] = gi;
    const float p = adam_step(sm, sv, sp, gi, bt.lr, bt.beta1, bt.beta2, bt.eps, bt.c1, bt.c2);
    o.pm[e] = sm, o.pv[e] = sv, o.pw[e] = p;
    if (o.tw) o.tw[e] = p;
  } else if (eones) {
    o.Cb[em] = gi;
    const float p = adam_step(sm, sv, sp, gi, bt.lr, bt.beta1, bt.beta2, bt.eps, bt.c1, bt.c2);
    o.qm[em] = sm, o.qv[em] = sv, o.qb[em] = p;
    if (o.tb) o.tb[em] = p;
  }
}

// Q from the forward's partial sums: q[e] = b3[e % A] + sum over the groups
// in group order of part[c * stride + e].
__global__ void k_learn_qsum(int64_t n, int32_t A, int32_t n_groups, int64_t stride,
                             const float* __restrict__ part, const float* __restrict__ b3,
                             float* __restrict__ q) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  float sum = 0.0f;
  for (int c = 0; c < n_groups; ++c) sum += part[c * stride + e];
  q[e] = b3[e % A] + sum;
}

__global__ void k_learn_bf16(int64_t n, const float* __restrict__ w, uint16_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = bf16_rne(w[i]);
}

int blocks_for(int64_t n, int t) { return (int)std::max<int64_t>(1, (n + t - 1) / t); }

}  // namespace

struct sparrow_learner {
  Dims dm{};
  sparrow_learner_config cfg{};
  int64_t nw = 0, nb = 0, steps = 0;
  int32_t max_batch = 0;
  hipStream_t stream = nullptr;
  std::vector<void*> allocs;
  // online (w, b), target (wt, bt), Adam moments, gradients
  float *w = nullptr, *b = nullptr, *wt = nullptr, *bt = nullptr;
  float *mw = nullptr, *vw = nullptr, *mb = nullptr, *vb = nullptr, *gw = nullptr, *gb = nullptr;
  // per-batch scratch: activations of the online net on s (kept for
  // back-propagation), Q of the three passes, output error, back-propagated
  // errors and the row blocks' Huber sums
  float *a1 = nullptr, *a2 = nullptr, *q = nullptr;
  float *da1 = nullptr, *da2 = nullptr, *G = nullptr, *loss_part = nullptr;
  size_t fwd_lds = 0, rows_lds = 0;  // dynamic LDS bytes of k_learn_fwd, k_learn_rows
};

namespace {

int lalloc(sparrow_learner* L, float** p, size_t n) {
  if (hipMalloc((void**)p, sizeof(float) * std::max<size_t>(n, 1)) != hipSuccess)
    return fail(SPARROW_ENOMEM, "hipMalloc failed");
  L->allocs.push_back(*p);
  return SPARROW_OK;
}

// One weight-gradient product (see MMOp) with its Adam step.
MMOp grad_op(int M, int N, int K, const float* X, int sxk, const float* Y, int syk, float* C,
             int ldc, float* Cb, float* pw, float* pm, float* pv, float* tw, float* qb, float* qm,
             float* qv, float* tb) {
  MMOp o{};
  o.X = X;
  o.Y = Y;
  o.C = C;
  o.Cb = Cb;
  o.pw = pw, o.pm = pm, o.pv = pv, o.tw = tw;
  o.qb = qb, o.qm = qm, o.qv = qv, o.tb = tb;
  o.sxk = sxk;
  o.syk = syk;
  o.ldc = ldc;
  o.M = M;
  o.N = N;
  o.K = K;
  return o;
}

}  // namespace

int sparrow_learner_create(const int32_t* dims, const float* w_host, const float* b_host,
                           const sparrow_learner_config* cfg, void* hip_stream,
                           sparrow_learner** out) {
  if (!dims || !w_host || !b_host || !cfg || !out) return fail(SPARROW_EINVAL, "NULL argument");
  *out = nullptr;
  const Dims d{dims[0], dims[1], dims[2], dims[3]};
  if (d.d0 < 1 || d.d0 > 128 || d.h1 < 1 || d.h1 > kMaxUnits || d.h2 < 1 || d.h2 > kMaxUnits ||
      d.A < 1 || d.A > 16)
    return fail(SPARROW_EINVAL, "learner dims must be d0 <= 128, h1, h2 <= 512, A <= 16");
  if (cfg->max_batch < 1 || cfg->max_batch > 65535 || !(cfg->lr >= 0.0f) ||
      !(cfg->gamma >= 0.0f) || !(cfg->huber_k > 0.0f) || cfg->target_every < 0)
    return fail(SPARROW_EINVAL, "bad learner configuration");
  auto* L = new sparrow_learner();
  L->dm = d;
  L->cfg = *cfg;
  L->max_batch = cfg->max_batch;
  L->stream = (hipStream_t)hip_stream;
  L->nw = (int64_t)d.h1 * d.d0 + (int64_t)d.h2 * d.h1 + (int64_t)d.A * d.h2;
  L->nb = (int64_t)d.h1 + d.h2 + d.A;
  const size_t B = (size_t)L->max_batch;
  int rc = SPARROW_OK;
  float** big[] = {&L->w, &L->wt, &L->mw, &L->vw, &L->gw};
  float** small[] = {&L->b, &L->bt, &L->mb, &L->vb, &L->gb};
  for (float** p : big)
    if (!rc) rc = lalloc(L, p, (size_t)L->nw);
  for (float** p : small)
    if (!rc) rc = lalloc(L, p, (size_t)L->nb);
  if (!rc) rc = lalloc(L, &L->a1, B * d.h1);
  if (!rc) rc = lalloc(L, &L->a2, B * d.h2);
  if (!rc) rc = lalloc(L, &L->loss_part, (B + kRB - 1) / kRB);
  if (!rc) rc = lalloc(L, &L->da1, B * d.h1);
  if (!rc) rc = lalloc(L, &L->da2, B * d.h2);
  if (!rc) rc = lalloc(L, &L->G, B * d.A);
  if (!rc) rc = lalloc(L, &L->q, (size_t)kMaxCG * 3 * B * d.A);
  // LDS of the row-block kernels: the block's input, hidden activations and
  // the last layer's partial tiles; the block's da2
  L->fwd_lds = sizeof(float) * ((size_t)kRB * (lds_stride(d.d0) + lds_stride(d.h1) +
                                               lds_stride(d.h2)) + (size_t)kRWaves * 256);
  L->rows_lds = sizeof(float) * ((size_t)kRB * lds_stride(d.h2) + (size_t)d.A * d.h2);
  if (!rc && hipFuncSetAttribute((const void*)k_learn_fwd,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)L->fwd_lds) != hipSuccess)
    rc = fail(SPARROW_EHIP, "k_learn_fwd: LDS size not accepted");
  if (!rc && hipFuncSetAttribute((const void*)k_learn_rows,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)L->rows_lds) != hipSuccess)
    rc = fail(SPARROW_EHIP, "k_learn_rows: LDS size not accepted");
  if (rc) {
    sparrow_learner_destroy(L);
    return rc;
  }
  auto up = [&](float* dst, const float* src, int64_t n) {
    return hipMemcpyAsync(dst, src, sizeof(float) * n, hipMemcpyHostToDevice, L->stream);
  };
  hipError_t e = up(L->w, w_host, L->nw);
  if (e == hipSuccess) e = up(L->wt, w_host, L->nw);
  if (e == hipSuccess) e = up(L->b, b_host, L->nb);
  if (e == hipSuccess) e = up(L->bt, b_host, L->nb);
  for (float* p : {L->mw, L->vw})
    if (e == hipSuccess) e = hipMemsetAsync(p, 0, sizeof(float) * L->nw, L->stream);
  for (float* p : {L->mb, L->vb})
    if (e == hipSuccess) e = hipMemsetAsync(p, 0, sizeof(float) * L->nb, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) {
    sparrow_learner_destroy(L);
    return fail(SPARROW_EHIP, std::string("learner upload: ") + hipGetErrorString(e));
  }
  *out = L;
  return SPARROW_OK;
}

// Column groups of the second layer (and of da1): four 16-unit tiles each.
int col_groups(int units) { return std::max(1, ((units + 15) / 16 + 3) / 4); }

// The last layer's partial sums of the online network on s (pass 0,
// activations kept in a1, a2), of the online network on s' (pass 1) and of
// the target network on s' (pass 2): passes pass0 .. pass0 + n_pass - 1 in
// one launch, over the column groups of the second layer.
static int learner_forward(sparrow_learner* L, int32_t B, const float* s, const float* sn,
                           int pass0, int n_pass) {
  const Dims& d = L->dm;
  FwdArgs f{};
  f.dm = d;
  f.B = B;
  f.pass0 = pass0;
  f.in[0] = s, f.in[1] = sn, f.in[2] = sn;
  f.w[0] = L->w, f.w[1] = L->w, f.w[2] = L->wt;
  f.b[0] = L->b, f.b[1] = L->b, f.b[2] = L->bt;
  // 16-byte loads of weight rows: every row and block start on a multiple of 4
  const int64_t o2 = (int64_t)d.h1 * d.d0, o3 = o2 + (int64_t)d.h2 * d.h1;
  f.vw = d.d0 % 4 == 0 && d.h1 % 4 == 0 && d.h2 % 4 == 0 && o2 % 4 == 0 && o3 % 4 == 0;
  f.a1 = L->a1;
  f.a2 = L->a2;
  f.q = L->q;
  hipLaunchKernelGGL(k_learn_fwd, dim3((B + kRB - 1) / kRB, n_pass, col_groups(d.h2)),
                     dim3(kRWaves * 64), L->fwd_lds, L->stream, f);
  HIP_TRY(hipGetLastError());
  return SPARROW_OK;
}

int sparrow_learner_update(sparrow_learner* L, int32_t B, const float* s, const int32_t* a,
                           const float* r, const float* s_next, const uint8_t* done,
                           float* loss) {
  if (!L || !s || !a || !r || !s_next || !done) return fail(SPARROW_EINVAL, "NULL argument");
  if (B < 1 || B > L->max_batch) return fail(SPARROW_EINVAL, "mini-batch size out of range");
  const Dims& d = L->dm;
  int rc = learner_forward(L, B, s, s_next, 0, 3);
  if (rc) return rc;
  const int64_t off2 = (int64_t)d.h1 * d.d0, off3 = off2 + (int64_t)d.h2 * d.h1;
  const int blocks = (B + kRB - 1) / kRB;
  RowsArgs ra{};
  ra.dm = d;
  ra.B = B;
  ra.gamma = L->cfg.gamma;
  ra.k_h = L->cfg.huber_k;
  ra.a = a;
  ra.r = r;
  ra.done = done;
  ra.n_q = col_groups(d.h2);
  ra.q = L->q;
  ra.b3 = L->b + d.h1 + d.h2;
  ra.bt3 = L->bt + d.h1 + d.h2;
  ra.W2 = L->w + off2;
  ra.W3 = L->w + off3;
  ra.a1 = L->a1;
  ra.a2 = L->a2;
  ra.G = L->G;
  ra.da2 = L->da2;
  ra.da1 = L->da1;
  ra.loss_part = L->loss_part;
  hipLaunchKernelGGL(k_learn_rows, dim3(blocks, col_groups(d.h1)), dim3(kRWaves * 64), L->rows_lds,
                     L->stream, ra);
  HIP_TRY(hipGetLastError());
  // gW3[o][u] = sum_b G[b][o] a2[b][u], gb3[o] = sum_b G[b][o];
  // gW2[u][k] = sum_b da2[b][u] a1[b][k], gb2[u] = sum_b da2[b][u];
  // gW1[k][i] = sum_b da1[b][k] s[b][i], gb1[k] = sum_b da1[b][k];
  // each followed by its Adam step, and by the target copy when it is due
  L->steps += 1;
  const bool copy = L->cfg.target_every > 0 && L->steps % L->cfg.target_every == 0;
  const int64_t ob2 = d.h1, ob3 = (int64_t)d.h1 + d.h2;
  auto tw = [&](int64_t off) { return copy ? L->wt + off : nullptr; };
  auto tb = [&](int64_t off) { return copy ? L->bt + off : nullptr; };
  const MMOp ops[3] = {
      grad_op(d.A, d.h2, B, L->G, d.A, L->a2, d.h2, L->gw + off3, d.h2, L->gb + ob3, L->w + off3,
              L->mw + off3, L->vw + off3, tw(off3), L->b + ob3, L->mb + ob3, L->vb + ob3, tb(ob3)),
      grad_op(d.h2, d.h1, B, L->da2, d.h2, L->a1, d.h1, L->gw + off2, d.h1, L->gb + ob2,
              L->w + off2, L->mw + off2, L->vw + off2, tw(off2), L->b + ob2, L->mb + ob2,
              L->vb + ob2, tb(ob2)),
      grad_op(d.h1, d.d0, B, L->da1, d.h1, s, d.d0, L->gw, d.d0, L->gb, L->w, L->mw, L->vw, tw(0),
              L->b, L->mb, L->vb, tb(0))};
  MMBatch bt{};
  int tiles = 0;
  for (const MMOp& o0 : ops) {
    MMOp o = o0;
    o.tiles_n = (o.N + 1 + kMT - 1) / kMT;  // + the column of ones
    o.tile0 = tiles;
    tiles += o.tiles_n * ((o.M + kMT - 1) / kMT);
    bt.op[bt.n_ops++] = o;
  }
  bt.lr = L->cfg.lr;
  bt.beta1 = L->cfg.beta1;
  bt.beta2 = L->cfg.beta2;
  bt.eps = L->cfg.adam_eps;
  bt.c1 = (float)(1.0 - std::pow((double)L->cfg.beta1, (double)L->steps));
  bt.c2 = (float)(1.0 - std::pow((double)L->cfg.beta2, (double)L->steps));
  bt.loss_part = L->loss_part;
  bt.n_parts = blocks;
  bt.inv_b = 1.0f / (float)B;
  bt.loss = loss;
  hipLaunchKernelGGL(k_learn_mm, dim3(tiles), dim3(kGW * 64), 0, L->stream, bt);
  HIP_TRY(hipGetLastError());
  return SPARROW_OK;
}

int sparrow_learner_q(sparrow_learner* L, int32_t which, int32_t n, const float* x, float* q) {
  if (!L || !x || !q || n < 1 || n > L->max_batch || (which != 0 && which != 1))
    return fail(SPARROW_EINVAL, "bad argument");
  // pass 1 computes the online net on its second input, pass 2 the target
  const int pass = which ? 2 : 1;
  int rc = learner_forward(L, n, x, x, pass, 1);
  if (rc) return rc;
  const Dims& d = L->dm;
  const float* b3 = (which ? L->bt : L->b) + d.h1 + d.h2;
  hipLaunchKernelGGL(k_learn_qsum, dim3(blocks_for((int64_t)n * d.A, 256)), dim3(256), 0,
                     L->stream, (int64_t)n * d.A, d.A, col_groups(d.h2), (int64_t)3 * n * d.A,
                     L->q + (size_t)pass * n * d.A, b3, q);
  HIP_TRY(hipGetLastError());
  return SPARROW_OK;
}

int sparrow_learner_export_bf16(sparrow_learner* L, uint16_t* w_bf16, float* b) {
  if (!L || !w_bf16 || !b) return fail(SPARROW_EINVAL, "NULL argument");
  hipLaunchKernelGGL(k_learn_bf16, dim3(blocks_for(L->nw, 256)), dim3(256), 0, L->stream, L->nw,
                     L->w, w_bf16);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(b, L->b, sizeof(float) * L->nb, hipMemcpyDeviceToDevice, L->stream));
  return SPARROW_OK;
}

int sparrow_learner_read(sparrow_learner* L, float* w, float* b, float* wt, float* bt, float* gw,
                         float* gb) {
  if (!L) return fail(SPARROW_EINVAL, "NULL argument");
  HIP_TRY(hipStreamSynchronize(L->stream));
  auto down = [&](float* dst, const float* src, int64_t n) {
    return dst ? hipMemcpy(dst, src, sizeof(float) * n, hipMemcpyDeviceToHost) : hipSuccess;
  };
  HIP_TRY(down(w, L->w, L->nw));
  HIP_TRY(down(b, L->b, L->nb));
  HIP_TRY(down(wt, L->wt, L->nw));
  HIP_TRY(down(bt, L->bt, L->nb));
  HIP_TRY(down(gw, L->gw, L->nw));
  HIP_TRY(down(gb, L->gb, L->nb));
  return SPARROW_OK;
}

int64_t sparrow_learner_steps(const sparrow_learner* L) { return L ? L->steps : -1; }

void sparrow_learner_destroy(sparrow_learner* L) {
  if (!L) return;
  if (L->stream) (void)hipStreamSynchronize(L->stream);
  for (void* p : L->allocs) (void)hipFree(p);
  delete L;
}

// ---------------------------------------------------------------------------
// Time feedback mechanism (Sec. 3.1.2): host-side pacing of actor and learner.
// ---------------------------------------------------------------------------
struct sparrow_tfm {
  double rho = 0.0, v_sum = 0.0, b_sum = 0.0;
  int64_t v_n = 0, b_n = 0;
  mutable std::mutex mu;  // the actor and the learner report from their own threads
};

int sparrow_tfm_create(double rho, sparrow_tfm** out) {
  if (!out) return fail(SPARROW_EINVAL, "NULL argument");
  *out = nullptr;
  if (!(rho > 0.0)) return fail(SPARROW_EINVAL, "rho must be positive");
  auto* t = new sparrow_tfm();
  t->rho = rho;
  *out = t;
  return SPARROW_OK;
}

void sparrow_tfm_actor_period(sparrow_tfm* t, double seconds) {
  if (!t) return;
  std::lock_guard<std::mutex> g(t->mu);
  t->v_sum += seconds;
  t->v_n += 1;
}

void sparrow_tfm_learner_period(sparrow_tfm* t, double seconds) {
  if (!t) return;
  std::lock_guard<std::mutex> g(t->mu);
  t->b_sum += seconds;
  t->b_n += 1;
}

double sparrow_tfm_xi(const sparrow_tfm* t) {
  if (!t) return 0.0;
  std::lock_guard<std::mutex> g(t->mu);
  if (t->v_n == 0 || t->b_n == 0) return 0.0;
  return t->rho * (t->b_sum / (double)t->b_n) - t->v_sum / (double)t->v_n;
}

double sparrow_tfm_actor_sleep(const sparrow_tfm* t) {
  const double xi = sparrow_tfm_xi(t);
  return xi > 0.0 ? xi : 0.0;
}

double sparrow_tfm_learner_sleep(const sparrow_tfm* t) {
  if (!t) return 0.0;
  const double xi = sparrow_tfm_xi(t);
  return xi <= 0.0 ? -xi / t->rho : 0.0;
}

void sparrow_tfm_destroy(sparrow_tfm* t) { delete t; }
