// sparrow_learner.hip -- the learner's update (Alg. 2 step 2: a mini-batch
// sampled from the sharer's buffer trains the learner's model with DDQN;
// Table 6: gamma, learning rate, target-network period, mini-batch 256).
//
// One update on B transitions (s, a, r, s', done), all in FP32 with every sum
// in a fixed order (the products are small -- a 256-row mini-batch through a
// 36-256-256-7 network is ~0.1 GFLOP per pass -- and latency-bound, so the
// vector units serve them and keep them within FP32 rounding of binary64):
//   k_learn_fwd   Q of the online network on s (its activations kept for
//                 back-propagation), of the online and the target network on
//                 s'; one workgroup per (pass, row), one thread per unit
//   k_learn_loss  a* = argmax Q_online(s') (lowest index on ties), y = r +
//                 gamma (1 - done) Q_target(s')[a*], delta = Q(s)[a] - y,
//                 dloss/dQ[a] = clip(delta, -k, k) / B, loss = mean Huber
//   k_learn_delta G[b][o] = [a_b == o] dloss/dQ_b (the output error as a
//                 B x A matrix) and da2[b][u] = [a2 > 0] dloss/dQ_b W3[a_b][u]
//   k_learn_gemm  back-propagation as four small products, C = X^T Y over
//                 the mini-batch (or over the units for da1), tiled through
//                 LDS: gW3 = G^T a2, gW2 = da2^T a1, da1 = [a1 > 0] (da2 W2),
//                 gW1 = da1^T s; each bias gradient is the column sum of X,
//                 computed as an extra column of ones in Y; relu'(0) = 0
//   k_learn_adam  Adam on every weight and bias in one launch, writing the
//                 transposed copies the forward pass reads as it goes; every
//                 target_every-th update the target network becomes a copy
//                 of the online one
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

struct Net {  // device views of one network
  const float* W1T;  // [d0][h1] (transposed copy for the forward pass)
  const float* W2T;  // [h1][h2]
  const float* W3;   // [A][h2]
  const float* b1;
  const float* b2;
  const float* b3;
};

struct Dims {
  int32_t d0, h1, h2, A;
};

// pass 0: online on s (activations kept), 1: online on s', 2: target on s'
__global__ void __launch_bounds__(kMaxUnits)
k_learn_fwd(Dims dm, Net on, Net tg, int32_t B, const float* __restrict__ s,
            const float* __restrict__ sn, float* __restrict__ a1_out, float* __restrict__ a2_out,
            float* __restrict__ q_out /* [3][B][A] */) {
  __shared__ float x[128];
  __shared__ float h1v[kMaxUnits];
  __shared__ float h2v[kMaxUnits];
  const int pass = blockIdx.y, row = blockIdx.x, tid = threadIdx.x;
  const Net& n = pass == 2 ? tg : on;
  const float* src = (pass == 0 ? s : sn) + (size_t)row * dm.d0;
  for (int k = tid; k < dm.d0; k += blockDim.x) x[k] = src[k];
  __syncthreads();
  if (tid < dm.h1) {
    float acc = n.b1[tid];
    for (int k = 0; k < dm.d0; ++k) acc += n.W1T[(size_t)k * dm.h1 + tid] * x[k];
    const float a = fmaxf(acc, 0.0f);
    h1v[tid] = a;
    if (pass == 0) a1_out[(size_t)row * dm.h1 + tid] = a;
  }
  __syncthreads();
  if (tid < dm.h2) {
    float acc = n.b2[tid];
    for (int k = 0; k < dm.h1; ++k) acc += n.W2T[(size_t)k * dm.h2 + tid] * h1v[k];
    const float a = fmaxf(acc, 0.0f);
    h2v[tid] = a;
    if (pass == 0) a2_out[(size_t)row * dm.h2 + tid] = a;
  }
  __syncthreads();
  // output o: 32 lanes take every 32nd unit, then a fixed-order halving sum
  const int o = tid >> 5, j = tid & 31;
  float part = 0.0f;
  if (o < dm.A)
    for (int k = j; k < dm.h2; k += 32) part += n.W3[(size_t)o * dm.h2 + k] * h2v[k];
  for (int off = 16; off > 0; off >>= 1) part += __shfl_down(part, off, 32);
  if (o < dm.A && j == 0) q_out[((size_t)pass * B + row) * dm.A + o] = n.b3[o] + part;
}

// One workgroup: per-row targets and Huber gradients, then the mean loss by a
// fixed-order tree.
__global__ void __launch_bounds__(1024)
k_learn_loss(Dims dm, int32_t B, float gamma, float k_h, const int32_t* __restrict__ a,
             const float* __restrict__ r, const uint8_t* __restrict__ done,
             const float* __restrict__ q, float* __restrict__ g_out, float* __restrict__ loss) {
  __shared__ float part[1024];
  const int tid = threadIdx.x;
  float acc = 0.0f;
  for (int b = tid; b < B; b += blockDim.x) {
    const float* qon_s = q + (size_t)b * dm.A;
    const float* qon_n = q + ((size_t)B + b) * dm.A;
    const float* qtg_n = q + ((size_t)2 * B + b) * dm.A;
    int best = 0;
    for (int o = 1; o < dm.A; ++o)
      if (qon_n[o] > qon_n[best]) best = o;
    const float y = r[b] + gamma * (done[b] ? 0.0f : 1.0f) * qtg_n[best];
    const float delta = qon_s[a[b]] - y;
    const float ad = fabsf(delta);
    acc += ad <= k_h ? 0.5f * delta * delta : k_h * (ad - 0.5f * k_h);
    g_out[b] = fminf(fmaxf(delta, -k_h), k_h) / (float)B;
  }
  part[tid] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (tid < w) part[tid] += part[tid + w];
    __syncthreads();
  }
  if (tid == 0 && loss) loss[0] = part[0] / (float)B;
}

// G[b][o] = [a_b == o] g_b (B x A); da2[b][u] = [a2[b][u] > 0] g_b W3[a_b][u]
__global__ void k_learn_delta(Dims dm, int32_t B, const int32_t* __restrict__ a,
                              const float* __restrict__ g, const float* __restrict__ W3,
                              const float* __restrict__ a2, float* __restrict__ G,
                              float* __restrict__ da2) {
  const int b = blockIdx.x;
  const float gb = g[b];
  const int ab = a[b];
  for (int u = threadIdx.x; u < dm.h2; u += blockDim.x) {
    const float a2v = a2[(size_t)b * dm.h2 + u];
    da2[(size_t)b * dm.h2 + u] = a2v > 0.0f ? gb * W3[(size_t)ab * dm.h2 + u] : 0.0f;
  }
  for (int o = threadIdx.x; o < dm.A; o += blockDim.x)
    G[(size_t)b * dm.A + o] = o == ab ? gb : 0.0f;
}

// C[m][n] = sum_k X(k, m) Y(k, n), X(k, m) = X[k sxk + m sxm], Y(k, n) =
// Y[k syk + n syn], for m < M and n < N; with Cb, column N of Y is ones and
// Cb[m] = sum_k X(k, m) (a bias gradient); with mask, C[m][n] is kept only
// where mask[m ldm + n] > 0 (relu'). 32 x 32 output tiles, 256 threads of
// 2 x 2 outputs, K in chunks of 16 staged through LDS with the next chunk's
// loads in flight during the current chunk's products. Each output sums its
// K terms in ascending k.
constexpr int kGT = 32, kGK = 16;

__device__ __forceinline__ void gemm_load(const float* X, int sxk, int sxm, int M, const float* Y,
                                          int syk, int syn, int N, bool ones, int K, int k0,
                                          int m0, int n0, float (&xr)[2], float (&yr)[2]) {
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int e = threadIdx.x + r * 256;  // 512 elements of each 16 x 32 tile
    // consecutive threads walk the operand's unit-stride index
    const int xk = sxm == 1 ? e / kGT : e % kGK, xm = sxm == 1 ? e % kGT : e / kGK;
    const int yk = syn == 1 ? e / kGT : e % kGK, yn = syn == 1 ? e % kGT : e / kGK;
    const int kx = k0 + xk, ky = k0 + yk, m = m0 + xm, n = n0 + yn;
    xr[r] = (kx < K && m < M) ? X[(size_t)kx * sxk + (size_t)m * sxm] : 0.0f;
    yr[r] = (ky < K && n < N) ? Y[(size_t)ky * syk + (size_t)n * syn]
            : (ky < K && ones && n == N) ? 1.0f : 0.0f;
  }
}

__global__ void __launch_bounds__(256)
k_learn_gemm(int M, int N, int K, const float* __restrict__ X, int sxk, int sxm,
             const float* __restrict__ Y, int syk, int syn, float* __restrict__ C, int ldc,
             float* __restrict__ Cb, const float* __restrict__ mask, int ldm) {
  __shared__ float xs[kGK][kGT];
  __shared__ float ys[kGK][kGT];
  const int m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
  const int tm = (threadIdx.x / 16) * 2, tn = (threadIdx.x % 16) * 2;
  const bool ones = Cb != nullptr;
  float acc[2][2] = {{0.0f, 0.0f}, {0.0f, 0.0f}};
  float xr[2], yr[2];
  gemm_load(X, sxk, sxm, M, Y, syk, syn, N, ones, K, 0, m0, n0, xr, yr);
  for (int k0 = 0; k0 < K; k0 += kGK) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int e = threadIdx.x + r * 256;
      const int xk = sxm == 1 ? e / kGT : e % kGK, xm = sxm == 1 ? e % kGT : e / kGK;
      const int yk = syn == 1 ? e / kGT : e % kGK, yn = syn == 1 ? e % kGT : e / kGK;
      xs[xk][xm] = xr[r];
      ys[yk][yn] = yr[r];
    }
    __syncthreads();
    if (k0 + kGK < K)
      gemm_load(X, sxk, sxm, M, Y, syk, syn, N, ones, K, k0 + kGK, m0, n0, xr, yr);
#pragma unroll
    for (int kk = 0; kk < kGK; ++kk) {
      const float x0 = xs[kk][tm], x1 = xs[kk][tm + 1];
      const float y0 = ys[kk][tn], y1 = ys[kk][tn + 1];
      acc[0][0] += x0 * y0;
      acc[0][1] += x0 * y1;
      acc[1][0] += x1 * y0;
      acc[1][1] += x1 * y1;
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int m = m0 + tm + i, n = n0 + tn + j;
      if (m >= M) continue;
      if (n < N) {
        float v = acc[i][j];
        if (mask && !(mask[(size_t)m * ldm + n] > 0.0f)) v = 0.0f;
        C[(size_t)m * ldc + n] = v;
      } else if (ones && n == N) {
        Cb[m] = acc[i][j];
      }
    }
}

// Adam on the nw weights (threads [0, nw)) and the nb biases (threads
// [nw, nw + nb)) in one launch; each updated W1 or W2 entry is also written to
// the transposed copy the forward pass reads.
__global__ void k_learn_adam(Dims dm, int64_t nw, int64_t nb, float* __restrict__ w,
                             float* __restrict__ mw, float* __restrict__ vw,
                             const float* __restrict__ gw, float* __restrict__ b,
                             float* __restrict__ mb, float* __restrict__ vb,
                             const float* __restrict__ gb, float* __restrict__ w1t,
                             float* __restrict__ w2t, float lr, float beta1, float beta2,
                             float eps, float c1, float c2) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nw + nb) return;
  const bool is_w = t < nw;
  const int64_t i = is_w ? t : t - nw;
  float* p = is_w ? w : b;
  float* m = is_w ? mw : mb;
  float* v = is_w ? vw : vb;
  const float gi = (is_w ? gw : gb)[i];
  const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
  const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  if (!is_w) return;
  const int64_t n1 = (int64_t)dm.h1 * dm.d0, n2 = (int64_t)dm.h2 * dm.h1;
  if (i < n1) {
    const int64_t r = i / dm.d0, c = i % dm.d0;  // W1[r][c] -> W1T[c][r]
    w1t[c * dm.h1 + r] = pi;
  } else if (i < n1 + n2) {
    const int64_t j = i - n1, r = j / dm.h1, c = j % dm.h1;  // W2[r][c] -> W2T[c][r]
    w2t[c * dm.h2 + r] = pi;
  }
}

// W [rows][cols] -> WT [cols][rows]
__global__ void k_learn_transpose(const float* __restrict__ W, float* __restrict__ WT, int rows,
                                  int cols) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * cols) return;
  const int r = t / cols, c = t % cols;
  WT[(size_t)c * rows + r] = W[t];
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
  // online (w, b), target (wt, bt), Adam moments, gradients, transposes
  float *w = nullptr, *b = nullptr, *wt = nullptr, *bt = nullptr;
  float *mw = nullptr, *vw = nullptr, *mb = nullptr, *vb = nullptr, *gw = nullptr, *gb = nullptr;
  float *w1t = nullptr, *w2t = nullptr, *w1t_t = nullptr, *w2t_t = nullptr;
  // per-batch scratch
  float *a1 = nullptr, *a2 = nullptr, *q = nullptr, *g = nullptr, *da1 = nullptr;
  float *da2 = nullptr, *G = nullptr;
};

namespace {

int lalloc(sparrow_learner* L, float** p, size_t n) {
  if (hipMalloc((void**)p, sizeof(float) * std::max<size_t>(n, 1)) != hipSuccess)
    return fail(SPARROW_ENOMEM, "hipMalloc failed");
  L->allocs.push_back(*p);
  return SPARROW_OK;
}

Net net_of(const sparrow_learner* L, bool target) {
  const Dims& d = L->dm;
  const float* w = target ? L->wt : L->w;
  const float* b = target ? L->bt : L->b;
  Net n;
  n.W1T = target ? L->w1t_t : L->w1t;
  n.W2T = target ? L->w2t_t : L->w2t;
  n.W3 = w + (size_t)d.h1 * d.d0 + (size_t)d.h2 * d.h1;
  n.b1 = b;
  n.b2 = b + d.h1;
  n.b3 = b + d.h1 + d.h2;
  return n;
}

int refresh_transposes(sparrow_learner* L, bool target) {
  const Dims& d = L->dm;
  const float* w = target ? L->wt : L->w;
  const int n1 = d.h1 * d.d0, n2 = d.h2 * d.h1;
  hipLaunchKernelGGL(k_learn_transpose, dim3(blocks_for(n1, 256)), dim3(256), 0, L->stream, w,
                     target ? L->w1t_t : L->w1t, d.h1, d.d0);
  hipLaunchKernelGGL(k_learn_transpose, dim3(blocks_for(n2, 256)), dim3(256), 0, L->stream,
                     w + n1, target ? L->w2t_t : L->w2t, d.h2, d.h1);
  HIP_TRY(hipGetLastError());
  return SPARROW_OK;
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
  if (!rc) rc = lalloc(L, &L->w1t, (size_t)d.h1 * d.d0);
  if (!rc) rc = lalloc(L, &L->w2t, (size_t)d.h2 * d.h1);
  if (!rc) rc = lalloc(L, &L->w1t_t, (size_t)d.h1 * d.d0);
  if (!rc) rc = lalloc(L, &L->w2t_t, (size_t)d.h2 * d.h1);
  if (!rc) rc = lalloc(L, &L->a1, B * d.h1);
  if (!rc) rc = lalloc(L, &L->a2, B * d.h2);
  if (!rc) rc = lalloc(L, &L->da1, B * d.h1);
  if (!rc) rc = lalloc(L, &L->da2, B * d.h2);
  if (!rc) rc = lalloc(L, &L->G, B * d.A);
  if (!rc) rc = lalloc(L, &L->q, 3 * B * d.A);
  if (!rc) rc = lalloc(L, &L->g, B);
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
  rc = refresh_transposes(L, false);
  if (!rc) rc = refresh_transposes(L, true);
  if (rc) {
    sparrow_learner_destroy(L);
    return rc;
  }
  *out = L;
  return SPARROW_OK;
}

static int learner_forward(sparrow_learner* L, int32_t B, const float* s, const float* sn) {
  const Dims& d = L->dm;
  const int threads = std::max(64, ((std::max({d.h1, d.h2, 32 * d.A}) + 63) / 64) * 64);
  hipLaunchKernelGGL(k_learn_fwd, dim3(B, 3), dim3(threads), 0, L->stream, d, net_of(L, false),
                     net_of(L, true), B, s, sn, L->a1, L->a2, L->q);
  HIP_TRY(hipGetLastError());
  return SPARROW_OK;
}

int sparrow_learner_update(sparrow_learner* L, int32_t B, const float* s, const int32_t* a,
                           const float* r, const float* s_next, const uint8_t* done,
                           float* loss) {
  if (!L || !s || !a || !r || !s_next || !done) return fail(SPARROW_EINVAL, "NULL argument");
  if (B < 1 || B > L->max_batch) return fail(SPARROW_EINVAL, "mini-batch size out of range");
  const Dims& d = L->dm;
  int rc = learner_forward(L, B, s, s_next);
  if (rc) return rc;
  hipLaunchKernelGGL(k_learn_loss, dim3(1), dim3(1024), 0, L->stream, d, B, L->cfg.gamma,
                     L->cfg.huber_k, a, r, done, L->q, L->g, loss);
  const int64_t off2 = (int64_t)d.h1 * d.d0, off3 = off2 + (int64_t)d.h2 * d.h1;
  const float* W2 = L->w + off2;
  const float* W3 = L->w + off3;
  hipLaunchKernelGGL(k_learn_delta, dim3(B), dim3(256), 0, L->stream, d, B, a, L->g, W3, L->a2,
                     L->G, L->da2);
  // C[M][N] (+ bias column) = X^T Y over K
  auto gemm = [&](int M, int N, int K, const float* X, int sxk, int sxm, const float* Y, int syk,
                  int syn, float* C, int ldc, float* Cb, const float* mask, int ldm) {
    const int cols = N + (Cb ? 1 : 0);
    hipLaunchKernelGGL(k_learn_gemm, dim3((cols + kGT - 1) / kGT, (M + kGT - 1) / kGT), dim3(256),
                       0, L->stream, M, N, K, X, sxk, sxm, Y, syk, syn, C, ldc, Cb, mask, ldm);
  };
  // gW3[o][u] = sum_b G[b][o] a2[b][u]; gb3[o] = sum_b G[b][o]
  gemm(d.A, d.h2, B, L->G, d.A, 1, L->a2, d.h2, 1, L->gw + off3, d.h2, L->gb + d.h1 + d.h2,
       nullptr, 0);
  // gW2[u][k] = sum_b da2[b][u] a1[b][k]; gb2[u] = sum_b da2[b][u]
  gemm(d.h2, d.h1, B, L->da2, d.h2, 1, L->a1, d.h1, 1, L->gw + off2, d.h1, L->gb + d.h1, nullptr,
       0);
  // da1[b][k] = [a1[b][k] > 0] sum_u da2[b][u] W2[u][k]
  gemm(B, d.h1, d.h2, L->da2, 1, d.h2, W2, d.h1, 1, L->da1, d.h1, nullptr, L->a1, d.h1);
  // gW1[k][i] = sum_b da1[b][k] s[b][i]; gb1[k] = sum_b da1[b][k]
  gemm(d.h1, d.d0, B, L->da1, d.h1, 1, s, d.d0, 1, L->gw, d.d0, L->gb, nullptr, 0);
  HIP_TRY(hipGetLastError());
  L->steps += 1;
  const double c1 = 1.0 - std::pow((double)L->cfg.beta1, (double)L->steps);
  const double c2 = 1.0 - std::pow((double)L->cfg.beta2, (double)L->steps);
  hipLaunchKernelGGL(k_learn_adam, dim3(blocks_for(L->nw + L->nb, 256)), dim3(256), 0, L->stream,
                     d, L->nw, L->nb, L->w, L->mw, L->vw, L->gw, L->b, L->mb, L->vb, L->gb,
                     L->w1t, L->w2t, L->cfg.lr, L->cfg.beta1, L->cfg.beta2, L->cfg.adam_eps,
                     (float)c1, (float)c2);
  HIP_TRY(hipGetLastError());
  if (L->cfg.target_every > 0 && L->steps % L->cfg.target_every == 0) {
    HIP_TRY(hipMemcpyAsync(L->wt, L->w, sizeof(float) * L->nw, hipMemcpyDeviceToDevice, L->stream));
    HIP_TRY(hipMemcpyAsync(L->bt, L->b, sizeof(float) * L->nb, hipMemcpyDeviceToDevice, L->stream));
    rc = refresh_transposes(L, true);
    if (rc) return rc;
  }
  return SPARROW_OK;
}

int sparrow_learner_q(sparrow_learner* L, int32_t which, int32_t n, const float* x, float* q) {
  if (!L || !x || !q || n < 1 || n > L->max_batch || (which != 0 && which != 1))
    return fail(SPARROW_EINVAL, "bad argument");
  // pass 1 computes the online net on its second input, pass 2 the target
  int rc = learner_forward(L, n, x, x);
  if (rc) return rc;
  const size_t A = (size_t)L->dm.A;
  HIP_TRY(hipMemcpyAsync(q, L->q + (size_t)(which ? 2 : 1) * n * A, sizeof(float) * n * A,
                         hipMemcpyDeviceToDevice, L->stream));
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
