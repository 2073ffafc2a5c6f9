// sparrow_learner.hip -- the learner's update (Alg. 2 step 2: a mini-batch
// sampled from the sharer's buffer trains the learner's model with DDQN;
// Table 6: gamma, learning rate, target-network period, mini-batch 256).
//
// One update on B transitions (s, a, r, s', done), all in FP32 with every sum
// in a fixed order (the products are small -- a 256-row mini-batch through a
// 36-256-256-7 network is ~0.1 GFLOP per pass -- and latency-bound, so the
// vector units serve them and keep them within FP32 rounding of binary64).
// Every product runs through one tiled kernel, k_learn_mm: a launch takes up
// to three independent products C = X^T Y (16 x 16 output tiles, K staged
// through LDS 128 at a time, each output summed in ascending k after its
// bias), so the forward pass is one launch per layer for the three passes
// together and the backward pass two launches:
//   forward       layer l of the online network on s (activations kept for
//                 back-propagation), of the online and of the target network
//                 on s': out = relu(b + W x), the last layer without relu
//   loss + delta  a* = argmax Q_online(s') (lowest index on ties), y = r +
//                 gamma (1 - done) Q_target(s')[a*], delta = Q(s)[a] - y,
//                 dloss/dQ[a] = clip(delta, -k, k) / B, loss = mean Huber;
//                 then the output error G[b][o] = [a_b == o] dloss/dQ_b and
//                 da2[b][u] = [a2 > 0] dloss/dQ_b W3[a_b][u]
//   backward      gW3 = G^T a2, gW2 = da2^T a1 and da1 = [a1 > 0] (da2 W2) in
//                 one launch, then gW1 = da1^T s; each bias gradient is the
//                 column sum of X, an extra column of ones in Y; relu'(0) = 0
//   k_learn_adam  Adam on every weight and bias in one launch; every
//                 target_every-th update the target network becomes a copy
//                 of the online one
// Weights are row-major [out][in], concatenated [W1 | W2 | W3]; biases
// [b1 | b2 | b3].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <initializer_list>
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

// One product C[m][n] = epi(bias[n] + sum_k X(k, m) Y(k, n)) for m < M and
// n < N, X(k, m) = X[k sxk + m sxm], Y(k, n) = Y[k syk + n syn], each output
// summed in ascending k after its bias (bias nullable: 0). relu: max(., 0)
// after the sum; mask: C[m][n] kept only where mask[m ldm + n] > 0 (relu'); Cb:
// Cb[m] = sum_k X(k, m), computed as column N of a Y with a column of ones
// (a bias gradient). tile0: the first tile (workgroup) of this product in
// the launch.
struct MMOp {
  const float* X;
  const float* Y;
  float* C;
  const float* bias;
  const float* mask;
  float* Cb;
  int32_t sxk, sxm, syk, syn, ldc, ldm;
  int32_t M, N, K, relu;
  int32_t tiles_n, tile0;
};
struct MMBatch {
  MMOp op[3];
  int32_t n_ops;
};

constexpr int kMT = 16, kMK = 128;  // output tile side, K chunk
constexpr int kMR = kMT * kMK / 256;  // elements of each operand chunk per thread

__device__ __forceinline__ void mm_load(const MMOp& o, int k0, int m0, int n0, float (&xr)[kMR],
                                        float (&yr)[kMR]) {
  const bool ones = o.Cb != nullptr;
#pragma unroll
  for (int r = 0; r < kMR; ++r) {
    const int e = (int)threadIdx.x + r * 256;  // the chunk's kMK x kMT elements
    // consecutive threads walk the operand's unit-stride index
    const int xk = o.sxm == 1 ? e / kMT : e % kMK, xm = o.sxm == 1 ? e % kMT : e / kMK;
    const int yk = o.syn == 1 ? e / kMT : e % kMK, yn = o.syn == 1 ? e % kMT : e / kMK;
    const int kx = k0 + xk, ky = k0 + yk, m = m0 + xm, n = n0 + yn;
    xr[r] = (kx < o.K && m < o.M) ? o.X[(size_t)kx * o.sxk + (size_t)m * o.sxm] : 0.0f;
    yr[r] = (ky < o.K && n < o.N) ? o.Y[(size_t)ky * o.syk + (size_t)n * o.syn]
            : (ky < o.K && ones && n == o.N) ? 1.0f : 0.0f;
  }
}

// One 16 x 16 output tile per workgroup, one output per thread, summed over
// ascending k after its bias. K goes through LDS 128 at a time (a 256-long
// sum is two chunks); the next chunk's global loads are issued before this
// chunk's multiply-adds.
__global__ void __launch_bounds__(256) k_learn_mm(MMBatch bt) {
  __shared__ float xs[kMK][kMT + 1];
  __shared__ float ys[kMK][kMT + 1];
  int which = 0;
  for (int q = 1; q < bt.n_ops; ++q)
    if ((int)blockIdx.x >= bt.op[q].tile0) which = q;
  const MMOp& o = bt.op[which];
  const int t = (int)blockIdx.x - o.tile0;
  const int m0 = (t / o.tiles_n) * kMT, n0 = (t % o.tiles_n) * kMT;
  const int tn = (int)threadIdx.x % kMT, tm = (int)threadIdx.x / kMT;
  const int m = m0 + tm, n = n0 + tn;
  float acc = (o.bias && n < o.N) ? o.bias[n] : 0.0f;
  float xr[kMR], yr[kMR];
  mm_load(o, 0, m0, n0, xr, yr);
  for (int k0 = 0; k0 < o.K; k0 += kMK) {
    if (k0 > 0) __syncthreads();  // every thread is done with the previous chunk
#pragma unroll
    for (int r = 0; r < kMR; ++r) {
      const int e = (int)threadIdx.x + r * 256;
      const int xk = o.sxm == 1 ? e / kMT : e % kMK, xm = o.sxm == 1 ? e % kMT : e / kMK;
      const int yk = o.syn == 1 ? e / kMT : e % kMK, yn = o.syn == 1 ? e % kMT : e / kMK;
      xs[xk][xm] = xr[r];
      ys[yk][yn] = yr[r];
    }
    __syncthreads();
    if (k0 + kMK < o.K) mm_load(o, k0 + kMK, m0, n0, xr, yr);
    const int kn = min(kMK, o.K - k0);
    for (int kk = 0; kk < kn; ++kk) acc += xs[kk][tm] * ys[kk][tn];
  }
  if (m >= o.M) return;
  if (n < o.N) {
    float v = acc;
    if (o.relu) v = fmaxf(v, 0.0f);
    if (o.mask && !(o.mask[(size_t)m * o.ldm + n] > 0.0f)) v = 0.0f;
    o.C[(size_t)m * o.ldc + n] = v;
  } else if (o.Cb && n == o.N) {
    o.Cb[m] = acc;
  }
}

// Per-row targets and Huber gradients of the whole mini-batch (each
// workgroup computes them all; workgroup 0 also the mean loss by a
// fixed-order tree), then this workgroup's rows of the output error G[b][o]
// = [a_b == o] g_b and of da2[b][u] = [a2[b][u] > 0] g_b W3[a_b][u].
__global__ void __launch_bounds__(1024)
k_learn_loss_delta(Dims dm, int32_t B, int32_t rows_per_block, float gamma, float k_h,
                   const int32_t* __restrict__ a, const float* __restrict__ r,
                   const uint8_t* __restrict__ done, const float* __restrict__ q,
                   const float* __restrict__ W3, const float* __restrict__ a2,
                   float* __restrict__ G, float* __restrict__ da2, float* __restrict__ loss) {
  __shared__ float part[1024];
  __shared__ float gs[1024];
  const int tid = threadIdx.x;
  const int b0 = blockIdx.x * rows_per_block, b1 = min(B, b0 + rows_per_block);
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
    if (b >= b0 && b < b1) gs[b - b0] = fminf(fmaxf(delta, -k_h), k_h) / (float)B;
  }
  part[tid] = acc;
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if (tid < w) part[tid] += part[tid + w];
      __syncthreads();
    }
    if (tid == 0 && loss) loss[0] = part[0] / (float)B;
  }
  const int nrow = b1 - b0;
  for (int e = tid; e < nrow * dm.h2; e += blockDim.x) {
    const int bl = e / dm.h2, u = e % dm.h2, b = b0 + bl;
    const float a2v = a2[(size_t)b * dm.h2 + u];
    da2[(size_t)b * dm.h2 + u] = a2v > 0.0f ? gs[bl] * W3[(size_t)a[b] * dm.h2 + u] : 0.0f;
  }
  for (int e = tid; e < nrow * dm.A; e += blockDim.x) {
    const int bl = e / dm.A, o = e % dm.A, b = b0 + bl;
    G[(size_t)b * dm.A + o] = o == a[b] ? gs[bl] : 0.0f;
  }
}

// Adam on the nw weights (threads [0, nw)) and the nb biases (threads
// [nw, nw + nb)) in one launch.
__global__ void k_learn_adam(int64_t nw, int64_t nb, float* __restrict__ w,
                             float* __restrict__ mw, float* __restrict__ vw,
                             const float* __restrict__ gw, float* __restrict__ b,
                             float* __restrict__ mb, float* __restrict__ vb,
                             const float* __restrict__ gb, float lr, float beta1, float beta2,
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
  p[i] = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
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
  // back-propagation) and of the two passes on s', Q of the three passes,
  // output error and back-propagated errors
  float *a1 = nullptr, *a2 = nullptr, *hs1 = nullptr, *hs2 = nullptr, *q = nullptr;
  float *da1 = nullptr, *da2 = nullptr, *G = nullptr;
};

namespace {

int lalloc(sparrow_learner* L, float** p, size_t n) {
  if (hipMalloc((void**)p, sizeof(float) * std::max<size_t>(n, 1)) != hipSuccess)
    return fail(SPARROW_ENOMEM, "hipMalloc failed");
  L->allocs.push_back(*p);
  return SPARROW_OK;
}

// Launch up to three products as one grid (k_learn_mm).
int launch_mm(sparrow_learner* L, std::initializer_list<MMOp> ops) {
  MMBatch bt{};
  int tiles = 0;
  for (const MMOp& o0 : ops) {
    MMOp o = o0;
    const int cols = o.N + (o.Cb ? 1 : 0);
    o.tiles_n = (cols + kMT - 1) / kMT;
    o.tile0 = tiles;
    tiles += o.tiles_n * ((o.M + kMT - 1) / kMT);
    bt.op[bt.n_ops++] = o;
  }
  hipLaunchKernelGGL(k_learn_mm, dim3(tiles), dim3(256), 0, L->stream, bt);
  HIP_TRY(hipGetLastError());
  return SPARROW_OK;
}

// C = epi(bias + X^T Y) with C (ldc), X (sxk, sxm), Y (syk, syn) strides.
MMOp mm(int M, int N, int K, const float* X, int sxk, int sxm, const float* Y, int syk, int syn,
        float* C, int ldc, const float* bias = nullptr, bool relu = false,
        const float* mask = nullptr, int ldm = 0, float* Cb = nullptr) {
  MMOp o{};
  o.X = X;
  o.Y = Y;
  o.C = C;
  o.bias = bias;
  o.mask = mask;
  o.Cb = Cb;
  o.sxk = sxk;
  o.sxm = sxm;
  o.syk = syk;
  o.syn = syn;
  o.ldc = ldc;
  o.ldm = ldm;
  o.M = M;
  o.N = N;
  o.K = K;
  o.relu = relu ? 1 : 0;
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
  if (!rc) rc = lalloc(L, &L->hs1, 2 * B * d.h1);
  if (!rc) rc = lalloc(L, &L->hs2, 2 * B * d.h2);
  if (!rc) rc = lalloc(L, &L->da1, B * d.h1);
  if (!rc) rc = lalloc(L, &L->da2, B * d.h2);
  if (!rc) rc = lalloc(L, &L->G, B * d.A);
  if (!rc) rc = lalloc(L, &L->q, 3 * B * d.A);
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

// Q of the online network on s (pass 0, activations kept in a1, a2), of the
// online network on s' (pass 1) and of the target network on s' (pass 2):
// one launch per layer for the three passes.
static int learner_forward(sparrow_learner* L, int32_t B, const float* s, const float* sn) {
  const Dims& d = L->dm;
  const size_t o2 = (size_t)d.h1 * d.d0, o3 = o2 + (size_t)d.h2 * d.h1;
  const float* w[3] = {L->w, L->w, L->wt};
  const float* b[3] = {L->b, L->b, L->bt};
  const float* in[3] = {s, sn, sn};
  float* h1[3] = {L->a1, L->hs1, L->hs1 + (size_t)B * d.h1};
  float* h2[3] = {L->a2, L->hs2, L->hs2 + (size_t)B * d.h2};
  int rc = launch_mm(L, {mm(B, d.h1, d.d0, in[0], 1, d.d0, w[0], 1, d.d0, h1[0], d.h1, b[0], true),
                         mm(B, d.h1, d.d0, in[1], 1, d.d0, w[1], 1, d.d0, h1[1], d.h1, b[1], true),
                         mm(B, d.h1, d.d0, in[2], 1, d.d0, w[2], 1, d.d0, h1[2], d.h1, b[2], true)});
  if (rc) return rc;
  rc = launch_mm(L, {mm(B, d.h2, d.h1, h1[0], 1, d.h1, w[0] + o2, 1, d.h1, h2[0], d.h2, b[0] + d.h1, true),
                     mm(B, d.h2, d.h1, h1[1], 1, d.h1, w[1] + o2, 1, d.h1, h2[1], d.h2, b[1] + d.h1, true),
                     mm(B, d.h2, d.h1, h1[2], 1, d.h1, w[2] + o2, 1, d.h1, h2[2], d.h2, b[2] + d.h1, true)});
  if (rc) return rc;
  const size_t bq = (size_t)B * d.A, ob = (size_t)d.h1 + d.h2;
  return launch_mm(L, {mm(B, d.A, d.h2, h2[0], 1, d.h2, w[0] + o3, 1, d.h2, L->q, d.A, b[0] + ob),
                       mm(B, d.A, d.h2, h2[1], 1, d.h2, w[1] + o3, 1, d.h2, L->q + bq, d.A, b[1] + ob),
                       mm(B, d.A, d.h2, h2[2], 1, d.h2, w[2] + o3, 1, d.h2, L->q + 2 * bq, d.A,
                          b[2] + ob)});
}

int sparrow_learner_update(sparrow_learner* L, int32_t B, const float* s, const int32_t* a,
                           const float* r, const float* s_next, const uint8_t* done,
                           float* loss) {
  if (!L || !s || !a || !r || !s_next || !done) return fail(SPARROW_EINVAL, "NULL argument");
  if (B < 1 || B > L->max_batch) return fail(SPARROW_EINVAL, "mini-batch size out of range");
  const Dims& d = L->dm;
  int rc = learner_forward(L, B, s, s_next);
  if (rc) return rc;
  const int64_t off2 = (int64_t)d.h1 * d.d0, off3 = off2 + (int64_t)d.h2 * d.h1;
  const float* W2 = L->w + off2;
  const float* W3 = L->w + off3;
  const int rows = 16;
  hipLaunchKernelGGL(k_learn_loss_delta, dim3((B + rows - 1) / rows), dim3(1024), 0, L->stream, d,
                     B, rows, L->cfg.gamma, L->cfg.huber_k, a, r, done, L->q, W3, L->a2, L->G,
                     L->da2, loss);
  HIP_TRY(hipGetLastError());
  // gW3[o][u] = sum_b G[b][o] a2[b][u], gb3[o] = sum_b G[b][o];
  // gW2[u][k] = sum_b da2[b][u] a1[b][k], gb2[u] = sum_b da2[b][u];
  // da1[b][k] = [a1[b][k] > 0] sum_u da2[b][u] W2[u][k]
  rc = launch_mm(L, {mm(d.A, d.h2, B, L->G, d.A, 1, L->a2, d.h2, 1, L->gw + off3, d.h2, nullptr,
                        false, nullptr, 0, L->gb + d.h1 + d.h2),
                     mm(d.h2, d.h1, B, L->da2, d.h2, 1, L->a1, d.h1, 1, L->gw + off2, d.h1, nullptr,
                        false, nullptr, 0, L->gb + d.h1),
                     mm(B, d.h1, d.h2, L->da2, 1, d.h2, W2, d.h1, 1, L->da1, d.h1, nullptr, false,
                        L->a1, d.h1)});
  if (rc) return rc;
  // gW1[k][i] = sum_b da1[b][k] s[b][i], gb1[k] = sum_b da1[b][k]
  rc = launch_mm(L, {mm(d.h1, d.d0, B, L->da1, d.h1, 1, s, d.d0, 1, L->gw, d.d0, nullptr, false,
                        nullptr, 0, L->gb)});
  if (rc) return rc;
  L->steps += 1;
  const double c1 = 1.0 - std::pow((double)L->cfg.beta1, (double)L->steps);
  const double c2 = 1.0 - std::pow((double)L->cfg.beta2, (double)L->steps);
  hipLaunchKernelGGL(k_learn_adam, dim3(blocks_for(L->nw + L->nb, 256)), dim3(256), 0, L->stream,
                     L->nw, L->nb, L->w, L->mw, L->vw, L->gw, L->b, L->mb, L->vb, L->gb,
                     L->cfg.lr, L->cfg.beta1, L->cfg.beta2, L->cfg.adam_eps, (float)c1, (float)c2);
  HIP_TRY(hipGetLastError());
  if (L->cfg.target_every > 0 && L->steps % L->cfg.target_every == 0) {
    HIP_TRY(hipMemcpyAsync(L->wt, L->w, sizeof(float) * L->nw, hipMemcpyDeviceToDevice, L->stream));
    HIP_TRY(hipMemcpyAsync(L->bt, L->b, sizeof(float) * L->nb, hipMemcpyDeviceToDevice, L->stream));
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
