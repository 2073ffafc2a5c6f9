// sparrow_ring.hip -- the experience buffer on the device (Sec. 3.1.2: Alg. 1
// step 5 adds each batch of transitions, Alg. 2 step 1 samples a mini-batch;
// Table 6 sizes it at 1 M transitions and the mini-batch at 256).
//
// Storage: sparrow_ring_dev.h (structure of arrays over the slots).
// A push writes a contiguous run of slots (one wrap at most); a wave per
// transition reads its FP32 rows coalesced and writes the encoded rows next
// to each other.
//
// Kernels:
//   k_ring_push   encode n transitions into slots head .. head + n - 1 (mod cap)
//   k_ring_read   decode B slots (drawn by Philox, or given) back to FP32
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sparrow.h"
#include "sparrow_device.h"
#include "sparrow_host.h"
#include "sparrow_ring_dev.h"

using namespace sp;

namespace {

constexpr uint32_t kRingSample = 8;  // Philox counter word 2 of the sampler
constexpr int kScalars = kRingScalars;
constexpr int kRingThreads = 256;

// One wave per transition: lanes take the row's entries, so the FP32 rows
// are read and the encoded rows written contiguously with no division.
__global__ void __launch_bounds__(kRingThreads)
k_ring_push(RingDev R, int64_t head, int32_t n, const float* __restrict__ s,
            const int32_t* __restrict__ a, const float* __restrict__ r,
            const float* __restrict__ sn, const float* __restrict__ sf,
            const uint8_t* __restrict__ done) {
  const int D = R.nr + kScalars;
  const int lane = threadIdx.x & 63;
  const int waves = gridDim.x * (kRingThreads / 64);
  for (int i = blockIdx.x * (kRingThreads / 64) + (threadIdx.x >> 6); i < n; i += waves) {
    int64_t slot = head + i;  // head < cap and i < n <= cap: at most one wrap
    if (slot >= R.cap) slot -= R.cap;
    const bool d = done[i] != 0;
    const float* srow = s + (size_t)i * D;
    const float* nrow = ((d && sf) ? sf : sn) + (size_t)i * D;
    for (int j = lane; j < D; j += 64) {
      const float v = srow[j], vn = nrow[j];
      if (j < R.nr) {
        R.rs[slot * R.nr + j] = quant_u8(v);
        R.rsn[slot * R.nr + j] = quant_u8(vn);
      } else {
        R.cs[slot * kScalars + (j - R.nr)] = f16_bits(v);
        R.csn[slot * kScalars + (j - R.nr)] = f16_bits(vn);
      }
    }
    if (lane == 0) {
      R.act[slot] = (int8_t)a[i];
      R.rew[slot] = r[i];
    }
  }
  // Done bits: one thread owns each 32-slot word the add touches and
  // rebuilds it, keeping the bits of slots outside the add, so no atomics.
  // Without a wrap the touched words are one run; an add that wraps (rare)
  // visits every word, so no word has two owners.
  const bool wraps = head + n > R.cap;
  const int64_t w0 = wraps ? 0 : head >> 5;
  const int64_t w1 = wraps ? ((int64_t)R.cap - 1) >> 5 : (head + n - 1) >> 5;
  for (int64_t w = w0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w <= w1;
       w += (int64_t)gridDim.x * blockDim.x) {
    uint32_t bits = 0, keep = 0;
    for (int b = 0; b < 32; ++b) {
      const int64_t slot = w * 32 + b;
      int64_t i = slot - head;  // index in the add, modulo the capacity
      if (i < 0) i += R.cap;
      if (slot < R.cap && i < n)
        bits |= (done[i] != 0 ? 1u : 0u) << b;
      else
        keep |= 1u << b;
    }
    uint32_t* dst = &R.done[w];
    *dst = keep ? ((*dst & keep) | bits) : bits;
  }
}

// Clear the done bits of slots head .. head + n - 1 (mod cap) and keep the
// others, one thread per word (the same word walk as the push): a kernel
// that adds those n transitions afterwards only sets the bits of done slots.
__global__ void __launch_bounds__(kRingThreads)
k_ring_clear_done(RingDev R, int64_t head, int64_t n) {
  const bool wraps = head + n > R.cap;
  const int64_t w0 = wraps ? 0 : head >> 5;
  const int64_t w1 = wraps ? ((int64_t)R.cap - 1) >> 5 : (head + n - 1) >> 5;
  for (int64_t w = w0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w <= w1;
       w += (int64_t)gridDim.x * blockDim.x) {
    uint32_t keep = 0;
    for (int b = 0; b < 32; ++b) {
      const int64_t slot = w * 32 + b;
      int64_t i = slot - head;
      if (i < 0) i += R.cap;
      if (!(slot < R.cap && i < n)) keep |= 1u << b;
    }
    R.done[w] &= keep;
  }
}

// Decode B slots. With `slots` NULL, slot b is floor(w * size / 2^32) for the
// first word w of Philox (b, draw, 8, 0); every entry of a row recomputes it,
// which costs less than a second launch.
__global__ void __launch_bounds__(kRingThreads)
k_ring_read(RingDev R, uint32_t size, int32_t B, uint32_t draw, uint32_t key0, uint32_t key1,
            const int32_t* __restrict__ slots, float* __restrict__ s, int32_t* __restrict__ a,
            float* __restrict__ r, float* __restrict__ sn, uint8_t* __restrict__ done,
            int32_t* __restrict__ idx) {
  const int D = R.nr + kScalars;
  const int total = B * D;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
    const int b = t / D, j = t - b * D;
    int64_t slot;
    if (slots) {
      slot = slots[b];
    } else {
      const U4 w = philox((uint32_t)b, draw, kRingSample, 0u, key0, key1);
      slot = scale_u32(w.x, size);
    }
    if (j < R.nr) {
      if (s) s[t] = dequant_u8(R.rs[slot * R.nr + j]);
      if (sn) sn[t] = dequant_u8(R.rsn[slot * R.nr + j]);
    } else {
      if (s) s[t] = f16_value(R.cs[slot * kScalars + (j - R.nr)]);
      if (sn) sn[t] = f16_value(R.csn[slot * kScalars + (j - R.nr)]);
    }
    if (j == 0) {
      if (a) a[b] = R.act[slot];
      if (r) r[b] = R.rew[slot];
      if (done) done[b] = (uint8_t)((R.done[slot >> 5] >> (uint32_t)(slot & 31)) & 1u);
      if (idx) idx[b] = (int32_t)slot;
    }
  }
}

int grid_for(int64_t work) {
  const int64_t blocks = (work + kRingThreads - 1) / kRingThreads;
  return (int)std::max<int64_t>(1, std::min<int64_t>(blocks, 4096));
}

}  // namespace

// Staging of sparrow_ring_gather_static: the slots of one gather, copied from
// the host. Each GPU the library runs on holds one copy of the array until
// the process ends; every call on that GPU shares it. In host code the name
// stands for no device address: its address on a device comes from
// hipGetSymbolAddress with that device current (gather_scratch below).
constexpr int32_t kGatherStaticMax = SPARROW_GATHER_STATIC_MAX;
static __device__ __align__(256) int32_t scratch[kGatherStaticMax];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t* g_scratch[kMaxDevices] = {};

// The staging array's address on `device`, looked up once per device with
// that device current (the caller's current device is restored).
int gather_scratch(int device, int32_t** out) {
  if (device < 0 || device >= kMaxDevices) return fail(SPARROW_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != device) HIP_TRY(hipSetDevice(device));
    void* ptr = nullptr;
    const hipError_t err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) HIP_TRY(hipSetDevice(cur));
    if (err != hipSuccess || !ptr)
      return fail(SPARROW_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(err));
    g_scratch[device] = (int32_t*)ptr;
  }
  *out = g_scratch[device];
  return SPARROW_OK;
}
}  // namespace

struct sparrow_ring {
  RingDev dev{};
  void* block = nullptr;
  int32_t* d_slots = nullptr;  // staging for sparrow_ring_gather
  int32_t d_slots_cap = 0;
  int device = 0;                   // the device holding the ring
  int32_t* gather_static = nullptr;  // this device's staging array (sparrow_ring_gather_static)
  int64_t head = 0, size = 0;
  uint32_t key0 = 0, key1 = 0;
  hipStream_t stream = nullptr;
};

int sparrow_ring_create(int32_t capacity, int32_t n_rays, uint64_t seed, void* hip_stream,
                        sparrow_ring** out) {
  if (!out) return fail(SPARROW_EINVAL, "NULL argument");
  *out = nullptr;
  if (capacity < 1 || capacity > (1 << 26)) return fail(SPARROW_EINVAL, "capacity must be in [1, 2^26]");
  if (n_rays < 1 || n_rays > SPARROW_MAX_RAYS) return fail(SPARROW_EINVAL, "n_rays out of range");
  auto* R = new sparrow_ring();
  R->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&R->device) != hipSuccess) {
    delete R;
    return fail(SPARROW_EHIP, "hipGetDevice failed");
  }
  if (const int rc = gather_scratch(R->device, &R->gather_static)) {
    delete R;
    return rc;
  }
  R->key0 = (uint32_t)seed;
  R->key1 = (uint32_t)(seed >> 32);
  const size_t cap = (size_t)capacity;
  auto align = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t b_r = align(cap * n_rays), b_c = align(cap * kScalars * 2), b_a = align(cap),
               b_w = align(cap * 4), b_d = align((cap + 31) / 32 * 4);
  const size_t bytes = 2 * b_r + 2 * b_c + b_a + b_w + b_d;
  if (hipMalloc(&R->block, bytes) != hipSuccess) {
    delete R;
    return fail(SPARROW_ENOMEM, "hipMalloc of the ring failed");
  }
  char* p = (char*)R->block;
  R->dev.rs = (uint8_t*)p;
  p += b_r;
  R->dev.rsn = (uint8_t*)p;
  p += b_r;
  R->dev.cs = (uint16_t*)p;
  p += b_c;
  R->dev.csn = (uint16_t*)p;
  p += b_c;
  R->dev.act = (int8_t*)p;
  p += b_a;
  R->dev.rew = (float*)p;
  p += b_w;
  R->dev.done = (uint32_t*)p;
  R->dev.cap = capacity;
  R->dev.nr = n_rays;
  if (hipMemsetAsync(R->block, 0, bytes, R->stream) != hipSuccess ||
      hipStreamSynchronize(R->stream) != hipSuccess) {
    (void)hipFree(R->block);
    delete R;
    return fail(SPARROW_EHIP, "clearing the ring failed");
  }
  *out = R;
  return SPARROW_OK;
}

int sparrow_ring_push(sparrow_ring* R, int32_t n, const float* s, const int32_t* a, const float* r,
                      const float* s_next, const float* s_final, const uint8_t* done) {
  if (!R) return fail(SPARROW_EINVAL, "NULL argument");
  if (n < 0 || n > R->dev.cap) return fail(SPARROW_EINVAL, "push size must be in [0, capacity]");
  if (n == 0) return SPARROW_OK;
  if (!s || !a || !r || !s_next || !done) return fail(SPARROW_EINVAL, "NULL argument");
  const int64_t rows_per_block = kRingThreads / 64;
  hipLaunchKernelGGL(k_ring_push, dim3(grid_for(n * (int64_t)kRingThreads / rows_per_block)),
                     dim3(kRingThreads), 0, R->stream, R->dev, R->head, n, s, a, r, s_next, s_final,
                     done);
  HIP_TRY(hipGetLastError());
  R->head = (R->head + n) % R->dev.cap;
  R->size = std::min<int64_t>(R->size + n, R->dev.cap);
  return SPARROW_OK;
}

static int ring_read(sparrow_ring* R, int32_t B, uint32_t draw, const int32_t* d_slots, float* s,
                     int32_t* a, float* r, float* s_next, uint8_t* done, int32_t* idx) {
  const int64_t work = (int64_t)B * (R->dev.nr + kScalars);
  hipLaunchKernelGGL(k_ring_read, dim3(grid_for(work)), dim3(kRingThreads), 0, R->stream, R->dev,
                     (uint32_t)R->size, B, draw, R->key0, R->key1, d_slots, s, a, r, s_next, done,
                     idx);
  HIP_TRY(hipGetLastError());
  return SPARROW_OK;
}

int sparrow_ring_sample(sparrow_ring* R, int32_t B, uint32_t draw, float* s, int32_t* a, float* r,
                        float* s_next, uint8_t* done, int32_t* idx) {
  if (!R) return fail(SPARROW_EINVAL, "NULL argument");
  if (B < 0 || (int64_t)B * (R->dev.nr + kScalars) > INT32_MAX)
    return fail(SPARROW_EINVAL, "bad mini-batch size");
  if (R->size == 0) return fail(SPARROW_EINVAL, "the ring is empty");
  if (B == 0) return SPARROW_OK;
  return ring_read(R, B, draw, nullptr, s, a, r, s_next, done, idx);
}

int sparrow_ring_gather(sparrow_ring* R, int32_t n, const int32_t* slots_host, float* s, int32_t* a,
                        float* r, float* s_next, uint8_t* done) {
  if (!R || (n > 0 && !slots_host)) return fail(SPARROW_EINVAL, "NULL argument");
  if (n < 0 || (int64_t)n * (R->dev.nr + kScalars) > INT32_MAX)
    return fail(SPARROW_EINVAL, "bad gather size");
  for (int32_t b = 0; b < n; ++b)
    if (slots_host[b] < 0 || slots_host[b] >= R->size)
      return fail(SPARROW_EINVAL, "slot outside the stored range");
  if (n == 0) return SPARROW_OK;
  if (n > R->d_slots_cap) {
    if (R->d_slots) HIP_TRY(hipFree(R->d_slots));
    R->d_slots = nullptr;
    R->d_slots_cap = 0;
    if (hipMalloc((void**)&R->d_slots, sizeof(int32_t) * (size_t)n) != hipSuccess)
      return fail(SPARROW_ENOMEM, "hipMalloc failed");
    R->d_slots_cap = n;
  }
  // the previous gather may still read the staging buffer: order the copy
  // after it on the ring's stream, and wait for the copy before returning
  HIP_TRY(hipMemcpyAsync(R->d_slots, slots_host, sizeof(int32_t) * (size_t)n,
                         hipMemcpyHostToDevice, R->stream));
  const int rc = ring_read(R, n, 0u, R->d_slots, s, a, r, s_next, done, nullptr);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(R->stream));
  return SPARROW_OK;
}

int sparrow_ring_gather_static(sparrow_ring* R, int32_t n, const int32_t* slots_host, float* s,
                               int32_t* a, float* r, float* s_next, uint8_t* done) {
  if (!R || (n > 0 && !slots_host)) return fail(SPARROW_EINVAL, "NULL argument");
  if (n < 0 || n > kGatherStaticMax)
    return fail(SPARROW_EINVAL, "gather size must be in [0, SPARROW_GATHER_STATIC_MAX]");
  for (int32_t b = 0; b < n; ++b)
    if (slots_host[b] < 0 || slots_host[b] >= R->size)
      return fail(SPARROW_EINVAL, "slot outside the stored range");
  if (n == 0) return SPARROW_OK;
  // staged in this device's static array (looked up at create): no allocation
  HIP_TRY(hipMemcpyAsync(R->gather_static, slots_host, sizeof(int32_t) * (size_t)n,
                         hipMemcpyHostToDevice, R->stream));
  const int rc = ring_read(R, n, 0u, R->gather_static, s, a, r, s_next, done, nullptr);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(R->stream));
  return SPARROW_OK;
}

int64_t sparrow_ring_size(const sparrow_ring* R) { return R ? R->size : -1; }
int64_t sparrow_ring_head(const sparrow_ring* R) { return R ? R->head : -1; }

int sparrow_ring_status(sparrow_ring* R) {
  if (!R) return fail(SPARROW_EINVAL, "NULL argument");
  HIP_TRY(hipStreamSynchronize(R->stream));
  return SPARROW_OK;
}

void sparrow_ring_destroy(sparrow_ring* R) {
  if (!R) return;
  (void)hipStreamSynchronize(R->stream);
  if (R->d_slots) (void)hipFree(R->d_slots);
  if (R->block) (void)hipFree(R->block);
  delete R;
}

int sp::ring_view(const sparrow_ring* R, RingDev* view, int64_t* head) {
  if (!R || !view || !head) return fail(SPARROW_EINVAL, "NULL argument");
  *view = R->dev;
  *head = R->head;
  return SPARROW_OK;
}

int sp::ring_clear_done(const RingDev& R, int64_t head, int64_t n, hipStream_t stream) {
  if (n <= 0) return SPARROW_OK;
  const int64_t words = n / 32 + 2;
  hipLaunchKernelGGL(k_ring_clear_done, dim3(grid_for(words)), dim3(kRingThreads), 0, stream, R,
                     head, n);
  HIP_TRY(hipGetLastError());
  return SPARROW_OK;
}

void sp::ring_advance(sparrow_ring* R, int64_t n) {
  if (!R || n <= 0) return;
  R->head = (R->head + n) % R->dev.cap;
  R->size = std::min<int64_t>(R->size + n, R->dev.cap);
}
