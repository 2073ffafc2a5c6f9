// sparrow_peaks.hip -- peak-rate probes of the device, for the roofline of the
// step kernels. They measure the hardware, not the method: LDS read
// bandwidth (16-byte and 4-byte lane reads, bank-conflict free), HBM
// streaming (read + write of a large buffer) and dense BF16 MFMA issue.
//
// Each probe is a short, fixed-size kernel with in-bounds addressing and a
// bounded loop; every lane writes one word of its result so that no load or
// multiply can be dropped by the compiler.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/sparrow.h"
#include "sparrow_host.h"

namespace {

constexpr int kLdsWords = 16384;  // 64 KiB per workgroup: two workgroups per CU

// Lane l of a wave reads 16 bytes at 16 (l + 64 i) mod 64 KiB: the 64 lanes
// cover 1 KiB of consecutive words, so every bank serves the same number of
// lanes (no conflicts beyond the instruction's own width).
__global__ void __launch_bounds__(1024) k_peak_lds128(int iters, uint32_t* __restrict__ out) {
  __shared__ uint4 buf[kLdsWords / 4];
  for (int k = threadIdx.x; k < kLdsWords / 4; k += blockDim.x)
    buf[k] = make_uint4(k, 3u * k, 5u * k, 7u * k);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t a0 = 0, a1 = 0;
  int idx = lane + 64 * wave;
#pragma unroll 8
  for (int i = 0; i < iters; ++i) {
    const uint4 v = buf[idx & (kLdsWords / 4 - 1)];
    a0 = a0 + v.x + v.y;  // one three-input add per two words
    a1 = a1 + v.z + v.w;
    idx += 64;
  }
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = a0 ^ a1;
}

// Lane l reads 4 bytes at word l + 64 i: 64 consecutive words, each bank
// twice per instruction (64 lanes over 32 or 64 banks).
__global__ void __launch_bounds__(1024) k_peak_lds32(int iters, uint32_t* __restrict__ out) {
  __shared__ uint32_t buf[kLdsWords];
  for (int k = threadIdx.x; k < kLdsWords; k += blockDim.x) buf[k] = 2654435761u * k;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t a0 = 0, a1 = 0;
  int idx = lane + 64 * wave;
#pragma unroll 8
  for (int i = 0; i < iters; i += 2) {
    a0 += buf[idx & (kLdsWords - 1)];
    a1 += buf[(idx + 64) & (kLdsWords - 1)];
    idx += 128;
  }
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = a0 ^ a1;
}

// Grid-stride copy of n 16-byte elements.
__global__ void __launch_bounds__(256) k_peak_copy(const uint4* __restrict__ src,
                                                   uint4* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
    dst[k] = src[k];
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Eight independent accumulation chains of v_mfma_f32_16x16x32_bf16 per wave
// (16 x 16 x 32 x 2 = 16,384 FLOP each), operands held in registers.
__global__ void __launch_bounds__(256) k_peak_mfma(int iters, float* __restrict__ out) {
  bf16x8 a, b;
  for (int k = 0; k < 8; ++k) {
    a[k] = (__bf16)(0.001f * (float)((threadIdx.x + k) & 15));
    b[k] = (__bf16)(0.002f * (float)((threadIdx.x * 3 + k) & 15));
  }
  f32x4 acc[8];
  for (int c = 0; c < 8; ++c) acc[c] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.0f;
  for (int c = 0; c < 8; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

extern "C" int sparrow_peak(int32_t kind, int64_t size, int32_t iters, void* hip_stream,
                            double* rate, double* seconds) {
  if (!rate || iters < 1 || iters > (1 << 20) || kind < 0 || kind > 3)
    return sp::fail(SPARROW_EINVAL, "sparrow_peak: kind in 0..3, iters in 1..2^20, rate non-NULL");
  hipStream_t st = (hipStream_t)hip_stream;
  int dev = 0, cus = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  void* a = nullptr;
  void* b = nullptr;
  int rc = SPARROW_OK;
  double work = 0.0;
  float ms = 0.0f;
  // one untimed launch, then `reps` timed ones
  const int reps = kind == 2 ? iters : 3;
  auto run = [&](bool timed) -> hipError_t {
    const int n = timed ? reps : 1;
    for (int r = 0; r < n; ++r) {
      if (kind == 0) {
        const int blocks = 2 * cus * 16;
        hipLaunchKernelGGL(k_peak_lds128, dim3(blocks), dim3(1024), 0, st, iters, (uint32_t*)a);
        if (timed) work += (double)blocks * 1024 * iters * 16;
      } else if (kind == 1) {
        const int blocks = 2 * cus * 16;
        hipLaunchKernelGGL(k_peak_lds32, dim3(blocks), dim3(1024), 0, st, iters & ~1,
                           (uint32_t*)a);
        if (timed) work += (double)blocks * 1024 * (iters & ~1) * 4;
      } else if (kind == 2) {
        const int64_t n16 = size / 16;
        hipLaunchKernelGGL(k_peak_copy, dim3(cus * 32), dim3(256), 0, st, (const uint4*)a,
                           (uint4*)b, n16);
        if (timed) work += 2.0 * (double)n16 * 16;
      } else {
        const int blocks = cus * 16;
        hipLaunchKernelGGL(k_peak_mfma, dim3(blocks), dim3(256), 0, st, iters, (float*)a);
        if (timed) work += (double)blocks * 4 * iters * 8 * 16384.0;
      }
      const hipError_t err = hipGetLastError();
      if (err != hipSuccess) return err;
    }
    return hipSuccess;
  };
  do {
    if (kind == 2) {
      if (size < (1 << 20) || size > ((int64_t)16 << 30) || size % 16) {
        rc = sp::fail(SPARROW_EINVAL, "sparrow_peak: HBM size in [1 MiB, 16 GiB], a multiple of 16");
        break;
      }
      if (hipMalloc(&a, (size_t)size) != hipSuccess || hipMalloc(&b, (size_t)size) != hipSuccess) {
        rc = sp::fail(SPARROW_ENOMEM, "sparrow_peak: device buffers");
        break;
      }
      if (hipMemsetAsync(a, 1, (size_t)size, st) != hipSuccess) {
        rc = sp::fail(SPARROW_EHIP, "sparrow_peak: memset");
        break;
      }
    } else {
      const size_t words = (size_t)2 * cus * 16 * 1024;
      if (hipMalloc(&a, words * 4) != hipSuccess) {
        rc = sp::fail(SPARROW_ENOMEM, "sparrow_peak: result buffer");
        break;
      }
    }
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      rc = sp::fail(SPARROW_EHIP, "sparrow_peak: events");
      break;
    }
    hipError_t err = run(false);
    if (err == hipSuccess) err = hipEventRecord(e0, st);
    if (err == hipSuccess) err = run(true);
    if (err == hipSuccess) err = hipEventRecord(e1, st);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err != hipSuccess) {
      rc = sp::fail(SPARROW_EHIP, std::string("sparrow_peak: ") + hipGetErrorString(err));
      break;
    }
    *rate = work / ((double)ms * 1e-3);
    if (seconds) *seconds = (double)ms * 1e-3;
  } while (false);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  return rc;
}
