// Measured machine peaks for the roofline: int8 MFMA throughput from registers
// (no memory traffic) and streaming HBM copy bandwidth.
#include <cstdio>

#include "context.h"

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

// Each wave keeps 8 independent 16x16x64 int8 accumulators busy for `iters` rounds.
__global__ void __launch_bounds__(256) mfma_peak_kernel(int iters, int* sink) {
  v4i a = {(int)threadIdx.x, 1, 2, 3}, b = {3, 2, 1, (int)blockIdx.x};
  v4i acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = v4i{i, 0, 0, 0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, acc[i], 0, 0, 0);
  }
  int s = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += acc[i].x + acc[i].y + acc[i].z + acc[i].w;
  if (s == 0x7fffffff) sink[0] = s;   // keeps the work alive; practically never stores
}

typedef int v16i __attribute__((ext_vector_type(16)));

// Same with v_mfma_i32_32x32x32_i8 (4 independent 32x32 accumulators per wave).
__global__ void __launch_bounds__(256) mfma32_peak_kernel(int iters, int* sink) {
  v4i a = {(int)threadIdx.x, 1, 2, 3}, b = {3, 2, 1, (int)blockIdx.x};
  v16i acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = v16i{};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[i], 0, 0, 0);
  }
  int s = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) s += acc[i][0] + acc[i][15];
  if (s == 0x7fffffff) sink[0] = s;
}

__global__ void __launch_bounds__(256) copy_kernel(const v4i* __restrict__ src, v4i* __restrict__ dst, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

}  // namespace

extern "C" {

cross_status cross_measure_peak(cross_ctx ctx, int which, double* out) {
  if (!ctx || !out || which < 0 || which > 2) return CROSS_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return cross::fail(ctx, CROSS_EDEVICE, "hipSetDevice failed");
  int ncu = 0;
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device);
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  cross_status st = CROSS_OK;
  if (which == 2) {
    int* sink = nullptr;
    if (hipMalloc(&sink, 64) != hipSuccess) return cross::fail(ctx, CROSS_ENOMEM, "peak sink");
    const int iters = 2048, blocks = ncu * 8;
    hipLaunchKernelGGL(mfma32_peak_kernel, dim3(blocks), dim3(256), 0, nullptr, 64, sink);
    (void)hipEventRecord(e0, nullptr);
    hipLaunchKernelGGL(mfma32_peak_kernel, dim3(blocks), dim3(256), 0, nullptr, iters, sink);
    (void)hipEventRecord(e1, nullptr);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double ops = 2.0 * 32 * 32 * 32 * 4 * (double)iters * blocks * 4;
    *out = ops / (ms * 1e-3) / 1e12;
    (void)hipFree(sink);
  } else if (which == 0) {
    int* sink = nullptr;
    if (hipMalloc(&sink, 64) != hipSuccess) return cross::fail(ctx, CROSS_ENOMEM, "peak sink");
    const int iters = 4096, blocks = ncu * 8;            // 8 waves per SIMD
    hipLaunchKernelGGL(mfma_peak_kernel, dim3(blocks), dim3(256), 0, nullptr, 64, sink);
    (void)hipEventRecord(e0, nullptr);
    hipLaunchKernelGGL(mfma_peak_kernel, dim3(blocks), dim3(256), 0, nullptr, iters, sink);
    (void)hipEventRecord(e1, nullptr);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double ops = 2.0 * 16 * 16 * 64 * 8 * (double)iters * blocks * 4;   // 4 waves per block
    *out = ops / (ms * 1e-3) / 1e12;                                           // TOP/s
    (void)hipFree(sink);
  } else {
    const uint64_t bytes = 1ull << 30;
    void *s = nullptr, *d = nullptr;
    if (hipMalloc(&s, bytes) != hipSuccess || hipMalloc(&d, bytes) != hipSuccess) {
      (void)hipFree(s);
      return cross::fail(ctx, CROSS_ENOMEM, "peak copy buffers");
    }
    (void)hipMemset(s, 1, bytes);
    const uint64_t n = bytes / 16;
    hipLaunchKernelGGL(copy_kernel, dim3(ncu * 16), dim3(256), 0, nullptr, (const v4i*)s, (v4i*)d, n);
    (void)hipEventRecord(e0, nullptr);
    const int reps = 5;
    for (int r = 0; r < reps; ++r)
      hipLaunchKernelGGL(copy_kernel, dim3(ncu * 16), dim3(256), 0, nullptr, (const v4i*)s, (v4i*)d, n);
    (void)hipEventRecord(e1, nullptr);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    *out = 2.0 * bytes * reps / (ms * 1e-3) / 1e9;                             // GB/s read + written
    (void)hipFree(s);
    (void)hipFree(d);
  }
  if (hipGetLastError() != hipSuccess) st = cross::fail(ctx, CROSS_EDEVICE, "peak kernel failed");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

}  // extern "C"
