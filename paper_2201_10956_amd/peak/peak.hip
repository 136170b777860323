// Peak-rate microbenchmarks of the gfx950 pipes the count kernels run on:
// register-only chains of matrix-core products (FP4 and int8 operands, the
// instructions the matrix-core count kernels issue) and of the vector-ALU
// AND + popcount pair the popcount kernel issues.  Each wave keeps several
// independent accumulators so that dependent latency never limits the
// issue rate; nothing is read from memory inside the timed loops, and one
// value per lane is written at the end so the loops are not removed.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kChains = 4;  // independent accumulators per wave

__global__ void __launch_bounds__(256) mfma_fp4_kernel(int64_t iters, float *out) {
  const int lane = threadIdx.x & 63;
  // arbitrary FP4 bit patterns: the rate does not depend on the values
  v4i a = {lane * 0x11111111, lane ^ 0x2a2a2a2a, 0x22222222, lane};
  v4i b = {0x12121212, lane * 3, lane ^ 0x0f0f0f0f, 0x21212121};
  const v8i a8 = {a.x, a.y, a.z, a.w, 0, 0, 0, 0};
  const v8i b8 = {b.x, b.y, b.z, b.w, 0, 0, 0, 0};
  v16f c[kChains];
#pragma unroll
  for (int x = 0; x < kChains; ++x)
#pragma unroll
    for (int v = 0; v < 16; ++v) c[x][v] = 0.f;
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int x = 0; x < kChains; ++x)
      c[x] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a8, b8, c[x], 4, 4, 0, 127, 0, 127);
  }
  float s = 0.f;
#pragma unroll
  for (int x = 0; x < kChains; ++x)
#pragma unroll
    for (int v = 0; v < 16; ++v) s += c[x][v];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) mfma_i8_kernel(int64_t iters, float *out) {
  const int lane = threadIdx.x & 63;
  const v4i a = {lane, lane * 7, 0x01010101, lane ^ 0x55};
  const v4i b = {0x01000100, lane * 5, lane, 0x7f};
  v16i c[kChains];
#pragma unroll
  for (int x = 0; x < kChains; ++x)
#pragma unroll
    for (int v = 0; v < 16; ++v) c[x][v] = 0;
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int x = 0; x < kChains; ++x)
      c[x] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c[x], 0, 0, 0);
  }
  int s = 0;
#pragma unroll
  for (int x = 0; x < kChains; ++x)
#pragma unroll
    for (int v = 0; v < 16; ++v) s += c[x][v];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = (float)s;
}

// acc + popcount(x) as one v_bcnt_u32_b32
__device__ __forceinline__ uint32_t bcnt_acc(uint32_t x, uint32_t acc) {
  uint32_t r;
  asm volatile("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
  return r;
}

__device__ __forceinline__ uint32_t and_op(uint32_t x, uint32_t y) {
  uint32_t r;
  asm volatile("v_and_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(y));
  return r;
}

// 8 independent AND + v_bcnt pairs per iteration: 16 INT32 lane-ops per lane
// (both opaque to the compiler, so none is hoisted or merged).
__global__ void __launch_bounds__(256) valu_popc_kernel(int64_t iters, float *out) {
  const uint32_t lane = threadIdx.x;
  uint32_t x[8], acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    x[q] = lane * 0x9e3779b9u + q;
    acc[q] = 0u;
  }
  const uint32_t m = lane | 0x80000001u;
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = bcnt_acc(and_op(x[q], m), acc[q]);
  }
  uint32_t s = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) s += acc[q];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = (float)s;
}

}  // namespace

// kind 0: FP4 32x32x64 products (2 x 32 x 32 x 64 FLOP each), 1: int8
// 32x32x32 products (2 x 32 x 32 x 32 OP), 2: AND + v_bcnt (16 lane-ops per
// lane and iteration).  Launches `blocks` workgroups of 256 threads
// (out_dev: blocks x 256 floats), times `reps` launches with HIP events on
// stream 0 after one untimed launch, and returns the average ms per launch
// and the operations of one launch.  0 on success, -1 on bad arguments,
// -6 when a HIP call fails.
extern "C" int epi3_peak_run(int32_t kind, int64_t iters, int32_t blocks, int32_t reps,
                             float *out_dev, double *ms_out, double *ops_out) {
  if (kind < 0 || kind > 2 || iters <= 0 || blocks <= 0 || reps <= 0 || !out_dev || !ms_out ||
      !ops_out)
    return -1;
  auto launch = [&]() {
    if (kind == 0)
      hipLaunchKernelGGL(mfma_fp4_kernel, dim3(blocks), dim3(256), 0, 0, iters, out_dev);
    else if (kind == 1)
      hipLaunchKernelGGL(mfma_i8_kernel, dim3(blocks), dim3(256), 0, 0, iters, out_dev);
    else
      hipLaunchKernelGGL(valu_popc_kernel, dim3(blocks), dim3(256), 0, 0, iters, out_dev);
    return hipGetLastError();
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (launch() != hipSuccess) return -6;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -6;
  int rc = 0;
  if (hipEventRecord(e0, 0) != hipSuccess) rc = -6;
  for (int r = 0; r < reps && rc == 0; ++r)
    if (launch() != hipSuccess) rc = -6;
  float ms = 0.f;
  if (rc == 0 && (hipEventRecord(e1, 0) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                  hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    rc = -6;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != 0) return rc;
  const double waves = (double)blocks * 4.0;
  const double per_wave = kind == 0   ? 2.0 * 32 * 32 * 64 * kChains
                          : kind == 1 ? 2.0 * 32 * 32 * 32 * kChains
                                      : 16.0 * 64;
  *ms_out = ms / reps;
  *ops_out = waves * per_wave * (double)iters;
  return 0;
}
