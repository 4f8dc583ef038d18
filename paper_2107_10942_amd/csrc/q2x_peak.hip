// q2x_peak.hip -- peak microbenchmarks of the vector ALU and of HBM on the
// running GPU (measurement aid: the denominators of the roofline fractions).
//   FMA64 / FMA32: every lane runs 8 independent FMA chains (no packed FP32:
//   the library is built without packed FP32 instructions), enough waves to
//   fill every SIMD several times; FLOPs = lanes x iterations x 8 x 2.
//   COPY: a 16-byte-per-lane copy of a buffer half to the other half; bytes =
//   read + written.
// Timed with HIP events on the caller's stream.
#include "q2x_internal.hpp"

namespace q2x {
namespace {

constexpr int kPeakIters = 2048;
constexpr int kChains = 8;

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__global__ __launch_bounds__(256) void peak_fma(T* out, T seed) {
  T a[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) a[k] = seed + (T)(threadIdx.x + k);
  const T x = seed * (T)0.999, y = (T)1e-3;
  for (int i = 0; i < kPeakIters; ++i) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = fma_t(a[k], x, y);
  }
  T s = 0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += a[k];
  if (s == (T)-1.2345) out[blockIdx.x] = s;  // keeps the chains alive; never true
}

__global__ __launch_bounds__(256) void peak_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                                 int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace
}  // namespace q2x

using namespace q2x;

extern "C" q2x_status q2x_peak_measure(int which, void* buffer, size_t buffer_bytes, int reps, void* stream,
                                       double* value, double* ms_per_rep) {
  if (!value || reps <= 0 || which < 0 || which > 2) return Q2X_ERR_ARG;
  if (!buffer || ((uintptr_t)buffer % 256) != 0) return Q2X_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  const int blocks = 256 * 4 * 16;  // 16 waves of 256 threads per SIMD of 256 CUs
  int64_t n4 = 0;
  if (which == 2) {
    n4 = (int64_t)(buffer_bytes / 2 / sizeof(float4));
    if (n4 <= 0) return Q2X_ERR_ARG;
  } else if (buffer_bytes < (size_t)blocks * sizeof(double)) {
    return Q2X_ERR_ARG;
  }
  auto launch = [&]() {
    if (which == 0) hipLaunchKernelGGL(peak_fma<double>, dim3(blocks), dim3(256), 0, s, (double*)buffer, 1.0);
    else if (which == 1) hipLaunchKernelGGL(peak_fma<float>, dim3(blocks), dim3(256), 0, s, (float*)buffer, 1.0f);
    else
      hipLaunchKernelGGL(peak_copy, dim3(8192), dim3(256), 0, s, (const float4*)buffer, (float4*)buffer + n4, n4);
  };
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return Q2X_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return Q2X_ERR_HIP;
  }
  launch();  // warm-up
  (void)hipEventRecord(e0, s);
  for (int r = 0; r < reps; ++r) launch();
  (void)hipEventRecord(e1, s);
  float ms = 0.f;
  const bool ok = hipGetLastError() == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                  hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!ok || ms <= 0.f) return Q2X_ERR_HIP;
  const double t = (double)ms / reps * 1e-3;  // seconds per launch
  if (which == 2) *value = 2.0 * (double)n4 * sizeof(float4) / t / 1e9;  // GB/s
  else *value = (double)blocks * 256.0 * kPeakIters * kChains * 2.0 / t / 1e12;  // TFLOP/s
  if (ms_per_rep) *ms_per_rep = (double)ms / reps;
  return Q2X_OK;
}
