// Calibration of the kernel apply's roofline: the sustained rate of the
// 16x16x4 matrix-core instruction it issues (v_mfma_f64_16x16x4f64 in FP64,
// v_mfma_f32_16x16x4f32 in FP32), measured with independent accumulator
// chains and no memory traffic, so that the apply's measured rate can be
// read against what the matrix cores of this part sustain as well as
// against the published peak.  Each thread writes one value at the end.
#include <algorithm>
#include <stdexcept>
#include <type_traits>

#include "device_common.h"
#include "kernels.h"

namespace hm {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T, int NA>
__global__ void __launch_bounds__(256) mfma_rate_kernel(int iters, T *__restrict__ out) {
  typedef typename std::conditional<sizeof(T) == 8, d4, f4>::type acc_t;
  acc_t acc[NA];
#pragma unroll
  for (int t = 0; t < NA; ++t) acc[t] = (acc_t){0, 0, 0, 0};
  const T a = (T)1 + (T)threadIdx.x * (T)1e-7, b = (T)1 - (T)threadIdx.x * (T)1e-7;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int t = 0; t < NA; ++t) {
      if constexpr (sizeof(T) == 8)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
      else
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
    }
  }
  T s = 0;
#pragma unroll
  for (int t = 0; t < NA; ++t) s += acc[t][0] + acc[t][1] + acc[t][2] + acc[t][3];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

// TFLOP/s of one launch: `blocks` workgroups of 4 waves, NA chains each
template <typename T, int NA>
double time_rate(int blocks, int iters, T *out, hipStream_t s) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) throw std::runtime_error("hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    throw std::runtime_error("hipEventCreate failed");
  }
  mfma_rate_kernel<T, NA><<<blocks, 256, 0, s>>>(iters / 8, out);  // warm-up
  (void)hipEventRecord(e0, s);
  mfma_rate_kernel<T, NA><<<blocks, 256, 0, s>>>(iters, out);
  (void)hipEventRecord(e1, s);
  const hipError_t le = hipGetLastError();
  float ms = 0.f;
  const hipError_t se = hipEventSynchronize(e1);
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (le != hipSuccess || se != hipSuccess || !(ms > 0.f))
    throw std::runtime_error("matrix-core probe launch failed");
  const double flops = 2.0 * 16 * 16 * 4 * NA * (double)iters * (double)blocks * 4.0;
  return flops / ((double)ms * 1e-3) / 1e12;
}

}  // namespace

double measure_mfma_rate(bool f32, int cus, hipStream_t s) {
  const int per_cu[3] = {1, 2, 4};
  const int max_blocks = std::max(cus, 1) * 4;
  void *out = nullptr;
  if (hipMalloc(&out, (size_t)max_blocks * 256 * 8) != hipSuccess) {
    (void)hipGetLastError();
    throw std::runtime_error("device allocation failed");
  }
  double best = 0.0;
  try {
    for (int k = 0; k < 3; ++k) {
      const int blocks = std::max(cus, 1) * per_cu[k];
      const int iters = 4096 / per_cu[k];
      if (f32) {
        best = std::max(best, time_rate<float, 4>(blocks, iters, (float *)out, s));
        best = std::max(best, time_rate<float, 8>(blocks, iters, (float *)out, s));
      } else {
        best = std::max(best, time_rate<double, 4>(blocks, iters, (double *)out, s));
        best = std::max(best, time_rate<double, 8>(blocks, iters, (double *)out, s));
      }
    }
  } catch (...) {
    (void)hipFree(out);
    throw;
  }
  (void)hipFree(out);
  return best;
}

}  // namespace hm
