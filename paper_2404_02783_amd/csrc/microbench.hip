// Measurement helper (not part of the method): the rate of the global float atomics the
// deposits flush their LDS windows with, on the same access pattern -- consecutive
// lanes add to consecutive, distinct cells, no two atomics of a pass on one address.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pm_common.h"
#include "pm_plan.h"

namespace pm {
namespace {

constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock) k_atomic_rate(float* __restrict__ buf, int64_t n, int passes) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int r = 0; r < passes; ++r)
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
      unsafeAtomicAdd(buf + i, 1.0f);
}

}  // namespace
}  // namespace pm

int pm_microbench_atomics(void* buf, int64_t n, int passes, void* stream) {
  using pm::hip_check;
  using pm::kBlock;
  using pm::set_error;
  using pm::k_atomic_rate;
  if (!buf || n <= 0 || passes <= 0) return set_error(PM_ERR_ARG, "pm_microbench_atomics: bad arguments");
  const unsigned g = (unsigned)std::min<int64_t>((n + kBlock - 1) / kBlock, 1 << 20);
  hipLaunchKernelGGL(k_atomic_rate, dim3(g), dim3(kBlock), 0, static_cast<hipStream_t>(stream),
                     static_cast<float*>(buf), n, passes);
  return hip_check(hipGetLastError(), "pm_microbench_atomics");
}
