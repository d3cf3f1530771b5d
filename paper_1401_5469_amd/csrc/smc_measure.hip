// smc_measure.hip -- measurement kernels of libsmc: the device's throughput
// of the FP64 atomic adds the estimator tallies issue, the peak the transport
// pass's atomic rate is compared with.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/smc.h"
#include "smc_internal.h"

namespace smc {
namespace {

// Each wavefront adds 1.0 to 64 consecutive doubles of the table (one per
// lane, as a J_blue window leaves a wavefront: consecutive lines of one
// shell row), n_rounds times, at a new pseudo-random window each round.
__global__ __launch_bounds__(256) void atomic_rate_kernel(double* __restrict__ table,
                                                          uint64_t n_windows, uint32_t n_rounds) {
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint32_t lane = threadIdx.x & 63u;
  uint64_t h = wave * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  for (uint32_t r = 0; r < n_rounds; ++r) {
    h ^= h >> 29;
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 32;
    const uint64_t w = h % n_windows;
    unsafeAtomicAdd(&table[w * 64u + lane], 1.0);
  }
}

}  // namespace

hipError_t launch_atomic_rate(double* table, uint64_t n_doubles, uint32_t n_rounds, int n_cu,
                              hipStream_t s) {
  hipLaunchKernelGGL(atomic_rate_kernel, dim3((unsigned)(8 * n_cu)), dim3(256), 0, s, table,
                     n_doubles / 64, n_rounds);
  return hipGetLastError();
}

}  // namespace smc
