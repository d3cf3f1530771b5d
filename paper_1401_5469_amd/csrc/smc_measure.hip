// smc_measure.hip -- measurement kernels of libsmc: the device's throughput
// of the FP64 atomic adds the estimator tallies issue, the peak the transport
// pass's atomic rate is compared with.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/smc.h"
#include "smc_internal.h"

namespace smc {
namespace {

// Each lane adds 1.0 to one double of the table n_rounds times, at a new
// pseudo-random place each round.  kScattered = false: a wavefront's lanes
// take 64 consecutive doubles (as a J_blue window leaves a wavefront:
// consecutive lines of one shell row); true: every lane its own place (as the
// lane-per-packet tallies land).
template <bool kScattered>
__global__ __launch_bounds__(256) void atomic_rate_kernel(double* __restrict__ table,
                                                          uint64_t n_doubles, uint32_t n_rounds) {
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t wave = gid >> 6;
  const uint32_t lane = threadIdx.x & 63u;
  uint64_t h = (kScattered ? gid : wave) * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  for (uint32_t r = 0; r < n_rounds; ++r) {
    h ^= h >> 29;
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 32;
    const uint64_t at = kScattered ? h % n_doubles : (h % (n_doubles / 64u)) * 64u + lane;
    unsafeAtomicAdd(&table[at], 1.0);
  }
}

}  // namespace

hipError_t launch_atomic_rate(double* table, uint64_t n_doubles, uint32_t n_rounds, int scattered,
                              int n_cu, hipStream_t s) {
  if (scattered)
    hipLaunchKernelGGL(atomic_rate_kernel<true>, dim3((unsigned)(8 * n_cu)), dim3(256), 0, s,
                       table, n_doubles, n_rounds);
  else
    hipLaunchKernelGGL(atomic_rate_kernel<false>, dim3((unsigned)(8 * n_cu)), dim3(256), 0, s,
                       table, n_doubles, n_rounds);
  return hipGetLastError();
}

}  // namespace smc
