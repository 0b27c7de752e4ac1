// Per-source statistics of a k x n level array (the output of the k-source BFS):
// reached count, sum of finite levels, eccentricity (largest finite level), the
// smallest vertex at that level and closeness (reached - 1) / sum.  Section 2
// names centrality and diameter computations among the multi-source problems the
// stacked frontiers serve; these are the reductions they need.
//
// Streaming reductions over 4kn bytes, bound by HBM: a (blocks x k) grid, each
// thread strides its row with coalesced 4-byte loads, wavefronts reduce with
// lane shuffles and one lane per wavefront adds into the row's counters.  The
// farthest vertex needs the row's maximum first, so it is a second pass.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.hpp"
#include "kernels.hpp"

namespace blest {
namespace {

constexpr uint32_t kStatBlock = 256;

__global__ void stats_init(uint32_t k, unsigned long long* reached, unsigned long long* total, int32_t* ecc,
                           uint32_t* far) {
  for (uint32_t j = threadIdx.x; j < k; j += blockDim.x) {
    reached[j] = 0;
    total[j] = 0;
    ecc[j] = -1;
    far[j] = 0xFFFFFFFFu;
  }
}

__global__ __launch_bounds__(kStatBlock) void stats_reduce(const int32_t* levels, uint32_t n,
                                                           unsigned long long* reached, unsigned long long* total,
                                                           int32_t* ecc) {
  const uint32_t j = blockIdx.y;
  const int32_t* row = levels + (uint64_t)j * n;
  uint32_t cnt = 0;
  unsigned long long sum = 0;
  int32_t mx = -1;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const int32_t l = row[v];
    if (l >= 0) {
      ++cnt;
      sum += (uint32_t)l;
      mx = max(mx, l);
    }
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    cnt += __shfl_xor(cnt, off);
    sum += __shfl_xor(sum, off);
    mx = max(mx, __shfl_xor(mx, off));
  }
  if (lane_id() == 0 && cnt) {
    atomicAdd(reached + j, (unsigned long long)cnt);
    atomicAdd(total + j, sum);
    atomicMax(ecc + j, mx);
  }
}

__global__ __launch_bounds__(kStatBlock) void stats_far(const int32_t* levels, uint32_t n, const int32_t* ecc,
                                                        uint32_t* far) {
  const uint32_t j = blockIdx.y;
  const int32_t e = ecc[j];
  if (e < 0) return;  // empty row (n = 0 or no source)
  const int32_t* row = levels + (uint64_t)j * n;
  uint32_t best = 0xFFFFFFFFu;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n && best == 0xFFFFFFFFu;
       v += gridDim.x * blockDim.x)
    if (row[v] == e) best = v;
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) best = min(best, (uint32_t)__shfl_xor(best, off));
  if (lane_id() == 0 && best != 0xFFFFFFFFu) atomicMin(far + j, best);
}

__global__ void stats_close(uint32_t k, const unsigned long long* reached, const unsigned long long* total,
                            double* closeness) {
  for (uint32_t j = threadIdx.x; j < k; j += blockDim.x)
    closeness[j] = total[j] ? (double)(reached[j] - 1) / (double)total[j] : 0.0;
}

}  // namespace

hipError_t launch_level_stats(const int32_t* levels, uint32_t k, uint32_t n, unsigned long long* reached,
                              unsigned long long* total, int32_t* ecc, uint32_t* far, double* closeness,
                              uint32_t num_cus, hipStream_t stream) {
  stats_init<<<1, 64, 0, stream>>>(k, reached, total, ecc, far);
  if (n) {
    // about eight workgroups per CU in all, split over the k rows
    const uint64_t want = std::max<uint64_t>(1, 8ull * num_cus / k);
    const uint32_t bx = (uint32_t)std::min<uint64_t>(want, (n + kStatBlock - 1) / kStatBlock);
    stats_reduce<<<dim3(bx, k), kStatBlock, 0, stream>>>(levels, n, reached, total, ecc);
    stats_far<<<dim3(bx, k), kStatBlock, 0, stream>>>(levels, n, ecc, far);
  }
  stats_close<<<1, 64, 0, stream>>>(k, reached, total, closeness);
  return hipGetLastError();
}

}  // namespace blest
