// Per-source statistics of a k x n level array (the output of the k-source BFS):
// reached count, sum of finite levels, eccentricity (largest finite level), the
// smallest vertex at that level and closeness (reached - 1) / sum.  Section 2
// names centrality and diameter computations among the multi-source problems the
// stacked frontiers serve; these are the reductions they need.
//
// One streaming pass over the 4kn bytes, bound by HBM: a (blocks x k) grid, each
// thread strides its row (16-byte loads when rows are 16-byte aligned) keeping
// its count, sum, largest level and the first (smallest) vertex at that level;
// wavefronts combine with lane shuffles and one lane per wavefront adds into the
// row's counters.  The (level, vertex) pair is packed as
// ((level + 1) << 32) | ~vertex so that one 64-bit atomic maximum keeps the
// largest level and, among equal levels, the smallest vertex; the key lives in
// the row's closeness slot until the last kernel unpacks it.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.hpp"
#include "kernels.hpp"

namespace blest {
namespace {

constexpr uint32_t kStatBlock = 256;

struct RowAcc {
  uint32_t cnt = 0;
  unsigned long long sum = 0;
  int32_t mx = -1;
  uint32_t vb = 0xFFFFFFFFu;

  __device__ __forceinline__ void add(int32_t l, uint32_t v) {
    if (l >= 0) {
      ++cnt;
      sum += (uint32_t)l;
      if (l > mx) {  // vertices arrive in increasing order per thread: keep the first
        mx = l;
        vb = v;
      }
    }
  }
};

__global__ void stats_init(uint32_t k, unsigned long long* reached, unsigned long long* total,
                           unsigned long long* key) {
  for (uint32_t j = threadIdx.x; j < k; j += blockDim.x) {
    reached[j] = 0;
    total[j] = 0;
    key[j] = 0;
  }
}

template <bool VEC>
__global__ __launch_bounds__(kStatBlock) void stats_reduce(const int32_t* levels, uint32_t n,
                                                           unsigned long long* reached, unsigned long long* total,
                                                           unsigned long long* key) {
  const uint32_t j = blockIdx.y;
  const int32_t* row = levels + (uint64_t)j * n;
  const uint32_t t0 = blockIdx.x * blockDim.x + threadIdx.x, step = gridDim.x * blockDim.x;
  RowAcc a;
  if (VEC) {
    const int4* r4 = reinterpret_cast<const int4*>(row);
    const uint32_t n4 = n / 4;
    uint32_t i = t0;
    for (; i + step < n4; i += 2 * step) {  // two loads in flight
      const int4 x = r4[i], y = r4[i + step];
      a.add(x.x, 4 * i), a.add(x.y, 4 * i + 1), a.add(x.z, 4 * i + 2), a.add(x.w, 4 * i + 3);
      const uint32_t b = 4 * (i + step);
      a.add(y.x, b), a.add(y.y, b + 1), a.add(y.z, b + 2), a.add(y.w, b + 3);
    }
    if (i < n4) {
      const int4 x = r4[i];
      a.add(x.x, 4 * i), a.add(x.y, 4 * i + 1), a.add(x.z, 4 * i + 2), a.add(x.w, 4 * i + 3);
    }
  } else {
    for (uint32_t v = t0; v < n; v += step) a.add(row[v], v);
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    a.cnt += __shfl_xor(a.cnt, off);
    a.sum += __shfl_xor(a.sum, off);
    const int32_t omx = __shfl_xor(a.mx, off);
    const uint32_t ovb = __shfl_xor(a.vb, off);
    if (omx > a.mx || (omx == a.mx && ovb < a.vb)) {
      a.mx = omx;
      a.vb = ovb;
    }
  }
  if (lane_id() == 0 && a.cnt) {
    atomicAdd(reached + j, (unsigned long long)a.cnt);
    atomicAdd(total + j, a.sum);
    atomicMax(key + j, ((unsigned long long)(uint32_t)(a.mx + 1) << 32) | (unsigned long long)(~a.vb));
  }
}

__global__ void stats_final(uint32_t k, const unsigned long long* reached, const unsigned long long* total,
                            int32_t* ecc, uint32_t* far, double* closeness) {
  unsigned long long* key = reinterpret_cast<unsigned long long*>(closeness);
  for (uint32_t j = threadIdx.x; j < k; j += blockDim.x) {
    const unsigned long long kv = key[j];
    ecc[j] = kv ? (int32_t)(kv >> 32) - 1 : -1;
    far[j] = kv ? ~(uint32_t)kv : 0xFFFFFFFFu;
    closeness[j] = total[j] ? (double)(reached[j] - 1) / (double)total[j] : 0.0;
  }
}

}  // namespace

hipError_t launch_level_stats(const int32_t* levels, uint32_t k, uint32_t n, unsigned long long* reached,
                              unsigned long long* total, int32_t* ecc, uint32_t* far, double* closeness,
                              uint32_t num_cus, hipStream_t stream) {
  static_assert(sizeof(double) == sizeof(unsigned long long), "key shares the closeness slot");
  unsigned long long* key = reinterpret_cast<unsigned long long*>(closeness);
  stats_init<<<1, 64, 0, stream>>>(k, reached, total, key);
  if (n) {
    // rows start 16-byte aligned when the array does and n is a multiple of 4
    const bool vec = n % 4 == 0 && (reinterpret_cast<uintptr_t>(levels) & 15) == 0;
    const uint64_t items = vec ? n / 4 : n;
    // about eight workgroups per CU in all, split over the k rows
    const uint64_t want = std::max<uint64_t>(1, 8ull * num_cus / k);
    const uint32_t bx = (uint32_t)std::min<uint64_t>(want, (items + kStatBlock - 1) / kStatBlock);
    if (vec)
      stats_reduce<true><<<dim3(bx, k), kStatBlock, 0, stream>>>(levels, n, reached, total, key);
    else
      stats_reduce<false><<<dim3(bx, k), kStatBlock, 0, stream>>>(levels, n, reached, total, key);
  }
  stats_final<<<1, 64, 0, stream>>>(k, reached, total, ecc, far, closeness);
  return hipGetLastError();
}

}  // namespace blest
