// HIP kernels for gfx950 (CDNA4) around the persistent single-source BFS: the
// kernel-symbol dispatch and launch, the parents post-pass, the barrier probe and
// the allocation-free entry point's static scratch.  The persistent kernel itself
// is in bfs_kernel.hpp, instantiated per scheme in kernels_eager.hip,
// kernels_lazy.hip and kernels_adaptive.hip.
#include <hip/hip_runtime.h>

#include <climits>
#include <mutex>

#include "../../include/blest.h"
#include "bfs_kernel.hpp"

namespace blest {
namespace {

// ---- parents post-pass ----
__global__ void parents_init(const int32_t* __restrict__ levels, int32_t* __restrict__ parents, uint32_t n) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    parents[v] = levels[v] < 0 ? -1 : (levels[v] == 0 ? (int32_t)v : INT_MAX);
}

template <typename MT>
__global__ void parents_scan(BfsParams p, const int32_t* __restrict__ levels, int32_t* parents) {
  constexpr int SIG = 8 * sizeof(MT);
  const MT* masks = static_cast<const MT*>(p.masks);
  const uint32_t lane = lane_id();
  const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const uint32_t nw = (gridDim.x * blockDim.x) / kWave;
  for (uint32_t v = wid; v < p.num_vss; v += nw) {
    const uint32_t ss = p.v2r[v];
    for (uint32_t k = p.vss_beg[v] + lane; k < p.vss_beg[v + 1]; k += kWave) {
      const uint32_t u = p.row_ids[k];
      const uint32_t uo = to_orig(p, u);
      const int32_t lu = levels[uo];
      if (lu <= 0) continue;
      uint32_t m = masks[k];
      while (m) {
        const uint32_t j = __ffs(m) - 1;
        m &= m - 1;
        const uint32_t co = to_orig(p, ss * SIG + j);
        if (levels[co] == lu - 1) atomicMin(parents + uo, (int32_t)co);
      }
    }
  }
}

// `rounds` grid barriers and nothing else, in the persistent kernels' launch shape.
__global__ __launch_bounds__(1024) void barrier_probe(uint32_t* ctrl, uint32_t rounds) {
  for (uint32_t r = 0; r < rounds; ++r) grid_barrier(ctrl);
}

__global__ void zero_words(uint32_t* __restrict__ p, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

}  // namespace

// Scratch of the allocation-free single-source entry point (blest_bfs_noalloc):
// visited bits, reached bytes, frontier bitmaps, queues and the control block of
// one call, carved out at 256-byte boundaries.  Each device holds its own copy
// for the life of the process.  In host code this name is only a stand-in for
// the symbol: kernels get the address that hipGetSymbolAddress reports for the
// current device (noalloc_scratch), never the name itself.
static __device__ __align__(256) unsigned char scratch[BLEST_NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch(int device, void** ptr) {
  static std::mutex mu;
  static void* addr[64] = {};
  if (device < 0 || device >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[device]) {
    void* a = nullptr;
    const hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = a;
  }
  *ptr = addr[device];
  return hipSuccess;
}

hipError_t launch_barrier_probe(uint32_t* ctrl, uint32_t rounds, uint32_t grid, uint32_t block, hipStream_t stream) {
  void* args[] = {&ctrl, &rounds};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&barrier_probe), dim3(grid), dim3(block), args, 0,
                                    stream);
}

const void* barrier_probe_symbol() { return reinterpret_cast<const void*>(&barrier_probe); }

hipError_t launch_zero_words(uint32_t* p, uint32_t n, hipStream_t stream) {
  hipLaunchKernelGGL(zero_words, dim3(1), dim3(512), 0, stream, p, n);
  return hipGetLastError();
}

const void* bfs_kernel_symbol(uint32_t sigma, uint32_t slots, int mode, uint32_t group, bool lds, bool packed) {
  switch (mode) {
    case kEager: return bfs_symbol_eager(sigma, slots, group, packed);
    case kLazy: return bfs_symbol_lazy(sigma, slots, group, lds, packed);
    case kAdaptive: return bfs_symbol_adaptive(sigma, slots, group, lds, packed);
    default: return nullptr;
  }
}

hipError_t launch_bfs(const BfsParams& p, uint32_t sigma, uint32_t slots, int mode, uint32_t group, uint32_t grid,
                      uint32_t block, hipStream_t stream) {
  const bool lds = mode != kEager && p.range_words > 0;
  const void* k = bfs_kernel_symbol(sigma, slots, mode, group, lds, p.packed != nullptr);
  if (!k || grid % p.nranges != 0) return hipErrorInvalidValue;
  BfsParams copy = p;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel(k, dim3(grid), dim3(block), args, lds ? 4 * p.range_words : 0, stream);
}

hipError_t launch_parents(const BfsParams& p, uint32_t sigma, const int32_t* levels, int32_t* parents,
                          hipStream_t stream) {
  const uint32_t block = 256;
  uint32_t g1 = (p.n + block - 1) / block;
  if (g1 > 65535) g1 = 65535;
  if (g1 == 0) g1 = 1;
  hipLaunchKernelGGL(parents_init, dim3(g1), dim3(block), 0, stream, levels, parents, p.n);
  uint32_t g2 = (p.num_vss + 3) / 4;
  if (g2 > 65535) g2 = 65535;
  if (g2 == 0) g2 = 1;
  switch (sigma) {
    case 8: hipLaunchKernelGGL(parents_scan<uint8_t>, dim3(g2), dim3(block), 0, stream, p, levels, parents); break;
    case 16: hipLaunchKernelGGL(parents_scan<uint16_t>, dim3(g2), dim3(block), 0, stream, p, levels, parents); break;
    case 32: hipLaunchKernelGGL(parents_scan<uint32_t>, dim3(g2), dim3(block), 0, stream, p, levels, parents); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace blest
