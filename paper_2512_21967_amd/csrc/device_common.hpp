// Device helpers shared by the BFS kernels: wavefront primitives and the grid
// barrier of the persistent launches.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace blest {
namespace {

constexpr int kWave = 64;
constexpr int kMaxWaves = 1024 / kWave;  // wavefronts per workgroup at most

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ uint32_t ld_relaxed(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Two-level grid barrier.  Block b arrives on the counter of group b % 8 (the
// XCD it is dispatched to); the last arrival of a group arrives on the root; the
// last root arrival resets the counters and bumps the generation, on which every
// other block spins.  Ordering comes from fences, not from the counters: each
// block issues an agent-scope release fence before arriving and an agent-scope
// acquire fence after seeing the new generation, and the last arrival of a group
// and the flipping block issue acq_rel fences between their counter updates
// (fence-to-fence synchronisation through the counters), so every write made before
// the barrier by any block is visible to every block after it.  Arrivals and the
// spin are relaxed, which keeps cache maintenance out of the spin loop (about 3x
// cheaper than acquire loads in the loop on MI355X).
__device__ __forceinline__ void grid_barrier(uint32_t* ctrl) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t nb = gridDim.x;
    const uint32_t grp = blockIdx.x % kBarGroups;
    const uint32_t ngroups = nb < kBarGroups ? nb : kBarGroups;
    const uint32_t gsize = (nb - grp + kBarGroups - 1) / kBarGroups;
    uint32_t* gen = ctrl + kBarGen;
    const uint32_t g0 = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    bool flipped = false;
    if (__hip_atomic_fetch_add(ctrl + grp * kLine, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gsize - 1) {
      __hip_atomic_store(ctrl + grp * kLine, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");  // carries the group's writes to the root
      if (__hip_atomic_fetch_add(ctrl + kBarRoot, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == ngroups - 1) {
        __hip_atomic_store(ctrl + kBarRoot, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
        __hip_atomic_store(gen, g0 + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        flipped = true;
      }
    }
    if (!flipped)
      while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g0) __builtin_amdgcn_s_sleep(1);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// Inclusive prefix sum across the 64 lanes of a wavefront.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    uint32_t y = __shfl_up(x, o, kWave);
    if (lane >= (uint32_t)o) x += y;
  }
  return x;
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, uint32_t lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)lane);
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, uint32_t lane) {
  const uint32_t lo = readlane((uint32_t)v, lane), hi = readlane((uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

struct PlainEntry {
  __device__ uint32_t operator()(uint32_t v, uint32_t) const { return v; }
};

// Writes a lane's VSS ranges [vb[i], vb[i] + vn[i]) for i < SETS (vn[i] = 0: none)
// at qn[pos ...], in order; cnt is the sum of vn.  Entry x of range i is
// enc(vb[i] + x, vt[i]) (vt: a per-range tag, e.g. the set's frontier chunk).
// Lanes with at most kSmallPush entries write their own; longer pushes (hub
// slice sets own thousands of VSSs) are written by the whole wavefront, 4 x 64
// entries per step, lane after lane.  The ranges arrive in registers, so the
// wavefront-wide part issues no load besides what the encoder reads.  Every
// lane of the wavefront must call this.
constexpr uint32_t kSmallPush = 8;
template <int SETS, class Q, class Enc>
__device__ __forceinline__ void wave_push(Q* qn, uint32_t pos, uint32_t cnt, const uint32_t (&vb)[SETS],
                                          const uint32_t (&vn)[SETS], const uint32_t (&vt)[SETS], Enc enc) {
  const bool small = cnt <= kSmallPush;
  if (small && cnt) {
#pragma unroll
    for (int i = 0; i < SETS; ++i)
      for (uint32_t v = vb[i]; v < vb[i] + vn[i]; ++v) qn[pos++] = enc(v, vt[i]);
  }
  uint64_t big = __ballot(!small);
  while (big) {
    const uint32_t l = __ffsll((unsigned long long)big) - 1;
    big &= big - 1;
    uint32_t lp = readlane(pos, l);
#pragma unroll
    for (int i = 0; i < SETS; ++i) {
      const uint32_t n = readlane(vn[i], l);
      if (n == 0) continue;
      const uint32_t b = readlane(vb[i], l);
      const uint32_t tag = readlane(vt[i], l);
      for (uint32_t x0 = 0; x0 < n; x0 += 4 * kWave) {
        Q val[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t x = x0 + j * kWave + lane_id();
          val[j] = enc(b + (x < n ? x : 0u), tag);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t x = x0 + j * kWave + lane_id();
          if (x < n) qn[lp + x] = val[j];
        }
      }
      lp += n;
    }
  }
}

// Plain VSS-ID pushes (no tag).
template <int SETS>
__device__ __forceinline__ void wave_push(uint32_t* qn, uint32_t pos, uint32_t cnt, const uint32_t (&vb)[SETS],
                                          const uint32_t (&vn)[SETS]) {
  uint32_t vt[SETS];
#pragma unroll
  for (int i = 0; i < SETS; ++i) vt[i] = 0;
  wave_push<SETS>(qn, pos, cnt, vb, vn, vt, PlainEntry{});
}

}  // namespace
}  // namespace blest
