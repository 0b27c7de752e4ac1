// Many independent single-source BFSs in one launch (one per workgroup).
//
// Graphs of up to 131,072 vertices keep their current/next visited bitmaps and
// their frontier bitmap in LDS (3 bits per vertex), so the visited checks and the
// lazy marks of Algorithm 3 are LDS operations and a level needs only workgroup
// barriers.  The VSS queues stay in global memory (per-item scratch).  The launch
// is an ordinary kernel with one workgroup per item; items are ordered largest
// first by the host, so the hardware dispatcher's in-order issue is a
// longest-processing-time schedule.  No grid-wide wait exists, so the launch can
// be captured into a HIP graph.
#include <hip/hip_runtime.h>

#include <climits>

#include "device_common.hpp"
#include "kernels.hpp"

namespace blest {
namespace {

template <typename MT, int SLOTS>
__global__ __launch_bounds__(kManyBlock) void bfs_many_kernel(const ManyItem* __restrict__ items) {
  constexpr int SIG = 8 * sizeof(MT);
  constexpr int SPW = 32 / SIG;
  extern __shared__ uint32_t lds[];
  __shared__ uint32_t s_qlen[2];
  __shared__ uint32_t s_wave[kMaxWaves];
  __shared__ uint32_t s_base;
  const ManyItem it = items[blockIdx.x];
  const MT* masks = static_cast<const MT*>(it.masks);
  const uint32_t nw = (it.n + 31) / 32;
  uint32_t* vis = lds;             // 2 * nw: (current, next) interleaved
  uint32_t* front = lds + 2 * nw;  // nw
  const uint32_t lane = lane_id();
  const uint32_t wave = threadIdx.x / kWave, nwaves = blockDim.x / kWave;
  const uint32_t qcap = it.num_vss > 0 ? it.num_vss : 1u;
  auto orig = [&](uint32_t u) { return it.orig_id ? it.orig_id[u] : u; };

  // ---- initialisation ----
  const uint32_t so = orig(it.src);
  for (uint32_t i = threadIdx.x; i < it.n; i += blockDim.x) it.levels[i] = (i == so) ? 0 : -1;
  const uint32_t sw = it.src >> 5, sbit = 1u << (it.src & 31);
  for (uint32_t t = threadIdx.x; t < nw; t += blockDim.x) {
    const uint32_t b = (t == sw) ? sbit : 0u;
    vis[2 * t] = b;
    vis[2 * t + 1] = b;
    front[t] = b;
  }
  const uint32_t sset = it.src / SIG;
  const uint32_t q0 = it.real_ptrs[sset], q0n = it.real_ptrs[sset + 1] - q0;
  for (uint32_t j = threadIdx.x; j < q0n; j += blockDim.x) it.queue[j] = q0 + j;
  if (threadIdx.x == 0) {
    s_qlen[0] = q0n;
    s_qlen[1] = 0;
  }
  __threadfence_block();
  __syncthreads();

  for (int32_t level = 1; level <= (int32_t)it.n + 1; ++level) {
    const uint32_t* qc = it.queue + ((level - 1) & 1) * qcap;
    uint32_t* qn = it.queue + (level & 1) * qcap;
    const uint32_t len = s_qlen[(level - 1) & 1];
    // ---- Stage 1: wavefronts take VSSs round-robin; marks go to LDS ----
    // Lane l first fetches the queue entry, slice range and frontier chunk of the
    // wavefront's l-th next VSS, so the dependent entry -> metadata loads are paid
    // once per 64 VSSs (values broadcast with readlane); the slice loads of two
    // VSSs are then issued before either is applied.
    for (uint32_t base = wave; base < len; base += nwaves * kWave) {
      const uint32_t pos = base + lane * nwaves;
      uint32_t mb = 0, me = 0, ma = 0;
      if (pos < len) {
        const uint32_t v = qc[pos];
        mb = it.vss_beg[v];
        me = it.vss_beg[v + 1];
        const uint32_t bitpos = it.v2r[v] * SIG;
        ma = (front[bitpos >> 5] >> (bitpos & 31)) & (SIG == 32 ? 0xFFFFFFFFu : ((1u << SIG) - 1u));
      }
      const uint32_t cnt = min((uint32_t)kWave, (len - base + nwaves - 1) / nwaves);
      for (uint32_t k = 0; k < cnt; k += 2) {
        MT m[2][SLOTS];
        uint32_t u[2][SLOTS], alpha[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const uint32_t src = k + h < cnt ? k + h : k;
          const uint32_t beg = readlane(mb, src), end = k + h < cnt ? readlane(me, src) : beg;
          alpha[h] = readlane(ma, src);
#pragma unroll
          for (int r = 0; r < SLOTS; ++r) {
            const uint32_t idx = beg + lane + r * kWave;
            const bool ok = idx < end;
            m[h][r] = ok ? masks[idx] : MT(0);
            u[h][r] = ok ? it.row_ids[idx] : 0u;
          }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int r = 0; r < SLOTS; ++r) {
            if ((uint32_t)m[h][r] & alpha[h]) {
              const uint32_t w = u[h][r] >> 5, bit = 1u << (u[h][r] & 31);
              if (!((vis[2 * w] | vis[2 * w + 1]) & bit)) atomicOr(&vis[2 * w + 1], bit);
            }
          }
      }
    }
    if (threadIdx.x == 0) s_qlen[level & 1] = 0;
    __syncthreads();
    // ---- Stage 2: sweep the LDS bitmaps ----
    for (uint32_t b0 = 0; b0 < nw; b0 += blockDim.x) {
      const uint32_t t = b0 + threadIdx.x;
      uint32_t cnt = 0, vb[SPW], vn[SPW];
#pragma unroll
      for (int i = 0; i < SPW; ++i) vb[i] = vn[i] = 0;
      if (t < nw) {
        const uint32_t cur = vis[2 * t], nxt = vis[2 * t + 1];
        const uint32_t diff = cur ^ nxt;
        front[t] = diff;
        if (diff) {
          vis[2 * t] = nxt;
          uint32_t d = diff;
          while (d) {
            const uint32_t b = __ffs(d) - 1;
            it.levels[orig(t * 32 + b)] = level;
            d &= d - 1;
          }
#pragma unroll
          for (int i = 0; i < SPW; ++i) {
            if ((diff >> (i * SIG)) & (SIG == 32 ? 0xFFFFFFFFu : ((1u << SIG) - 1u))) {
              const uint32_t s = t * SPW + i;
              vb[i] = it.real_ptrs[s];
              vn[i] = it.real_ptrs[s + 1] - vb[i];
              cnt += vn[i];
            }
          }
        }
      }
      const uint32_t incl = wave_inclusive_scan(cnt);
      if (lane == kWave - 1) s_wave[wave] = incl;
      __syncthreads();
      if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (uint32_t w = 0; w < nwaves; ++w) {
          const uint32_t x = s_wave[w];
          s_wave[w] = run;
          run += x;
        }
        s_base = s_qlen[level & 1];
        s_qlen[level & 1] += run;
      }
      __syncthreads();
      const uint32_t pos = s_base + s_wave[wave] + incl - cnt;
      wave_push<SPW>(qn, pos, cnt, vb, vn);
      __syncthreads();
    }
    // queue entries written by other waves must be visible before Stage 1 reads them
    __threadfence_block();
    __syncthreads();
    if (s_qlen[level & 1] == 0) break;
  }
}

template <typename MT>
hipError_t launch_t(const ManyItem* items, uint32_t g, uint32_t max_n, uint32_t slots, hipStream_t stream) {
  const uint32_t lds = 3 * ((max_n + 31) / 32) * sizeof(uint32_t);
  switch (slots) {
    case 1: hipLaunchKernelGGL((bfs_many_kernel<MT, 1>), dim3(g), dim3(kManyBlock), lds, stream, items); break;
    case 2: hipLaunchKernelGGL((bfs_many_kernel<MT, 2>), dim3(g), dim3(kManyBlock), lds, stream, items); break;
    case 4: hipLaunchKernelGGL((bfs_many_kernel<MT, 4>), dim3(g), dim3(kManyBlock), lds, stream, items); break;
    case 8: hipLaunchKernelGGL((bfs_many_kernel<MT, 8>), dim3(g), dim3(kManyBlock), lds, stream, items); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_bfs_many(const ManyItem* items, uint32_t g, uint32_t max_n, uint32_t sigma, uint32_t slots,
                           hipStream_t stream) {
  if (g == 0 || max_n == 0 || max_n > kManyMaxN) return hipErrorInvalidValue;
  switch (sigma) {
    case 8: return launch_t<uint8_t>(items, g, max_n, slots, stream);
    case 16: return launch_t<uint16_t>(items, g, max_n, slots, stream);
    case 32: return launch_t<uint32_t>(items, g, max_n, slots, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace blest
