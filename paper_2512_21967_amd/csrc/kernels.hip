// HIP kernels for gfx950 (CDNA4): the fused, persistent pull-BFS over Binarised
// Virtual Slice Sets.
//
// Mapping of the method onto a 64-lane wavefront:
//   * One wavefront owns one virtual slice set (VSS) at a time; VSSs of the
//     current queue are dealt to wavefronts round-robin (Section 2.1.1).
//   * Lane l handles slices l, l + 64, ... of the VSS, which are stored
//     contiguously in row order, so each round is one coalesced 256-byte row-ID
//     load and one mask load per wavefront (column-major placement, Section
//     2.1.2, with 64 lanes).
//   * The Boolean pull of a slice is (mask AND alpha) != 0, where alpha is the
//     sigma-bit frontier chunk of the VSS's slice set: the popcount-threshold of
//     Eq. (1) with a single frontier column, done with one VALU AND.  gfx950 has
//     no 1-bit matrix instruction, and a single frontier vector is not a dense
//     tile, so no MFMA is used here.
//   * Lazy scheme (Algorithm 3, Section 3.2): a hit only sets the vertex's bit in
//     the next-visited bitmap with a non-returning atomic OR (skipped when the bit
//     is already visible); a coalesced sweep over 32-vertex words then writes the
//     levels, the next frontier and the next queue, with one queue reservation
//     per wavefront (ballot-free prefix scan + one atomic add).
//   * Eager scheme (Algorithm 2): a hit claims the vertex with a returning atomic
//     OR on the next frontier; the first claimer in a slice set's chunk pushes the
//     set's VSS range.  The visited bitmap (not the level array) filters hits.
//   * All levels run in one cooperative launch with a two-level (per-XCD group,
//     then root) grid barrier (Section 3.3).
#include <hip/hip_runtime.h>

#include <climits>

#include "kernels.hpp"

namespace blest {
namespace {

constexpr int kWave = 64;

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ uint32_t ld_relaxed(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Two-level grid barrier.  Block b arrives on the counter of group b % 8 (the
// XCD it is dispatched to); the last arrival of a group arrives on the root; the
// last root arrival resets the counters and bumps the generation, on which every
// other block waits.  Arrivals are acq_rel and the generation is published with
// release and read with acquire, all at agent scope, so every write made before
// the barrier by any block is visible after it.
__device__ __forceinline__ void grid_barrier(uint32_t* ctrl) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t nb = gridDim.x;
    const uint32_t grp = blockIdx.x % kBarGroups;
    const uint32_t ngroups = nb < kBarGroups ? nb : kBarGroups;
    const uint32_t gsize = (nb - grp + kBarGroups - 1) / kBarGroups;
    uint32_t* gen = ctrl + kBarGen;
    const uint32_t g0 = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bool flipped = false;
    uint32_t prev = __hip_atomic_fetch_add(ctrl + grp * kLine, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == gsize - 1) {
      __hip_atomic_store(ctrl + grp * kLine, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      uint32_t r = __hip_atomic_fetch_add(ctrl + kBarRoot, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (r == ngroups - 1) {
        __hip_atomic_store(ctrl + kBarRoot, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(gen, g0 + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        flipped = true;
      }
    }
    if (!flipped)
      while (__hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g0) __builtin_amdgcn_s_sleep(1);
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

__device__ __forceinline__ uint32_t to_orig(const BfsParams& p, uint32_t u) {
  return p.orig_id ? p.orig_id[u] : u;
}

template <int SIG>
__device__ __forceinline__ uint32_t chunk_mask() {
  return SIG == 32 ? 0xFFFFFFFFu : ((1u << SIG) - 1u);
}

// sigma-bit frontier chunk of slice set ss inside a 32-bit-word bitmap.
template <int SIG>
__device__ __forceinline__ uint32_t frontier_chunk(const uint32_t* f, uint32_t ss) {
  const uint32_t bitpos = ss * SIG;
  return (f[bitpos >> 5] >> (bitpos & 31)) & chunk_mask<SIG>();
}

// Reserves `cnt` queue slots for this lane with one atomic add per wavefront and
// returns the lane's first slot (undefined when the wavefront total is zero).
// Every lane of the wavefront must call this.
__device__ __forceinline__ uint32_t wave_reserve(uint32_t* qlen, uint32_t cnt, uint32_t& total) {
  const uint32_t incl = wave_inclusive_scan(cnt);
  total = __shfl(incl, kWave - 1, kWave);
  uint32_t base = 0;
  if (total != 0 && lane_id() == 0) base = atomicAdd(qlen, total);
  base = __shfl(base, 0, kWave);
  return base + incl - cnt;
}

// Appends the VSS range of slice set ss at qn[pos ...].
__device__ __forceinline__ uint32_t push_set(const BfsParams& p, uint32_t* qn, uint32_t pos, uint32_t ss) {
  const uint32_t b = p.real_ptrs[ss], e = p.real_ptrs[ss + 1];
  for (uint32_t v = b; v < e; ++v) qn[pos++] = v;
  return pos;
}

// Stage 1 of the lazy scheme: mark the next-visited bits of all pulled rows.
template <typename MT, int SLOTS>
__device__ __forceinline__ void stage1_lazy(const BfsParams& p, const uint32_t* qc, uint32_t len) {
  constexpr int SIG = 8 * sizeof(MT);
  const MT* masks = static_cast<const MT*>(p.masks);
  const uint32_t lane = lane_id();
  const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const uint32_t nw = (gridDim.x * blockDim.x) / kWave;
  for (uint32_t q = wid; q < len; q += nw) {
    const uint32_t v = qc[q];
    const uint32_t beg = p.vss_beg[v], end = p.vss_beg[v + 1];
    const uint32_t alpha = frontier_chunk<SIG>(p.front, p.v2r[v]);
    MT m[SLOTS];
    uint32_t u[SLOTS];
#pragma unroll
    for (int r = 0; r < SLOTS; ++r) {
      const uint32_t k = beg + lane + r * kWave;
      const bool ok = k < end;
      m[r] = ok ? masks[k] : MT(0);
      u[r] = ok ? p.row_ids[k] : 0u;
    }
#pragma unroll
    for (int r = 0; r < SLOTS; ++r) {
      if ((uint32_t)m[r] & alpha) {
        const uint32_t w = u[r] >> 5, bit = 1u << (u[r] & 31);
        const uint2 cv = reinterpret_cast<const uint2*>(p.vis)[w];  // (current, next)
        if (!((cv.x | cv.y) & bit)) atomicOr(p.vis + 2 * w + 1, bit);
      }
    }
  }
}

// Stage 2 of the lazy scheme: coalesced sweep over 32-vertex words.
template <int SIG>
__device__ __forceinline__ void stage2_lazy(const BfsParams& p, uint32_t* qn, uint32_t* qlen, int32_t level) {
  constexpr int SPW = 32 / SIG;  // slice sets per word
  const uint32_t lane = lane_id();
  const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const uint32_t nw = (gridDim.x * blockDim.x) / kWave;
  for (uint32_t base = wid * kWave; base < p.n_words; base += nw * kWave) {
    const uint32_t t = base + lane;
    uint32_t cnt = 0, pushmask = 0;
    if (t < p.n_words) {
      const uint2 cv = reinterpret_cast<const uint2*>(p.vis)[t];
      const uint32_t diff = cv.x ^ cv.y;
      if (diff) {
        p.vis[2 * t] = cv.y;
        p.front[t] = diff;
        uint32_t d = diff;
        while (d) {
          const uint32_t b = __ffs(d) - 1;
          p.levels[to_orig(p, t * 32 + b)] = level;
          d &= d - 1;
        }
#pragma unroll
        for (int i = 0; i < SPW; ++i) {
          if ((diff >> (i * SIG)) & chunk_mask<SIG>()) {
            const uint32_t ss = t * SPW + i;
            pushmask |= 1u << i;
            cnt += p.real_ptrs[ss + 1] - p.real_ptrs[ss];
          }
        }
      }
    }
    uint32_t total;
    uint32_t pos = wave_reserve(qlen, cnt, total);
    if (total != 0 && cnt != 0) {
#pragma unroll
      for (int i = 0; i < SPW; ++i)
        if (pushmask & (1u << i)) pos = push_set(p, qn, pos, t * SPW + i);
    }
  }
}

// Stage 1 of the eager scheme: claim, write the level, push the set's VSSs.
template <typename MT, int SLOTS>
__device__ __forceinline__ void stage1_eager(const BfsParams& p, const uint32_t* qc, uint32_t len,
                                             const uint32_t* fc, uint32_t* fn, uint32_t* qn, uint32_t* qlen,
                                             int32_t level) {
  constexpr int SIG = 8 * sizeof(MT);
  const MT* masks = static_cast<const MT*>(p.masks);
  const uint32_t lane = lane_id();
  const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const uint32_t nw = (gridDim.x * blockDim.x) / kWave;
  for (uint32_t q = wid; q < len; q += nw) {
    const uint32_t v = qc[q];
    const uint32_t beg = p.vss_beg[v], end = p.vss_beg[v + 1];
    const uint32_t alpha = frontier_chunk<SIG>(fc, p.v2r[v]);
    MT m[SLOTS];
    uint32_t u[SLOTS];
#pragma unroll
    for (int r = 0; r < SLOTS; ++r) {
      const uint32_t k = beg + lane + r * kWave;
      const bool ok = k < end;
      m[r] = ok ? masks[k] : MT(0);
      u[r] = ok ? p.row_ids[k] : 0u;
    }
    uint32_t pushmask = 0, cnt = 0;
#pragma unroll
    for (int r = 0; r < SLOTS; ++r) {
      if ((uint32_t)m[r] & alpha) {
        const uint32_t x = u[r];
        const uint32_t w = x >> 5, bit = 1u << (x & 31);
        if (!(p.vis[w] & bit)) {
          const uint32_t old = atomicOr(fn + w, bit);
          if (!(old & bit)) {
            atomicOr(p.vis + w, bit);
            p.levels[to_orig(p, x)] = level;
            const uint32_t sh = (x & 31) & ~(uint32_t)(SIG - 1);
            if (((old >> sh) & chunk_mask<SIG>()) == 0) {
              const uint32_t ss = x / SIG;
              pushmask |= 1u << r;
              cnt += p.real_ptrs[ss + 1] - p.real_ptrs[ss];
            }
          }
        }
      }
    }
    uint32_t total;
    uint32_t pos = wave_reserve(qlen, cnt, total);
    if (total != 0 && cnt != 0) {
#pragma unroll
      for (int r = 0; r < SLOTS; ++r)
        if (pushmask & (1u << r)) pos = push_set(p, qn, pos, u[r] / SIG);
    }
  }
}

// Clears the frontier chunks of the sets named by queue qold (eager scheme).
template <int SIG>
__device__ __forceinline__ void clear_chunks(const BfsParams& p, uint32_t* f, const uint32_t* qold, uint32_t len) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t nt = gridDim.x * blockDim.x;
  for (uint32_t i = tid; i < len; i += nt) {
    const uint32_t ss = p.v2r[qold[i]];
    if (SIG == 8) reinterpret_cast<uint8_t*>(f)[ss] = 0;
    else if (SIG == 16) reinterpret_cast<uint16_t*>(f)[ss] = 0;
    else f[ss] = 0;
  }
}

template <typename MT, int SLOTS, bool LAZY>
__global__ __launch_bounds__(1024) void bfs_persistent(BfsParams p) {
  constexpr int SIG = 8 * sizeof(MT);
  uint32_t* ctrl = p.ctrl;
  uint32_t* qlen = ctrl + kQlen;  // qlen[i] at qlen[i * kLine]
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t nt = gridDim.x * blockDim.x;
  const uint32_t sw = p.src >> 5, sbit = 1u << (p.src & 31);
  const uint32_t sset = p.src / SIG;
  const uint32_t q0b = p.real_ptrs[sset], q0n = p.real_ptrs[sset + 1] - q0b;
  const uint32_t so = to_orig(p, p.src);

  // ---- initialisation (Algorithm 2/3, first lines) ----
  for (uint32_t i = tid; i < p.n; i += nt) p.levels[i] = (i == so) ? 0 : -1;
  if (LAZY) {
    for (uint32_t t = tid; t < p.n_words; t += nt) {
      const uint32_t b = (t == sw) ? sbit : 0u;
      p.vis[2 * t] = b;
      p.vis[2 * t + 1] = b;
      p.front[t] = b;
    }
  } else {
    for (uint32_t t = tid; t < p.n_words; t += nt) {
      const uint32_t b = (t == sw) ? sbit : 0u;
      p.vis[t] = b;
      p.front[t] = b;
      p.front[p.n_words + t] = 0;
      p.front[2 * p.n_words + t] = 0;
    }
  }
  for (uint32_t j = tid; j < q0n; j += nt) p.queue[j] = q0b + j;
  if (tid == 0) {
    qlen[0] = q0n;
    qlen[kLine] = 0;
    qlen[2 * kLine] = 0;
    qlen[3 * kLine] = 0;
  }
  grid_barrier(ctrl);

  for (int32_t level = 1; level <= (int32_t)p.n + 1; ++level) {
    if (LAZY) {
      const uint32_t* qc = p.queue + ((level - 1) & 1) * p.qcap;
      uint32_t* qn = p.queue + (level & 1) * p.qcap;
      const uint32_t len = ld_relaxed(qlen + ((level - 1) % 3) * kLine);
      uint32_t* qnext_len = qlen + (level % 3) * kLine;
      if (tid == 0) __hip_atomic_store(qlen + ((level + 1) % 3) * kLine, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      stage1_lazy<MT, SLOTS>(p, qc, len);
      grid_barrier(ctrl);
      stage2_lazy<SIG>(p, qn, qnext_len, level);
      grid_barrier(ctrl);
      if (ld_relaxed(qnext_len) == 0) break;
    } else {
      const uint32_t* qc = p.queue + ((level - 1) % 3) * p.qcap;
      uint32_t* qn = p.queue + (level % 3) * p.qcap;
      const uint32_t* qold = p.queue + ((level + 1) % 3) * p.qcap;  // queue of level - 2
      const uint32_t len = ld_relaxed(qlen + ((level - 1) % 4) * kLine);
      const uint32_t old_len = ld_relaxed(qlen + ((level + 2) % 4) * kLine);
      uint32_t* qnext_len = qlen + (level % 4) * kLine;
      if (tid == 0) __hip_atomic_store(qlen + ((level + 1) % 4) * kLine, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint32_t* fc = p.front + ((level - 1) % 3) * p.n_words;
      uint32_t* fn = p.front + (level % 3) * p.n_words;
      uint32_t* fold = p.front + ((level + 1) % 3) * p.n_words;
      clear_chunks<SIG>(p, fold, qold, old_len);
      stage1_eager<MT, SLOTS>(p, qc, len, fc, fn, qn, qnext_len, level);
      grid_barrier(ctrl);
      if (ld_relaxed(qnext_len) == 0) break;
    }
  }
}

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

template <typename MT, int SLOTS, bool LAZY>
const void* sym() {
  return reinterpret_cast<const void*>(&bfs_persistent<MT, SLOTS, LAZY>);
}

template <typename MT>
const void* sym_slots(uint32_t slots, bool lazy) {
  switch (slots) {
    case 1: return lazy ? sym<MT, 1, true>() : sym<MT, 1, false>();
    case 2: return lazy ? sym<MT, 2, true>() : sym<MT, 2, false>();
    case 4: return lazy ? sym<MT, 4, true>() : sym<MT, 4, false>();
    case 8: return lazy ? sym<MT, 8, true>() : sym<MT, 8, false>();
    default: return nullptr;
  }
}

}  // namespace

const void* bfs_kernel_symbol(uint32_t sigma, uint32_t slots, bool lazy) {
  switch (sigma) {
    case 8: return sym_slots<uint8_t>(slots, lazy);
    case 16: return sym_slots<uint16_t>(slots, lazy);
    case 32: return sym_slots<uint32_t>(slots, lazy);
    default: return nullptr;
  }
}

hipError_t launch_bfs(const BfsParams& p, uint32_t sigma, uint32_t slots, bool lazy, uint32_t grid,
                      uint32_t block, hipStream_t stream) {
  const void* k = bfs_kernel_symbol(sigma, slots, lazy);
  if (!k) return hipErrorInvalidValue;
  BfsParams copy = p;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel(k, dim3(grid), dim3(block), args, 0, stream);
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
