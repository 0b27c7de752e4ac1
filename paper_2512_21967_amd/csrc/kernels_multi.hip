// k-source BFS over the BVSS in one persistent launch (k <= 64).
//
// The k frontiers are stacked column-wise into an n x k bit-matrix (Section 2),
// one 64-bit word per vertex, so each level is a Boolean SpMM: for an active VSS
// of slice set s, the B tile is the sigma frontier words of the set's columns,
// and the pull of a slice (u, mask) is the OR of the B rows selected by the mask.
// That OR is the exact Boolean form of the popcount threshold of Eq. (1) taken
// over k columns at once.  The update is lazy (Algorithm 3): Stage 1 ORs the new
// bits into u's next-visited word with one 64-bit atomic (skipped when nothing is
// new); Stage 2 sweeps the vertices, sets the levels of every (source, vertex)
// pair that changed, rebuilds the frontier words and queues the VSSs of every
// slice set with a changed vertex.
//
// With sigma = 8 the B tile is 8 x 64 bits and a mask has about one set bit on
// skewed graphs, so the product is done with VALU selects and ORs; an int8 matrix
// instruction would spend its 16- or 32-deep K dimension on zeros.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"

namespace blest {
namespace {

__device__ __forceinline__ uint32_t morig(const MultiParams& p, uint32_t u) { return p.orig_id ? p.orig_id[u] : u; }

template <typename MT, int SLOTS>
__device__ __forceinline__ void multi_stage1(const MultiParams& p, const uint32_t* qc, uint32_t len) {
  constexpr int SIG = 8 * sizeof(MT);
  const MT* masks = static_cast<const MT*>(p.masks);
  const uint32_t lane = lane_id();
  const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const uint32_t nw = (gridDim.x * blockDim.x) / kWave;
  for (uint32_t base = wid; base < len; base += nw * kWave) {
    // lane l stages the metadata of this wavefront's l-th next queue position
    const uint32_t pos = base + lane * nw;
    uint32_t mb = 0, me = 0, ms = 0;
    if (pos < len) {
      const uint32_t v = qc[pos];
      mb = p.vss_beg[v];
      me = p.vss_beg[v + 1];
      ms = p.v2r[v];
    }
    const uint32_t cnt = min((uint32_t)kWave, (len - base + nw - 1) / nw);
    for (uint32_t k = 0; k < cnt; ++k) {
      const uint32_t beg = readlane(mb, k), end = readlane(me, k), ss = readlane(ms, k);
      // B tile: the frontier words of the set's sigma columns
      const uint32_t col = ss * SIG + lane;
      const uint64_t bw = (lane < (uint32_t)SIG && col < p.n) ? p.front[col] : 0ull;
      uint64_t B[SIG];
#pragma unroll
      for (int j = 0; j < SIG; ++j) B[j] = readlane64(bw, j);
      MT m[SLOTS];
      uint32_t u[SLOTS];
#pragma unroll
      for (int r = 0; r < SLOTS; ++r) {
        const uint32_t idx = beg + lane + r * kWave;
        const bool ok = idx < end;
        m[r] = ok ? masks[idx] : MT(0);
        u[r] = ok ? p.row_ids[idx] : 0u;
      }
      uint64_t acc[SLOTS];
      ulonglong2 cv[SLOTS];
#pragma unroll
      for (int r = 0; r < SLOTS; ++r) {
        uint64_t a = 0;
#pragma unroll
        for (int j = 0; j < SIG; ++j) a |= ((uint32_t)m[r] >> j & 1u) ? B[j] : 0ull;
        acc[r] = a;
        cv[r] = reinterpret_cast<const ulonglong2*>(p.vis)[a ? u[r] : 0u];
      }
#pragma unroll
      for (int r = 0; r < SLOTS; ++r) {
        const uint64_t fresh = acc[r] & ~cv[r].x & ~cv[r].y;
        if (fresh) atomicOr(p.vis + 2 * (uint64_t)u[r] + 1, (unsigned long long)fresh);
      }
    }
  }
}

template <int SIG>
__device__ __forceinline__ void multi_stage2(const MultiParams& p, uint32_t* qn, uint32_t* qlen, int32_t level) {
  __shared__ uint32_t s_wave[kMaxWaves];
  __shared__ uint32_t s_base;
  const uint32_t lane = lane_id();
  const uint32_t wave = threadIdx.x / kWave, nwaves = blockDim.x / kWave;
  for (uint32_t b0 = blockIdx.x * blockDim.x; b0 < p.n; b0 += gridDim.x * blockDim.x) {
    const uint32_t u = b0 + threadIdx.x;
    uint64_t diff = 0;
    if (u < p.n) {
      const ulonglong2 cv = reinterpret_cast<const ulonglong2*>(p.vis)[u];
      diff = cv.y & ~cv.x;
      p.front[u] = diff;
      if (diff) {
        p.vis[2 * (uint64_t)u] = cv.y;
        const uint32_t uo = morig(p, u);
        uint64_t d = diff;
        while (d) {
          const uint32_t j = __ffsll((unsigned long long)d) - 1;
          p.levels[(uint64_t)j * p.n + uo] = level;
          d &= d - 1;
        }
      }
    }
    // a slice set is active iff one of its sigma consecutive vertices changed
    const uint64_t changed = __ballot(diff != 0);
    uint32_t cnt = 0, vb[1] = {0}, vn[1] = {0};
    const bool leader = (lane % SIG) == 0 && u < p.n;
    if (leader && ((changed >> lane) & (SIG == 64 ? ~0ull : ((1ull << SIG) - 1))) != 0) {
      const uint32_t ss = u / SIG;
      vb[0] = p.real_ptrs[ss];
      vn[0] = cnt = p.real_ptrs[ss + 1] - vb[0];
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
      s_base = run ? atomicAdd(qlen, run) : 0u;
    }
    __syncthreads();
    const uint32_t pos = s_base + s_wave[wave] + incl - cnt;
    wave_push<1>(qn, pos, cnt, vb, vn);
    __syncthreads();
  }
}

template <typename MT, int SLOTS>
__global__ __launch_bounds__(1024) void bfs_multi_persistent(MultiParams p) {
  constexpr int SIG = 8 * sizeof(MT);
  uint32_t* ctrl = p.ctrl;
  uint32_t* qlen = ctrl + kQlen;
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t nt = gridDim.x * blockDim.x;

  // ---- initialisation ----
  for (uint32_t j = 0; j < p.k; ++j) {
    const uint32_t so = morig(p, p.src[j]);
    int32_t* row = p.levels + (uint64_t)j * p.n;
    for (uint32_t v = tid; v < p.n; v += nt) row[v] = (v == so) ? 0 : -1;
  }
  for (uint32_t u = tid; u < p.n; u += nt) {
    unsigned long long b = 0;
    for (uint32_t j = 0; j < p.k; ++j) b |= (p.src[j] == u) ? (1ull << j) : 0ull;
    p.vis[2 * (uint64_t)u] = b;
    p.vis[2 * (uint64_t)u + 1] = b;
    p.front[u] = b;
  }
  // initial queue: the VSS ranges of the sources' distinct slice sets
  {
    uint32_t off = 0;
    for (uint32_t i = 0; i < p.n_init_sets; ++i) {
      const uint32_t b = p.real_ptrs[p.init_sets[i]], e = p.real_ptrs[p.init_sets[i] + 1];
      for (uint32_t j = tid; j < e - b; j += nt) p.queue[off + j] = b + j;
      off += e - b;
    }
    if (tid == 0) {
      qlen[0] = off;
      qlen[kLine] = 0;
      qlen[2 * kLine] = 0;
    }
  }
  grid_barrier(ctrl);

  for (int32_t level = 1; level <= (int32_t)p.n + 1; ++level) {
    const uint32_t* qc = p.queue + ((level - 1) & 1) * p.qcap;
    uint32_t* qn = p.queue + (level & 1) * p.qcap;
    const uint32_t len = ld_relaxed(qlen + ((level - 1) % 3) * kLine);
    uint32_t* qnext_len = qlen + (level % 3) * kLine;
    if (tid == 0) __hip_atomic_store(qlen + ((level + 1) % 3) * kLine, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    multi_stage1<MT, SLOTS>(p, qc, len);
    grid_barrier(ctrl);
    multi_stage2<SIG>(p, qn, qnext_len, level);
    grid_barrier(ctrl);
    if (ld_relaxed(qnext_len) == 0) break;
  }
}

template <typename MT>
const void* msym(uint32_t slots) {
  switch (slots) {
    case 1: return reinterpret_cast<const void*>(&bfs_multi_persistent<MT, 1>);
    case 2: return reinterpret_cast<const void*>(&bfs_multi_persistent<MT, 2>);
    case 4: return reinterpret_cast<const void*>(&bfs_multi_persistent<MT, 4>);
    case 8: return reinterpret_cast<const void*>(&bfs_multi_persistent<MT, 8>);
    default: return nullptr;
  }
}

}  // namespace

const void* bfs_multi_kernel_symbol(uint32_t sigma, uint32_t slots) {
  switch (sigma) {
    case 8: return msym<uint8_t>(slots);
    case 16: return msym<uint16_t>(slots);
    case 32: return msym<uint32_t>(slots);
    default: return nullptr;
  }
}

hipError_t launch_bfs_multi(const MultiParams& p, uint32_t sigma, uint32_t slots, uint32_t grid, uint32_t block,
                            hipStream_t stream) {
  const void* k = bfs_multi_kernel_symbol(sigma, slots);
  if (!k) return hipErrorInvalidValue;
  MultiParams copy = p;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel(k, dim3(grid), dim3(block), args, 0, stream);
}

}  // namespace blest
