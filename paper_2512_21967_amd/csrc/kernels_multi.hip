// k-source BFS over the BVSS in one persistent launch (k <= 64).
//
// The k frontiers are stacked column-wise into an n x k bit-matrix (Section 2),
// one 64-bit word per vertex, so each level is a Boolean SpMM: for an active VSS
// of slice set s, the B tile is the sigma frontier words of the set's columns,
// and the pull of a slice (u, mask) is the OR of the B rows selected by the mask.
// That OR is the exact Boolean form of the popcount threshold of Eq. (1) taken
// over k columns at once.  The update is lazy (Algorithm 3): Stage 1 ORs the new
// bits into u's next-visited word with one 64-bit atomic (skipped when nothing is
// new); Stage 2 visits the vertices that changed (tracked by a state byte per
// vertex, or by a full sweep on dense levels), sets the levels of every (source,
// vertex) pair that changed, rebuilds the frontier words and queues the VSSs of
// every slice set with a changed vertex.
//
// With sigma = 8 the B tile is 8 x 64 bits and a mask has about one set bit on
// skewed graphs, so the product is done with VALU selects and ORs; an int8 matrix
// instruction would spend its 16- or 32-deep K dimension on zeros.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"

namespace blest {
namespace {

// A level is swept densely when its queue holds at least 1/kDenseFrac of the VSSs.
constexpr uint64_t kDenseFrac = 16;

__device__ __forceinline__ uint32_t morig(const MultiParams& p, uint32_t u) { return p.orig_id ? p.orig_id[u] : u; }

// Queue entry of VSS v: (v << kRangeBits) | its row range.
struct MultiEntry {
  const uint8_t* vss_range;  // nullptr: one range
  __device__ uint32_t operator()(uint32_t v, uint32_t) const {
    return vss_range ? (v << kRangeBits) | vss_range[v] : v << kRangeBits;
  }
};

// Stage 1.  With p.nranges = R > 1 every VSS pulls rows of one row range only,
// and workgroup b serves range b % R: wavefronts scan the queue in strides of the
// range group's wavefront count and take the entries of their range.  Workgroups
// are dealt to the 8 XCDs round-robin, so with R = 8 the rows of a range, and
// their visited pairs, are pulled, read and ORed from one XCD, whose L2 holds
// that range's share of the pairs.
template <typename MT, int SLOTS>
__device__ __forceinline__ void multi_stage1(const MultiParams& p, const uint32_t* qc, uint32_t len, bool mark) {
  constexpr int SIG = 8 * sizeof(MT);
  const MT* masks = static_cast<const MT*>(p.masks);
  const uint32_t lane = lane_id();
  const uint32_t R = p.nranges, rg = blockIdx.x % R;
  const uint32_t W = blockDim.x / kWave;
  const uint32_t wid = (blockIdx.x / R) * W + threadIdx.x / kWave;
  const uint32_t nw = (gridDim.x / R) * W;
  for (uint32_t base = wid; base < len; base += nw * kWave) {
    // lane l stages the metadata of this wavefront's l-th next queue position
    const uint32_t pos = base + lane * nw;
    const uint32_t e = pos < len ? qc[pos] : 0u;
    const bool mine = pos < len && (e & (kMaxRanges - 1)) == rg;
    uint32_t mb = 0, me = 0, ms = 0;
    if (mine) {
      const uint32_t v = e >> kRangeBits;
      mb = p.vss_beg[v];
      me = p.vss_beg[v + 1];
      ms = p.v2r[v];
    }
    uint64_t pick = __ballot(mine);
    // Two VSSs per step at sigma <= 16 (their B tiles, 2 x sigma 64-bit words, are
    // broadcast to scalar registers): the B-tile and slice loads of both are issued
    // before either is applied, and so are their visited-pair reads, which halves
    // the chain of dependent round trips per VSS.  At sigma = 32 two tiles would not
    // fit the scalar registers, so one VSS per step.
    constexpr int P = SIG <= 16 ? 2 : 1;
    while (pick) {
      uint32_t beg[P], end[P], ss[P];
#pragma unroll
      for (int h = 0; h < P; ++h) {
        const bool any = pick != 0;
        const uint32_t k = any ? __ffsll((unsigned long long)pick) - 1 : 0u;
        if (any) pick &= pick - 1;
        beg[h] = readlane(mb, k);
        end[h] = any ? readlane(me, k) : beg[h];  // no VSS left: an empty one
        ss[h] = readlane(ms, k);
      }
      // B tiles: the frontier words of each set's sigma columns
      uint64_t bw[P];
#pragma unroll
      for (int h = 0; h < P; ++h) {
        const uint32_t col = ss[h] * SIG + lane;
        bw[h] = (lane < (uint32_t)SIG && col < p.n && end[h] > beg[h]) ? p.front[col] : 0ull;
      }
      MT m[P][SLOTS];
      uint32_t u[P][SLOTS];
#pragma unroll
      for (int h = 0; h < P; ++h)
#pragma unroll
        for (int r = 0; r < SLOTS; ++r) {
          const uint32_t idx = beg[h] + lane + r * kWave;
          const bool ok = idx < end[h];
          m[h][r] = ok ? masks[idx] : MT(0);
          u[h][r] = ok ? p.row_ids[idx] : 0u;
        }
      uint64_t acc[P][SLOTS];
      ulonglong2 cv[P][SLOTS];
#pragma unroll
      for (int h = 0; h < P; ++h) {
        uint64_t B[SIG];
#pragma unroll
        for (int j = 0; j < SIG; ++j) B[j] = readlane64(bw[h], j);
#pragma unroll
        for (int r = 0; r < SLOTS; ++r) {
          uint64_t a = 0;
#pragma unroll
          for (int j = 0; j < SIG; ++j) a |= ((uint32_t)m[h][r] >> j & 1u) ? B[j] : 0ull;
          acc[h][r] = a;
          cv[h][r] = reinterpret_cast<const ulonglong2*>(p.vis)[a ? u[h][r] : 0u];
        }
      }
#pragma unroll
      for (int h = 0; h < P; ++h)
#pragma unroll
        for (int r = 0; r < SLOTS; ++r) {
          const uint64_t fresh = acc[h][r] & ~cv[h][r].x & ~cv[h][r].y;
          if (fresh) {
            atomicOr(p.vis + 2 * (uint64_t)u[h][r] + 1, (unsigned long long)fresh);
            // Every level starts with next == current for all vertices, so the first
            // OR that changes u's next word was issued by a thread that read them
            // equal: only such threads need to mark u touched.
            if (mark && cv[h][r].y == cv[h][r].x) p.touched[u[h][r]] = 1;
          }
        }
    }
  }
}

// Stage 2, driven by one state byte per vertex: 1 = Stage 1 gave the vertex new
// bits this level (stored next to the OR), 2 = the vertex is on the current
// frontier.  Each thread reads the bytes of four consecutive vertices as one
// word; wavefronts whose words are all zero do nothing else.  A touched vertex
// loads its visited pair, writes its levels and frontier word and moves to state
// 2; a state-2 vertex that was not touched again gets a zero frontier word and
// state 0.  So the frontier words are exactly the per-level differences, as if
// every vertex were swept, while vertices in neither state cost one byte read.
// On high-diameter graphs (small frontiers, thousands of levels) this avoids
// touching every vertex's 24 bytes of visited and frontier words at every level.
// A slice set (sigma / 4 consecutive lanes) with a touched vertex queues its VSS
// range.  Levels flagged dense (a large queue, so most vertices change) skip the
// byte stores in Stage 1 and sweep every vertex here instead, rewriting all
// state bytes.
template <int SIG>
__device__ __forceinline__ void multi_stage2(const MultiParams& p, uint32_t* qn, uint32_t* qlen, int32_t level,
                                             bool dense) {
  constexpr uint32_t L = SIG / 4;  // lanes per slice set
  static_assert(L >= 2 && L <= kWave, "slice set must span whole lanes of one wavefront");
  __shared__ uint32_t s_wave[kMaxWaves];
  __shared__ uint32_t s_base;
  const uint32_t lane = lane_id();
  const uint32_t wave = threadIdx.x / kWave, nwaves = blockDim.x / kWave;
  const uint32_t nq = p.num_sets * L;
  uint32_t* tq = reinterpret_cast<uint32_t*>(p.touched);
  const ulonglong2* vis2 = reinterpret_cast<const ulonglong2*>(p.vis);
  for (uint32_t b0 = blockIdx.x * blockDim.x; b0 < nq; b0 += gridDim.x * blockDim.x) {
    const uint32_t q = b0 + threadIdx.x;
    // The wavefront's 64 words cover 256 consecutive vertices; in round r lane l
    // takes vertex r * 64 + l, so that level and frontier stores of a round are
    // contiguous across lanes.
    const uint32_t base = 4 * (q - lane);
    uint32_t hit;  // per word: nonzero iff one of its four vertices changed
    if (dense) {
      // full sweep: every vertex, state bytes rewritten (Stage 1 stored none).  The
      // four vertices' loads come first: a store to the visited pairs between them
      // would order each load after the previous vertex's round trip.
      ulonglong2 cv[4];
      uint32_t uo[4];
#pragma unroll
      for (uint32_t r = 0; r < 4; ++r) {
        const uint32_t u = base + r * kWave + lane;
        const uint32_t ui = u < p.n ? u : 0u;
        cv[r] = vis2[ui];
        uo[r] = morig(p, ui);
      }
      uint64_t m[4];
#pragma unroll
      for (uint32_t r = 0; r < 4; ++r) {
        const uint32_t u = base + r * kWave + lane;
        uint64_t diff = 0;
        if (u < p.n) {
          diff = cv[r].y & ~cv[r].x;
          p.front[u] = diff;
          p.touched[u] = diff ? 2 : 0;
          if (diff) {
            p.vis[2 * (uint64_t)u] = cv[r].y;
            uint64_t d = diff;
            while (d) {
              const uint32_t jj = __ffsll((unsigned long long)d) - 1;
              p.levels[(uint64_t)jj * p.n + uo[r]] = level;
              d &= d - 1;
            }
          }
        }
        m[r] = __ballot(diff != 0);
      }
      const uint32_t r = lane >> 4;
      const uint64_t mr = r == 0 ? m[0] : r == 1 ? m[1] : r == 2 ? m[2] : m[3];
      hit = (uint32_t)(mr >> ((4 * lane) & 63u)) & 0xFu;
    } else {
      const uint32_t tw = q < nq ? tq[q] : 0u;
      hit = tw & 0x01010101u;  // touched this level
      if (__ballot(tw != 0)) {
        // loads of the four vertices first (index 0 for an untouched one), then the
        // stores, so that the round trips overlap
        uint32_t bb[4], uo[4];
        ulonglong2 cv[4];
#pragma unroll
        for (uint32_t r = 0; r < 4; ++r) {
          const uint32_t w = (uint32_t)__shfl((int)tw, (int)(r * 16 + (lane >> 2)));
          bb[r] = (w >> (8 * (lane & 3u))) & 0xFFu;
          const uint32_t ui = (bb[r] & 1u) ? base + r * kWave + lane : 0u;
          cv[r] = vis2[ui];
          uo[r] = morig(p, ui);
        }
#pragma unroll
        for (uint32_t r = 0; r < 4; ++r) {
          const uint32_t u = base + r * kWave + lane;
          if (bb[r] == 2) p.front[u] = 0;  // left the frontier
          if (bb[r] & 1u) {
            const uint64_t diff = cv[r].y & ~cv[r].x;
            p.front[u] = diff;
            p.vis[2 * (uint64_t)u] = cv[r].y;
            uint64_t d = diff;
            while (d) {
              const uint32_t jj = __ffsll((unsigned long long)d) - 1;
              p.levels[(uint64_t)jj * p.n + uo[r]] = level;
              d &= d - 1;
            }
          }
        }
        if (tw) tq[q] = hit << 1;
      }
    }
    const uint64_t act = __ballot(hit != 0);
    uint32_t cnt = 0, vb[1] = {0}, vn[1] = {0};
    constexpr uint64_t kSetLanes = L == 64 ? ~0ull : ((1ull << L) - 1);
    if ((lane % L) == 0 && q < nq && ((act >> lane) & kSetLanes)) {
      const uint32_t ss = q / L;
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
    wave_push<1>(qn, pos, cnt, vb, vn, vb /* tags: unused */, MultiEntry{p.nranges > 1 ? p.vss_range : nullptr});
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
    p.touched[u] = b ? 2 : 0;  // the sources make up the level-0 frontier
  }
  for (uint32_t u = p.n + tid; u < p.num_sets * SIG; u += nt) p.touched[u] = 0;
  // initial queue: the VSS ranges of the sources' distinct slice sets
  {
    uint32_t off = 0;
    for (uint32_t i = 0; i < p.n_init_sets; ++i) {
      const uint32_t b = p.real_ptrs[p.init_sets[i]], e = p.real_ptrs[p.init_sets[i] + 1];
      for (uint32_t j = tid; j < e - b; j += nt)
        p.queue[off + j] = MultiEntry{p.nranges > 1 ? p.vss_range : nullptr}(b + j, 0u);
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
    // levels that queue many VSSs touch most vertices: there the per-vertex
    // state bytes cost more than sweeping every vertex
    const bool dense = (uint64_t)len * kDenseFrac >= p.num_vss;
    multi_stage1<MT, SLOTS>(p, qc, len, !dense);
    grid_barrier(ctrl);
    multi_stage2<SIG>(p, qn, qnext_len, level, dense);
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
  if (p.nranges == 0 || p.nranges > kMaxRanges || grid % p.nranges != 0) return hipErrorInvalidValue;
  MultiParams copy = p;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel(k, dim3(grid), dim3(block), args, 0, stream);
}

}  // namespace blest
