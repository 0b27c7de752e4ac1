// Device code of the fused, persistent single-source pull-BFS over Binarised
// Virtual Slice Sets (HIP, gfx950 / CDNA4).  Included by kernels.hip (launches,
// parents, scratch) and by kernels_eager.hip, kernels_lazy.hip and
// kernels_adaptive.hip, which instantiate the persistent kernel of one scheme each
// (so that the variants compile in parallel).
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
//   * Lazy scheme (Algorithm 3, Section 3.2): a hit on a row not visited when the
//     level started only marks the row, with a plain one-byte store into its
//     reached byte (the paper's non-returning atomic OR, made cheaper still: the
//     marks are idempotent, so no read-modify-write is needed); a coalesced sweep
//     over 32-vertex words then folds the reached bytes into the visited bits and
//     writes the levels, the next frontier and the next queue, with one queue
//     reservation per workgroup.  With row ranges, each workgroup checks hits
//     against its range's visited bits held in LDS.
//   * Eager scheme (Algorithm 2): a hit claims the vertex with a returning atomic
//     OR on the next frontier; the first claimer in a slice set's chunk pushes the
//     set's VSS range.  The visited bitmap (not the level array) filters hits.
//   * All levels run in one cooperative launch with a two-level (per-XCD group,
//     then root) grid barrier (Section 3.3).
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <mutex>
#include <type_traits>

#include "../../include/blest.h"
#include "device_common.hpp"
#include "kernels.hpp"

namespace blest {
namespace {

// Queue entry of VSS v (eager scheme): (v << kRangeBits) | row range.  With one
// range the table is not read (vss_range == nullptr), so pushes carry no load.
struct RangeEntry {
  const uint8_t* vss_range;
  __device__ uint32_t operator()(uint32_t v, uint32_t) const {
    return vss_range ? (v << kRangeBits) | vss_range[v] : v << kRangeBits;
  }
};
__device__ __forceinline__ RangeEntry range_entry(const BfsParams& p) {
  return RangeEntry{p.nranges > 1 ? p.vss_range : nullptr};
}

// Queue entry of VSS v (lazy scheme): x = (v << kRangeBits) | row range, y = the
// sigma-bit frontier chunk alpha of v's slice set.  Stage 2 knows a set's final
// chunk when it queues the set, so Stage 1 reads alpha from the entry instead of
// following VSS -> set -> frontier bitmap.
struct LazyEntry {
  const uint8_t* vss_range;
  __device__ uint2 operator()(uint32_t v, uint32_t alpha) const {
    return make_uint2(vss_range ? (v << kRangeBits) | vss_range[v] : v << kRangeBits, alpha);
  }
};
__device__ __forceinline__ LazyEntry lazy_entry(const BfsParams& p) {
  return LazyEntry{p.nranges > 1 ? p.vss_range : nullptr};
}

// Queue entry pushed by an eager level of the adaptive scheme: the 64-bit lazy
// layout with alpha = 0, because the set's chunk is only final when the level
// ends; the next level reads it from the claim bitmap instead.
struct EagerWideEntry {
  const uint8_t* vss_range;
  __device__ uint2 operator()(uint32_t v, uint32_t) const {
    return make_uint2(vss_range ? (v << kRangeBits) | vss_range[v] : v << kRangeBits, 0u);
  }
};

template <class QE>
__device__ __forceinline__ auto eager_entry(const BfsParams& p) {
  if constexpr (sizeof(QE) == 8) return EagerWideEntry{p.nranges > 1 ? p.vss_range : nullptr};
  else return RangeEntry{p.nranges > 1 ? p.vss_range : nullptr};
}

__device__ __forceinline__ uint32_t entry_vss(uint32_t e) { return e >> kRangeBits; }
__device__ __forceinline__ uint32_t entry_vss(uint2 e) { return e.x >> kRangeBits; }

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

// Mask type of the packed sigma = 8 layout (BfsParams::packed): each slice is one
// 32-bit word holding the row ID in its low 24 bits and the 8-bit mask in its
// high byte, so a slot is one 4-byte load instead of a 4-byte and a 1-byte load,
// and a slice takes 4 bytes instead of 5.
struct Packed8 {
  uint8_t v;
  __device__ operator uint32_t() const { return v; }
};

// Per-lane registers of G VSSs: SLOTS masks and row IDs each, plus alpha.
template <typename MT, int SLOTS, int G>
struct VssGroup {
  MT m[G][SLOTS];
  uint32_t u[G][SLOTS];
  uint32_t alpha[G];
};


// Raw buffer descriptor over `bytes` bytes at `base` (word 3: 32-bit data format,
// as gfx9 raw buffers use).  Buffer loads past `bytes` return zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, bytes, 0x00020000);
}

template <typename MT>
__device__ __forceinline__ MT buffer_load_mask(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  if constexpr (sizeof(MT) == 1) return __builtin_amdgcn_raw_buffer_load_b8(r, off, 0, 0);
  else if constexpr (sizeof(MT) == 2) return __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
  else return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}

// Loads the slots of a VSS whose slices are [beg, end) for every lane, through
// buffer descriptors that span exactly the VSS: lanes past the end read zero (an
// empty slice) with no clamp or select, the descriptor lives in scalar registers
// and the slot offset goes into the instruction, so a slot costs no vector ALU
// work.  The slices are streamed once per activation and are loaded
// non-temporally, so that they do not evict the reached bytes and bitmaps that
// the level keeps reusing.
template <typename MT, int SLOTS, int G>
__device__ __forceinline__ void load_vss(const BfsParams& p, uint32_t beg, uint32_t end, int k,
                                         VssGroup<MT, SLOTS, G>& g) {
  const uint32_t n = end - beg;
  const uint32_t lane = lane_id();
  constexpr int kSlc = 2;  // non-temporal (streaming) cache policy
  if constexpr (std::is_same<MT, Packed8>::value) {
    const __amdgpu_buffer_rsrc_t rs = buffer_of(p.packed + beg, n * 4u);
#pragma unroll
    for (int r = 0; r < SLOTS; ++r) {
      const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(rs, (lane + r * kWave) * 4u, 0, kSlc);
      g.u[k][r] = w & 0xFFFFFFu;
      g.m[k][r].v = (uint8_t)(w >> 24);
    }
  } else {
    const MT* masks = static_cast<const MT*>(p.masks);
    const __amdgpu_buffer_rsrc_t rr = buffer_of(p.row_ids + beg, n * 4u);
    const __amdgpu_buffer_rsrc_t rm = buffer_of(masks + beg, n * (uint32_t)sizeof(MT));
#pragma unroll
    for (int r = 0; r < SLOTS; ++r) {
      g.u[k][r] = __builtin_amdgcn_raw_buffer_load_b32(rr, (lane + r * kWave) * 4u, 0, kSlc);
      g.m[k][r] = buffer_load_mask<MT>(rm, (lane + r * kWave) * (uint32_t)sizeof(MT));
    }
  }
}

// Issues the mask and row-ID loads of the VSSs whose metadata sits in lanes
// k0 .. k0 + G - 1 of (mb, me, ma); lanes >= cnt are empty.
template <typename MT, int SLOTS, int G>
__device__ __forceinline__ void load_group(const BfsParams& p, uint32_t mb, uint32_t me, uint32_t ma, uint32_t k0,
                                           uint32_t cnt, VssGroup<MT, SLOTS, G>& g) {
#pragma unroll
  for (int k = 0; k < G; ++k) {
    const uint32_t src = k0 + k < cnt ? k0 + k : 63u;  // lane 63 holds an empty VSS when cnt < 64
    const uint32_t beg = readlane(mb, src), end = k0 + k < cnt ? readlane(me, src) : beg;
    g.alpha[k] = readlane(ma, src);
    load_vss<MT, SLOTS, G>(p, beg, end, k, g);
  }
}

// Stores 1 into row u's reached byte when a mark is due.  The store is masked
// per lane, not redirected: redirecting the lanes with no mark to padding lines
// (to keep the store unconditional) cost more in write traffic than it saved.
__device__ __forceinline__ void store_mark(__amdgpu_buffer_rsrc_t mark, bool need, uint32_t u) {
  if (need) __builtin_amdgcn_raw_buffer_store_b8((uint8_t)1, mark, u, 0, 0);
}
__device__ __forceinline__ __amdgpu_buffer_rsrc_t mark_buffer(const BfsParams& p) {
  return buffer_of(p.mark, 32u * p.n_words);
}

// Stage 1 driver shared by both schemes.  Wavefront w processes the queue
// positions w, w + nw, w + 2 nw, ... (round-robin over all wavefronts of the
// grid, Section 2.1.1).  Lane l first fetches the metadata of the wavefront's
// l-th next position - VSS slice range and the sigma-bit frontier chunk alpha of
// its slice set (from the lazy queue entry, or the eager frontier bitmap) - so
// the dependent queue -> metadata loads are paid once per 64 VSSs; the values are then broadcast with readlane.  VSSs are taken
// G at a time, with two groups in flight: while one group's own loads (issue,
// e.g. visited words) are waited for and applied (finish), the other group's
// slice loads are outstanding; the buffers swap roles rather than being copied,
// since a copy would wait for its loads.  Every step is free of branches around
// memory operations, so each wait covers only the loads it needs.
// `entry(pos, alpha)` returns the VSS at queue position pos and sets its alpha.
template <typename MT, int SLOTS, int G, class Entry, class Issue, class Finish>
__device__ __forceinline__ void stage1(const BfsParams& p, uint32_t len, Entry&& entry, Issue&& issue,
                                       Finish&& finish) {
  const uint32_t lane = lane_id();
  const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const uint32_t nw = (gridDim.x * blockDim.x) / kWave;
  for (uint32_t base = wid; base < len; base += nw * kWave) {
    const uint32_t pos = base + lane * nw;
    uint32_t mb = 0, me = 0, ma = 0;
    if (pos < len) {
      const uint32_t v = entry(pos, ma);
      mb = p.vss_beg[v];
      me = p.vss_beg[v + 1];
    }
    const uint32_t cnt = min((uint32_t)kWave, (len - base + nw - 1) / nw);
    VssGroup<MT, SLOTS, G> ga, gb;
    load_group<MT, SLOTS, G>(p, mb, me, ma, 0, cnt, ga);
    load_group<MT, SLOTS, G>(p, mb, me, ma, G, cnt, gb);  // empty past the end
    for (uint32_t k = 0; k < cnt; k += 2 * G) {
      finish(ga, issue(ga));
      load_group<MT, SLOTS, G>(p, mb, me, ma, k + 2 * G, cnt, ga);
      if (k + G >= cnt) break;
      finish(gb, issue(gb));
      load_group<MT, SLOTS, G>(p, mb, me, ma, k + 3 * G, cnt, gb);
    }
  }
}

// Stage 1 of the lazy scheme: mark every pulled row that was not visited when the
// level started.  The current-visited words of all hits of a group are loaded back
// to back; a mark is a plain one-byte store of 1 into the row's reached byte.  The
// stores are idempotent and all write the same value, so no read-modify-write is
// needed (device-scope atomic ORs cost an order of magnitude more on MI355X).
// fca: when the queue was pushed by an eager level (adaptive scheme), the claim
// bitmap of that level, from which alpha is read; nullptr = alpha in the entry.
template <typename MT, int SLOTS, int G>
__device__ __forceinline__ void stage1_lazy(const BfsParams& p, const uint2* qc, uint32_t len,
                                            const uint32_t* fca) {
  constexpr int SIG = 8 * sizeof(MT);
  using Words = struct { uint32_t w[G][SLOTS]; };
  const __amdgpu_buffer_rsrc_t mrk = mark_buffer(p);
  stage1<MT, SLOTS, G>(
      p, len,
      [&](uint32_t pos, uint32_t& alpha) {
        const uint2 e = qc[pos];
        const uint32_t v = e.x >> kRangeBits;
        alpha = fca ? frontier_chunk<SIG>(fca, p.v2r[v]) : e.y;
        return v;
      },
      [&](const VssGroup<MT, SLOTS, G>& g) {
        Words cw;
#pragma unroll
        for (int k = 0; k < G; ++k)
#pragma unroll
          for (int r = 0; r < SLOTS; ++r) {
            const bool hit = ((uint32_t)g.m[k][r] & g.alpha[k]) != 0;
            cw.w[k][r] = p.vis[hit ? (g.u[k][r] >> 5) : 0u];
          }
        return cw;
      },
      [&](const VssGroup<MT, SLOTS, G>& g, const Words& cw) {
#pragma unroll
        for (int k = 0; k < G; ++k)
#pragma unroll
          for (int r = 0; r < SLOTS; ++r) {
            const bool hit = ((uint32_t)g.m[k][r] & g.alpha[k]) != 0;
            const bool need = hit && !(cw.w[k][r] & (1u << (g.u[k][r] & 31)));
            store_mark(mrk, need, g.u[k][r]);
          }
      });
}

// Stage 1 of the lazy scheme with an LDS cache of visited bits.  Rows are split
// into nranges ranges; workgroup b serves range b % nranges and, at the start of
// every level with at least lds_min_len queue entries, copies into LDS the current
// visited words 0 .. C-1 (C = 2^lds_cshift) of every 64-word chunk of its range:
// word w of the range sits at LDS index (w / 64) * C + w % 64 when w % 64 < C.
// With one range the hub sort puts the rows that draw most hits into exactly
// those words.  Each wavefront of the range group looks at 64 queue positions at a time,
// strided by the group's wavefront count so that short queues still spread over
// the group, keeps the entries of its range, stages their metadata in lanes and
// processes them G at a time.  A cached row's check and its de-duplication are LDS
// operations (only the first mark of a vertex within a workgroup reaches global
// memory); any other pulled row is marked without a check, since Stage 2 drops
// reached rows that are already visited: a check in memory would make nearly
// every group of slices wait for a load when hot and cold rows are interleaved.
// A mark is a one-byte store into the row's reached byte.
template <typename MT, int SLOTS, int G>
__device__ __forceinline__ void stage1_lazy_lds(const BfsParams& p, const uint2* qc, uint32_t len, uint32_t* lds,
                                                const uint32_t* fca) {
  if (len < p.lds_min_len) {
    stage1_lazy<MT, SLOTS, G>(p, qc, len, fca);
    return;
  }
  constexpr int SIG = 8 * sizeof(MT);
  const uint32_t R = p.nranges;
  const uint32_t r = blockIdx.x % R;
  const uint32_t rw = p.range_len >> 5;  // words per range
  const uint32_t w0 = r * rw;
  const uint32_t cs = p.lds_cshift, cmask = (1u << cs) - 1u;
  {
    // eight independent loads per thread and step (a load-then-store loop would
    // wait for each load in turn); words past the range read zero
    const uint32_t have = w0 < p.n_words ? min(rw, p.n_words - w0) : 0u;
    const __amdgpu_buffer_rsrc_t vb = buffer_of(p.vis + w0, have * 4u);
    for (uint32_t b = threadIdx.x; b < p.range_words; b += 8 * blockDim.x) {
      uint32_t v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const uint32_t i = b + j * blockDim.x;
        v[j] = __builtin_amdgcn_raw_buffer_load_b32(vb, (((i >> cs) << 6) | (i & cmask)) * 4u, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (b + j * blockDim.x < p.range_words) lds[b + j * blockDim.x] = v[j];
    }
  }
  __syncthreads();
  const uint32_t lane = lane_id();
  const uint32_t W = blockDim.x / kWave;
  const uint32_t wg = (blockIdx.x / R) * W + threadIdx.x / kWave;
  const uint32_t nwg = (gridDim.x / R) * W;
  const uint32_t rbase = r * p.range_len;
  for (uint32_t base = wg; base < len; base += nwg * kWave) {
    const uint32_t pos = base + lane * nwg;
    const uint2 e = pos < len ? qc[pos] : make_uint2(0u, 0u);
    const bool mine = pos < len && (e.x & (kMaxRanges - 1)) == r;
    uint64_t pick = __ballot(mine);
    uint32_t mb = 0, me = 0, ma = 0;
    if (mine) {
      const uint32_t v = e.x >> kRangeBits;
      mb = p.vss_beg[v];
      me = p.vss_beg[v + 1];
      ma = fca ? frontier_chunk<SIG>(fca, p.v2r[v]) : e.y;
    }
    // G picked lanes at a time (uniform); missing ones read an empty VSS.  The
    // next group's slice loads are issued before the current group is applied.
    auto take = [&](uint32_t (&src)[G], VssGroup<MT, SLOTS, G>& g) {
#pragma unroll
      for (int k = 0; k < G; ++k) {
        src[k] = pick ? (uint32_t)(__ffsll((unsigned long long)pick) - 1) : 64u;
        pick &= pick - 1;
        const bool ok_k = src[k] < 64u;
        const uint32_t beg = ok_k ? readlane(mb, src[k] & 63u) : 0u;
        const uint32_t end = ok_k ? readlane(me, src[k] & 63u) : 0u;
        g.alpha[k] = ok_k ? readlane(ma, src[k] & 63u) : 0u;
        load_vss<MT, SLOTS, G>(p, beg, end, k, g);
      }
    };
    const __amdgpu_buffer_rsrc_t mrk = mark_buffer(p);
    // Three groups are kept in flight: while one is applied, the slice loads of
    // the next two are outstanding.  The buffers rotate roles instead of being
    // copied, since a copy would wait for its loads.
    auto apply = [&](const VssGroup<MT, SLOTS, G>& cur) {
      // cached hits: all LDS words first, then de-duplicating ORs where unvisited
      uint32_t lw[G][SLOTS];
      bool need[G][SLOTS];
#pragma unroll
      for (int k = 0; k < G; ++k)
#pragma unroll
        for (int q = 0; q < SLOTS; ++q) {
          const uint32_t wr = (cur.u[k][q] - rbase) >> 5;
          const bool hit = ((uint32_t)cur.m[k][q] & cur.alpha[k]) != 0;
          const bool in = hit && (wr & 63u) <= cmask;
          lw[k][q] = lds[in ? (((wr >> 6) << cs) | (wr & 63u)) : 0u];
          // an uncached row is marked without a visited check: Stage 2 keeps only
          // reached rows that are not yet visited, and a check in memory would
          // make nearly every group wait for a load
          need[k][q] = hit && (!in || !(lw[k][q] & (1u << (cur.u[k][q] & 31))));
        }
      // unvisited cached hits are rare on dense levels: one wavefront-wide test
      // skips the per-slot de-duplication when the group has none
      bool any_new = false;
#pragma unroll
      for (int k = 0; k < G; ++k)
#pragma unroll
        for (int q = 0; q < SLOTS; ++q) any_new |= need[k][q] && ((((cur.u[k][q] - rbase) >> 5) & 63u) <= cmask);
      if (__ballot(any_new)) {
#pragma unroll
        for (int k = 0; k < G; ++k)
#pragma unroll
          for (int q = 0; q < SLOTS; ++q) {
            const uint32_t wr = (cur.u[k][q] - rbase) >> 5;
            if (need[k][q] && (wr & 63u) <= cmask) {
              const uint32_t bit = 1u << (cur.u[k][q] & 31);
              const uint32_t old = atomicOr(&lds[((wr >> 6) << cs) | (wr & 63u)], bit);
              need[k][q] = !(old & bit);
            }
          }
      }
#pragma unroll
      for (int k = 0; k < G; ++k)
#pragma unroll
        for (int q = 0; q < SLOTS; ++q) store_mark(mrk, need[k][q], cur.u[k][q]);
    };
    uint32_t sa[G], sb[G], sc[G];
    VssGroup<MT, SLOTS, G> ga, gb, gc;
    take(sa, ga);
    take(sb, gb);
    take(sc, gc);
    while (sa[0] < 64u) {
      apply(ga);
      take(sa, ga);
      if (sb[0] >= 64u) break;
      apply(gb);
      take(sb, gb);
      if (sc[0] >= 64u) break;
      apply(gc);
      take(sc, gc);
    }
  }
}

// Stage 2 of the lazy scheme: coalesced sweep over 32-vertex words, one word per
// thread: the word's 32 reached bytes (a 32-byte load) against its visited bits.  Queue space is reserved once per workgroup (wavefront scans, then one
// atomic add by thread 0): a reservation per wavefront would put thousands of
// atomics on one counter per level.
template <int SIG>
__device__ __forceinline__ void stage2_lazy(const BfsParams& p, uint2* qn, uint32_t* qlen, int32_t level) {
  constexpr int SPW = 32 / SIG;  // slice sets per word
  __shared__ uint32_t s_wave[kMaxWaves];
  __shared__ uint32_t s_base;
  const uint32_t lane = lane_id();
  const uint32_t wave = threadIdx.x / kWave, nwaves = blockDim.x / kWave;
  // Wavefront-sized chunks of 64 words are dealt round-robin over the workgroups,
  // so that the low IDs, where the hub sort puts the sets with the most VSSs,
  // spread over many workgroups instead of loading the first few.
  for (uint32_t b0 = 0; b0 < p.n_words; b0 += gridDim.x * blockDim.x) {
    const uint32_t t = b0 + (wave * gridDim.x + blockIdx.x) * kWave + lane;
    uint32_t cnt = 0, vb[SPW], vn[SPW], va[SPW];
#pragma unroll
    for (int i = 0; i < SPW; ++i) vb[i] = vn[i] = va[i] = 0;
    if (t < p.n_words) {
      // the 32 reached bytes of word t, folded into one bit each
      const uint4* mb = reinterpret_cast<const uint4*>(p.mark + 32ull * t);
      const uint4 m0 = mb[0], m1 = mb[1];
      const uint32_t mw[8] = {m0.x, m0.y, m0.z, m0.w, m1.x, m1.y, m1.z, m1.w};
      uint32_t reached = 0;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const uint32_t x = mw[i];
#pragma unroll
        for (int b = 0; b < 4; ++b) reached |= ((x >> (8 * b)) & 0xFFu) ? (1u << (4 * i + b)) : 0u;
      }
      const uint32_t cur = p.vis[t];
      const uint32_t diff = reached & ~cur;
      if (diff) {
        p.vis[t] = cur | diff;
        // the VSS ranges of the sets with new vertices are loaded before the level
        // stores, so that their round trip overlaps that of the original IDs
#pragma unroll
        for (int i = 0; i < SPW; ++i) {
          va[i] = (diff >> (i * SIG)) & chunk_mask<SIG>();
          if (va[i]) {
            const uint32_t ss = t * SPW + i;
            vb[i] = p.real_ptrs[ss];
            vn[i] = p.real_ptrs[ss + 1] - vb[i];
          }
        }
        // levels of the new vertices: their original IDs are loaded 8 at a time
        // (two 16-byte loads) so that the stores do not wait one by one
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const uint32_t d8 = (diff >> (8 * c)) & 0xFFu;
          if (!d8) continue;
          uint32_t o[8];
          if (p.orig_id) {
            const uint4* op = reinterpret_cast<const uint4*>(p.orig_id + 32ull * t + 8 * c);
            const uint4 a = op[0], b = op[1];
            o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w; o[4] = b.x; o[5] = b.y; o[6] = b.z; o[7] = b.w;
          } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) o[j] = t * 32 + 8 * c + j;
          }
#pragma unroll
          for (int j = 0; j < 8; ++j)
            if (d8 & (1u << j)) p.levels[o[j]] = level;
        }
#pragma unroll
        for (int i = 0; i < SPW; ++i) cnt += vn[i];
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
      s_base = run ? atomicAdd(qlen, run) : 0u;
    }
    __syncthreads();
    const uint32_t pos = s_base + s_wave[wave] + incl - cnt;
    wave_push<SPW>(qn, pos, cnt, vb, vn, va, lazy_entry(p));
    __syncthreads();
  }
}

// Entries of a wavefront's list of VSS ranges to queue (eager scheme).
constexpr uint32_t kPushList = 64;

// Stage 1 of the eager scheme: a hit whose vertex is not yet visited claims it with
// a returning atomic OR on the next frontier; the claimer marks it visited, writes
// its level, and - if it is the first claimer in its slice set's chunk - queues the
// set's VSS range.  Ranges collect in per-wavefront lists in LDS and the workgroup
// reserves queue space once at the end: on high-diameter graphs, where a level has
// a few thousand claims, a reservation per wavefront put thousands of returning
// atomics on one counter, serialised, into every level.
// QE is the queue entry: uint32_t (eager scheme: VSS and range) or uint2 (adaptive
// scheme: the lazy layout).  fc = the claim bitmap of the previous level, from
// which alpha is read; nullptr (uint2 entries only) = alpha in the entry.
template <typename MT, int SLOTS, int G, class QE>
__device__ __forceinline__ void stage1_eager(const BfsParams& p, const QE* qc, uint32_t len,
                                             const uint32_t* fc, uint32_t* fn, QE* qn, uint32_t* qlen,
                                             int32_t level) {
  constexpr int SIG = 8 * sizeof(MT);
  struct Pre {
    uint32_t w[G][SLOTS], o[G][SLOTS], rb[G][SLOTS], re[G][SLOTS];
  };
  // per-wavefront lists of VSS ranges to queue (first VSS, count)
  __shared__ uint32_t s_pb[kMaxWaves][kPushList], s_pn[kMaxWaves][kPushList];
  __shared__ uint32_t s_cnt[kMaxWaves], s_tot[kMaxWaves];
  __shared__ uint32_t s_qbase;
  const uint32_t lane = lane_id();
  const uint32_t wave = threadIdx.x / kWave, nwaves = blockDim.x / kWave;
  if (lane == 0) s_cnt[wave] = 0;
  // queues this wavefront's list with one reservation and empties it
  auto flush_list = [&]() {
    __builtin_amdgcn_wave_barrier();
    const uint32_t c = s_cnt[wave];
    uint32_t b[1] = {0}, n[1] = {0};
    if (lane < c) {
      b[0] = s_pb[wave][lane];
      n[0] = s_pn[wave][lane];
    }
    uint32_t total;
    const uint32_t pos = wave_reserve(qlen, n[0], total);
    wave_push<1>(qn, pos, n[0], b, n, b /* tags: unused */, eager_entry<QE>(p));
    if (lane == 0) s_cnt[wave] = 0;
  };
  // queues every wavefront's list with one reservation for the workgroup
  auto flush_block = [&]() {
    __builtin_amdgcn_wave_barrier();
    const uint32_t c = s_cnt[wave];
    uint32_t b[1] = {0}, n[1] = {0};
    if (lane < c) {
      b[0] = s_pb[wave][lane];
      n[0] = s_pn[wave][lane];
    }
    const uint32_t incl = wave_inclusive_scan(n[0]);
    if (lane == kWave - 1) s_tot[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t run = 0;
      for (uint32_t w = 0; w < nwaves; ++w) {
        const uint32_t x = s_tot[w];
        s_tot[w] = run;
        run += x;
      }
      s_qbase = run ? atomicAdd(qlen, run) : 0u;
    }
    __syncthreads();
    wave_push<1>(qn, s_qbase + s_tot[wave] + incl - n[0], n[0], b, n, b /* tags: unused */, eager_entry<QE>(p));
  };
  // Besides the visited words, a hit's original ID and its set's VSS range are
  // loaded up front, in parallel, so that neither the level store nor the push
  // waits for a further load after the claim (high-diameter graphs are bound by
  // this chain's length, one level after another).
  auto issue = [&](const VssGroup<MT, SLOTS, G>& g) {
    Pre pre;
#pragma unroll
    for (int k = 0; k < G; ++k)
#pragma unroll
      for (int r = 0; r < SLOTS; ++r) {
        const bool hit = ((uint32_t)g.m[k][r] & g.alpha[k]) != 0;
        const uint32_t x = hit ? g.u[k][r] : 0u;
        pre.w[k][r] = p.vis[x >> 5];
        pre.o[k][r] = to_orig(p, x);
        pre.rb[k][r] = p.real_ptrs[x / SIG];
        pre.re[k][r] = p.real_ptrs[x / SIG + 1];
      }
    return pre;
  };
  auto entry = [&](uint32_t pos, uint32_t& alpha) {
    const QE e = qc[pos];
    const uint32_t v = entry_vss(e);
    if constexpr (sizeof(QE) == 8) alpha = fc ? frontier_chunk<SIG>(fc, p.v2r[v]) : e.y;
    else alpha = frontier_chunk<SIG>(fc, p.v2r[v]);
    return v;
  };
  stage1<MT, SLOTS, G>(p, len, entry, issue, [&](const VssGroup<MT, SLOTS, G>& g, const Pre& pre) {
    const auto& vw = pre.w;
    uint32_t cnt = 0, vb[G * SLOTS], vn[G * SLOTS];
#pragma unroll
    for (int i = 0; i < G * SLOTS; ++i) vb[i] = vn[i] = 0;
#pragma unroll
    for (int k = 0; k < G; ++k)
#pragma unroll
      for (int r = 0; r < SLOTS; ++r) {
        const uint32_t x = g.u[k][r];
        const uint32_t bit = 1u << (x & 31);
        const bool hit = ((uint32_t)g.m[k][r] & g.alpha[k]) != 0;
        if (hit && !(vw[k][r] & bit)) {
          const uint32_t old = atomicOr(fn + (x >> 5), bit);
          if (!(old & bit)) {
            atomicOr(p.vis + (x >> 5), bit);
            p.levels[pre.o[k][r]] = level;
            const uint32_t sh = (x & 31) & ~(uint32_t)(SIG - 1);
            if (((old >> sh) & chunk_mask<SIG>()) == 0) {
              vb[k * SLOTS + r] = pre.rb[k][r];
              vn[k * SLOTS + r] = pre.re[k][r] - pre.rb[k][r];
              cnt += vn[k * SLOTS + r];
            }
          }
        }
      }
    // Queue the new sets' VSS ranges: appended to this wavefront's list in LDS
    // and reserved once per workgroup after the loop; a group with more ranges
    // than the list holds, or a full list, takes a wavefront reservation now.
    uint32_t nr = 0;
#pragma unroll
    for (int i = 0; i < G * SLOTS; ++i) nr += vn[i] != 0;
    const uint32_t rincl = wave_inclusive_scan(nr);
    const uint32_t rtot = __shfl(rincl, kWave - 1, kWave);
    if (rtot == 0) return;
    uint32_t used = s_cnt[wave];
    if (used + rtot > kPushList) {
      flush_list();
      used = 0;
    }
    if (rtot > kPushList) {
      uint32_t total;
      const uint32_t pos = wave_reserve(qlen, cnt, total);
      wave_push<G * SLOTS>(qn, pos, cnt, vb, vn, vb /* tags: unused */, eager_entry<QE>(p));
      return;
    }
    uint32_t at = used + rincl - nr;
#pragma unroll
    for (int i = 0; i < G * SLOTS; ++i)
      if (vn[i]) {
        s_pb[wave][at] = vb[i];
        s_pn[wave][at] = vn[i];
        ++at;
      }
    if (lane == 0) s_cnt[wave] = used + rtot;
  });
  flush_block();
}

// Clears the frontier chunks of the sets named by queue qold (eager scheme).
template <int SIG, class QE>
__device__ __forceinline__ void clear_chunks(const BfsParams& p, uint32_t* f, const QE* qold, uint32_t len) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t nt = gridDim.x * blockDim.x;
  // the highest-numbered threads take the clears: on the small levels of
  // high-diameter graphs they have no Stage 1 work, so the clears' dependent loads
  // stay off the Stage 1 chain of the low-numbered wavefronts
  for (uint32_t i = nt - 1 - tid; i < len; i += nt) {
    const uint32_t ss = p.v2r[entry_vss(qold[i])];
    if (SIG == 8) reinterpret_cast<uint8_t*>(f)[ss] = 0;
    else if (SIG == 16) reinterpret_cast<uint16_t*>(f)[ss] = 0;
    else f[ss] = 0;
  }
}

// MODE: kEager (Algorithm 2 every level), kLazy (Algorithm 3 every level) or
// kAdaptive: each level picks, on the device, from the length of its queue (the
// same value in every workgroup): levels with fewer than p.eager_max queued VSSs
// claim eagerly with one grid barrier and no vertex sweep; larger ones mark lazily
// and sweep (two barriers).  State shared across the switch: the visited bitmap
// (both schemes keep it exact), the reached bytes (zero for unvisited vertices;
// the lazy sweep masks visited ones), three claim bitmaps (an eager level's claims
// give the next level its alpha; they are cleared sparsely two levels later) and
// three queues of 64-bit lazy-layout entries.
constexpr int kEager = 0, kLazy = 1, kAdaptive = 2;

template <typename MT, int SLOTS, int MODE, int G, bool LDSVIS>
__global__ __launch_bounds__(1024) void bfs_persistent(BfsParams p) {
  extern __shared__ uint32_t lds_vis[];
  constexpr int SIG = 8 * sizeof(MT);
  constexpr bool MARKS = MODE != kEager;  // reached bytes in use
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
  for (uint32_t t = tid; t < p.n_words; t += nt) {
    const uint32_t b = (t == sw) ? sbit : 0u;
    p.vis[t] = b;
    if (MARKS) {
      // the word's 32 reached bytes: zero, except the source's
      uint32_t z[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (t == sw) z[(p.src & 31) >> 2] = 1u << (8 * (p.src & 3));
      uint4* mb = reinterpret_cast<uint4*>(p.mark + 32ull * t);
      mb[0] = make_uint4(z[0], z[1], z[2], z[3]);
      mb[1] = make_uint4(z[4], z[5], z[6], z[7]);
    }
    if (MODE != kLazy) {
      // eager: the source is the level-0 claim; adaptive: alpha of level 1 is in
      // the entries, and every claim bitmap starts empty
      p.front[t] = MODE == kEager ? b : 0u;
      p.front[p.n_words + t] = 0;
      p.front[2 * p.n_words + t] = 0;
    }
  }
  if (MODE == kEager) {
    for (uint32_t j = tid; j < q0n; j += nt) p.queue[j] = range_entry(p)(q0b + j, 0u);
  } else {
    const uint32_t a0 = 1u << (p.src % SIG);  // the source's bit in its set's frontier chunk
    for (uint32_t j = tid; j < q0n; j += nt) reinterpret_cast<uint2*>(p.queue)[j] = lazy_entry(p)(q0b + j, a0);
  }
  if (tid == 0) {
    qlen[0] = q0n;
    qlen[kLine] = 0;
    qlen[2 * kLine] = 0;
    qlen[3 * kLine] = 0;
  }
  grid_barrier(ctrl);

  bool prev_eager = false, prev2_eager = false;  // modes of levels l - 1 and l - 2 (adaptive)
  // The queue lengths of this level and of the one before, carried from the check
  // that ends each level (a fresh load would cost another round trip per level;
  // the slots do not change in between).  The initial queue is q0n long; the
  // queue before it is empty.
  uint32_t len = q0n, prev_len = 0;
  for (int32_t level = 1; level <= (int32_t)p.n + 1; ++level) {
    if (MODE == kLazy) {
      const uint2* qc = reinterpret_cast<const uint2*>(p.queue) + ((level - 1) & 1) * p.qcap;
      uint2* qn = reinterpret_cast<uint2*>(p.queue) + (level & 1) * p.qcap;
      uint32_t* qnext_len = qlen + (level % 3) * kLine;
      if (tid == 0) __hip_atomic_store(qlen + ((level + 1) % 3) * kLine, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (LDSVIS)
        stage1_lazy_lds<MT, SLOTS, G>(p, qc, len, lds_vis, nullptr);
      else
        stage1_lazy<MT, SLOTS, G>(p, qc, len, nullptr);
      grid_barrier(ctrl);
      stage2_lazy<SIG>(p, qn, qnext_len, level);
      grid_barrier(ctrl);
      prev_len = len;
      len = ld_relaxed(qnext_len);
      if (len == 0) break;
    } else if (MODE == kEager) {
      const uint32_t* qc = p.queue + ((level - 1) % 3) * p.qcap;
      uint32_t* qn = p.queue + (level % 3) * p.qcap;
      const uint32_t* qold = p.queue + ((level + 1) % 3) * p.qcap;  // queue of level - 2
      const uint32_t old_len = prev_len;
      uint32_t* qnext_len = qlen + (level % 4) * kLine;
      if (tid == 0) __hip_atomic_store(qlen + ((level + 1) % 4) * kLine, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint32_t* fc = p.front + ((level - 1) % 3) * p.n_words;
      uint32_t* fn = p.front + (level % 3) * p.n_words;
      uint32_t* fold = p.front + ((level + 1) % 3) * p.n_words;
      clear_chunks<SIG>(p, fold, qold, old_len);
      stage1_eager<MT, SLOTS, G>(p, qc, len, fc, fn, qn, qnext_len, level);
      grid_barrier(ctrl);
      prev_len = len;
      len = ld_relaxed(qnext_len);
      if (len == 0) break;
    } else {
      uint2* q2 = reinterpret_cast<uint2*>(p.queue);
      const uint2* qc = q2 + ((level - 1) % 3) * p.qcap;
      uint2* qn = q2 + (level % 3) * p.qcap;
      uint32_t* qnext_len = qlen + (level % 4) * kLine;
      if (tid == 0) __hip_atomic_store(qlen + ((level + 1) % 4) * kLine, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint32_t* fc = prev_eager ? p.front + ((level - 1) % 3) * p.n_words : nullptr;
      if (prev2_eager) {
        // the claims of level - 2 (sets of the queue it pushed) leave their bitmap
        const uint2* qold = q2 + ((level + 1) % 3) * p.qcap;
        clear_chunks<SIG>(p, p.front + ((level + 1) % 3) * p.n_words, qold, prev_len);
      }
      const bool eager = len < p.eager_max;
      if (eager) {
        stage1_eager<MT, SLOTS, G>(p, qc, len, fc, p.front + (level % 3) * p.n_words, qn, qnext_len, level);
        grid_barrier(ctrl);
      } else {
        if (LDSVIS)
          stage1_lazy_lds<MT, SLOTS, G>(p, qc, len, lds_vis, fc);
        else
          stage1_lazy<MT, SLOTS, G>(p, qc, len, fc);
        grid_barrier(ctrl);
        stage2_lazy<SIG>(p, qn, qnext_len, level);
        grid_barrier(ctrl);
      }
      prev_len = len;
      len = ld_relaxed(qnext_len);
      if (len == 0) break;
      prev2_eager = prev_eager;
      prev_eager = eager;
    }
  }
}

}  // namespace

// Kernel symbol of one scheme's persistent variant (kernels_eager.hip,
// kernels_lazy.hip, kernels_adaptive.hip); nullptr for combinations not built.
const void* bfs_symbol_eager(uint32_t sigma, uint32_t slots, uint32_t group, bool packed);
const void* bfs_symbol_lazy(uint32_t sigma, uint32_t slots, uint32_t group, bool lds, bool packed);
const void* bfs_symbol_adaptive(uint32_t sigma, uint32_t slots, uint32_t group, bool lds, bool packed);

}  // namespace blest
